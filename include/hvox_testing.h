/*
 * hvox_testing.h -- kernel-level test entry points of libhvox.so.
 *
 * Not needed to use the library: these run one internal kernel on caller
 * buffers so that tests can check it in isolation.
 */
#ifndef HVOX_TESTING_H
#define HVOX_TESTING_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * One pass of the library's LDS-resident mixed-radix FFT (the kernel of the
 * type-3 transform's FFT step, HVOX Sect. 3) on `nlines` lines:
 *   out[j][q] = sum_{e < nin} in[j][e] exp(sign 2 pi i (e - nin/2) m_q / n),
 *   m_q = (wstart + q) mod n,  q < wcount,
 * i.e. modes -nin/2 .. nin/2-1 zero-padded to an n-point FFT, of which the
 * window of wcount outputs starting at index wstart (may be negative) is
 * kept, written line by line.  n must be even, 2-3-5 smooth and <= 4096,
 * nin even and <= n, wcount <= n, sign = -1 or +1.
 * dtype HVOX_F32 (complex64) or HVOX_F64 (complex128); in and out are device
 * buffers of nlines*nin and nlines*wcount complex values.  Work is enqueued
 * on stream; the call returns after synchronising it.
 */
int hvox_test_fft(int32_t dtype, int32_t n, int32_t nin, int32_t nlines, int32_t wstart, int32_t wcount,
                  int32_t sign, const void *in, void *out, void *stream);

/*
 * The radix plan of the FFT passes for lines of n points (the stages of the
 * FFT step of HVOX Sect. 3): writes the radix of every Stockham stage, first
 * stage first, to radix[0 .. k-1] and returns k (at most 16), or a negative
 * HVOX error code when n is odd, not 2-3-5 smooth or beyond 4096.  radix is a
 * host buffer of at least 16 bytes owned by the caller.  Host code only: no
 * GPU is needed.
 */
int hvox_test_fft_radices(int32_t n, uint8_t *radix);

#ifdef __cplusplus
}
#endif
#endif /* HVOX_TESTING_H */
