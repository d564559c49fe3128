// HIP kernels of the HVOX library for gfx950 (MI355X): the hot path of the
// chunked 3D type-3 NUFFT (HVOX Sect. 3 and 3.1) and of its block-level
// direct evaluation.
//
// Data layout in HBM
//  * coordinates: float64 structure-of-arrays [3][n] in chunk order;
//  * user data:   complex (float2 / double2) in user order, gathered through
//                 the chunk-order permutation (Sect. 4, chunk-order views), or
//                 already in chunk order (pre-ordered plans);
//  * occupancy:   one bit per grid-1 tile (32 x 8 x 8 cells), set when the
//                 tile holds sources; spreading writes only those tiles and
//                 the x pass reads the others as zeros;
//  * grids:       per batch of sub-problems and per data row of a pass one
//                 workspace copy with three regions:
//                 G holds every pair's grid 1 as [n1z][n1y][n1x]; the x pass
//                 writes its kept window line-major to B ([n1z][n1y][wx]), a
//                 tiled transpose moves it to A ([n1z][wx][n1y]), the y pass
//                 writes B ([n1z][wx][wy]), and the z pass reads its lines
//                 strided and writes A as [wx][wy][wz] (z fastest), which the
//                 interpolation reads;
//  * accumulator: float64 complex per target (chunk order).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "hvox_internal.hpp"

namespace hvox {

template <typename T> struct C2;
template <> struct C2<float> { using type = float2; };
template <> struct C2<double> { using type = double2; };
template <typename T> using cplx = typename C2<T>::type;

template <typename T> __device__ __forceinline__ cplx<T> mk(T a, T b) { cplx<T> r; r.x = a; r.y = b; return r; }
template <typename T> __device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b)
{
    return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T> __device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
// multiply by s*i (s = +1 or -1)
template <typename T> __device__ __forceinline__ cplx<T> cmuli(cplx<T> a, T s) { return mk<T>(-s * a.y, s * a.x); }

// exponential of semicircle ES(z) = exp(beta (sqrt(1 - z^2) - 1)), |z| < 1
__device__ __forceinline__ float es_kernel(float z, float beta)
{
    // hardware square root and base-2 exponential (about 1 ulp each): far
    // below the kernel's own truncation error at any float32 tolerance
    float q = 1.0f - z * z;
    return q > 0.0f ? __builtin_amdgcn_exp2f(beta * 1.44269504088896341f * (__builtin_amdgcn_sqrtf(q) - 1.0f)) : 0.0f;
}
__device__ __forceinline__ double es_kernel(double z, double beta)
{
    double q = 1.0 - z * z;
    return q > 0.0 ? exp(beta * (sqrt(q) - 1.0)) : 0.0;
}

// exp(2 pi i s f) for a phase f in cycles, evaluated in float64 after
// reduction to [-1/2, 1/2]
__device__ __forceinline__ double2 cis_cycles(double f, double s)
{
    double r = f - rint(f);
    double sn, cs;
    sincospi(2.0 * r, &sn, &cs);
    return make_double2(cs, s * sn);
}

__device__ __forceinline__ int64_t find_segment(const int64_t *__restrict__ prefix, int n, int64_t g)
{
    int lo = 0, hi = n - 1;          // largest p with prefix[p] <= g
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// floor(a / d) for 0 <= a < 2^21, given rd = 1/d as a float.  (a + 1/2) / d
// is at least 1/(2d) away from every integer while the float product is off
// by at most (a + 1/2) / d * 2^-22 < 1/(2d), so truncation gives the exact
// quotient: a few full-rate instructions instead of a 32-bit integer division.
__device__ __forceinline__ int small_div(int a, float rd)
{
    return static_cast<int>((static_cast<float>(a) + 0.5f) * rd);
}
static_assert(kFftElems < (1 << 21), "FFT workgroup indices must stay below 2^21 for small_div");

// 1/d for small_div from the hardware reciprocal (within 1 ulp: the product
// in small_div then stays inside the 2^-22 budget above)
__device__ __forceinline__ float small_rcp(int d) { return __builtin_amdgcn_rcpf(static_cast<float>(d)); }
static_assert(int64_t(kFftMaxLen / kTileX) * (kFftMaxLen / kTileY) * (kFftMaxLen / kTileZ) < (int64_t(1) << 31),
              "grid-1 tiles of a sub-problem must fit 31 bits");

// ---------------------------------------------------------------------------
// accumulator clear
// ---------------------------------------------------------------------------
__global__ void k_zero(double *__restrict__ p, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0.0;
}

// ---------------------------------------------------------------------------
// deconvolution factors 1 / prod_d Psi_hat(nu_d) of every target, where
// nu_d = (s_d - s_c,d) h_d and Psi_hat(nu) = (w/2) int_{-1}^{1} ES(z) cos(pi nu w z) dz
// (Gauss-Legendre; aq = weight * ES(node)).
// ---------------------------------------------------------------------------
__global__ void k_deconv(const double *__restrict__ xyz, int64_t n, const int32_t *__restrict__ chunk_of,
                         const double *__restrict__ ctr, const double *__restrict__ hscale,
                         const double *__restrict__ zq, const double *__restrict__ aq, int nq, int w,
                         double *__restrict__ out)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int32_t c = chunk_of[k];
    double prod = 1.0;
    for (int d = 0; d < 3; ++d) {
        double nu = (xyz[d * n + k] - ctr[3 * c + d]) * hscale[3 * c + d];
        double s = 0.0;
        for (int q = 0; q < nq; ++q) s += aq[q] * cospi(nu * w * zq[q]);
        prod *= 0.5 * w * s;
    }
    out[k] = 1.0 / prod;
}

// ---------------------------------------------------------------------------
// spreading (type-3 step 1, Sect. 3):
//   b_l = sum_n c'_n prod_d ES((l_d - t_nd) 2/w),  c'_n = c_n exp(2 pi i iota s_c.x'_n),
// with t_n = (x_n - x_c) * kscale (grid-1 units) and l in [-n1/2, n1/2)^3.
// ---------------------------------------------------------------------------

// grid-1 footprint of a source: first cell (local index l + n1/2) and the
// float64 grid coordinate; shared by the binning and the spreading kernels so
// that both see exactly the same cells.
__device__ __forceinline__ void source_footprint(const PairDev &P, const double *__restrict__ xyz, int64_t nsrc,
                                                 int64_t n, int w, double xp[3], double t[3], int c0[3])
{
    for (int d = 0; d < 3; ++d) {
        xp[d] = xyz[d * nsrc + n] - P.xc[d];
        t[d] = xp[d] * P.kscale[d];
        c0[d] = (int)ceil(t[d] - 0.5 * w) + P.n1[d] / 2;
    }
}

// Plan-time binning: every (sub-problem, source) pair is listed under each
// grid-1 tile its w^3 footprint touches.  Pass 1 (cursor == nullptr)
// counts, pass 2 scatters the pair's index in the batch's staging order to
// the offsets the host computed.
__global__ void k_bin_points(const PairDev *__restrict__ pairs, const int64_t *__restrict__ prefix, int npairs,
                             int64_t total, const double *__restrict__ xyz, int64_t nsrc, int w,
                             int32_t *__restrict__ counts, unsigned long long *__restrict__ cursor,
                             int32_t *__restrict__ records)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    const int p = (int)find_segment(prefix, npairs, g);
    const PairDev &P = pairs[p];
    const int64_t n = P.src_off + (g - prefix[p]);
    double xp[3], t[3];
    int c0[3];
    source_footprint(P, xyz, nsrc, n, w, xp, t, c0);
    const int tdim[3] = {kTileX, kTileY, kTileZ};
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = max(0, c0[d]) / tdim[d];
        hi[d] = min(P.n1[d] - 1, c0[d] + w - 1);
        hi[d] = hi[d] < 0 ? -1 : hi[d] / tdim[d];
        hi[d] = min(hi[d], P.ntile[d] - 1);
    }
    for (int tz = lo[2]; tz <= hi[2]; ++tz)
        for (int ty = lo[1]; ty <= hi[1]; ++ty)
            for (int tx = lo[0]; tx <= hi[0]; ++tx) {
                const int64_t tile = P.tile0 + ((int64_t)tz * P.ntile[1] + ty) * P.ntile[0] + tx;
                if (cursor == nullptr) {
                    atomicAdd(counts + tile, 1);
                } else {
                    const unsigned long long pos = atomicAdd(cursor + tile, 1ull);
                    records[pos] = (int32_t)g;   // batches hold fewer than 2^31 sources
                }
            }
}

// Gather + pre-phase of a batch's sources (type-3 centring, the source side):
// c'_n = c_perm(n) exp(2 pi i iota s_c.(x_n - x_c)) for every source of every
// sub-problem of the batch, in the batch's order (sub-problem, then chunk
// order), staged with its kernel footprint on grid 1 for the spreading pass
// (computed once per source instead of once per tile it touches).  The phase
// and the footprint are float64.  With several data rows in the pass (the
// ntrans rows of Sect. 4), the footprint and phase factor are computed once
// and the further rows' values go to xval, row-major with stride xstride.
template <typename T>
__global__ void k_prephase(const PairDev *__restrict__ pairs, const int64_t *__restrict__ pprefix, int npairs,
                           int64_t total, const double *__restrict__ xyz, int64_t nsrc,
                           const int32_t *__restrict__ perm, const cplx<T> *__restrict__ in, int64_t in_stride,
                           int nr, StagedSrc<T> *__restrict__ stage, cplx<T> *__restrict__ xval, int64_t xstride,
                           double iota, int w)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    const int p = (int)find_segment(pprefix, npairs, g);
    const PairDev &P = pairs[p];
    const int64_t n = P.src_off + (g - pprefix[p]);
    double xp[3], t[3];
    int c0[3];
    source_footprint(P, xyz, nsrc, n, w, xp, t, c0);
    double ph = 0.0;
    for (int d = 0; d < 3; ++d) ph += P.sc[d] * xp[d];
    const double2 e = cis_cycles(ph, iota);
    const int64_t u = perm ? perm[n] : n;   // no permutation: data already in chunk order
    const cplx<T> c = in[u];
    StagedSrc<T> s;
    s.v[0] = T(c.x * e.x - c.y * e.y);
    s.v[1] = T(c.x * e.y + c.y * e.x);
    for (int d = 0; d < 3; ++d) {
        s.frac[d] = T((double)(c0[d] - P.n1[d] / 2) - t[d]);
        s.c0[d] = c0[d];
    }
    stage[g] = s;
    // further data rows of the pass: the same phase factor, values only
    for (int r = 1; r < nr; ++r) {
        const cplx<T> cr = in[r * in_stride + u];
        xval[(r - 1) * xstride + g] = mk<T>(T(cr.x * e.x - cr.y * e.y), T(cr.x * e.y + cr.y * e.x));
    }
}

// eight consecutive LDS values (16-byte aligned) as wide reads
__device__ __forceinline__ void load8(const float *p, float v[8])
{
    const float4 a = reinterpret_cast<const float4 *>(p)[0], b = reinterpret_cast<const float4 *>(p)[1];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}
__device__ __forceinline__ void load8(const double *p, double v[8])
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double2 a = reinterpret_cast<const double2 *>(p)[i];
        v[2 * i] = a.x;
        v[2 * i + 1] = a.y;
    }
}

// Spreading by grid-1 tile: one workgroup per tile.  Thread (x, y) of the
// 32 x 8 face owns the kTileZ cells of its column (a wavefront per 8 x 8 patch
// of the face); the tile's sources are staged kSpreadBatch at a time in LDS
// (pre-phased value, footprint origin relative to the tile, the 2w x and y
// kernel values in the source's frame and the kTileZ z values in the tile's
// frame, zero outside the footprint), every thread adds the contributions that
// fall in its column with two wide LDS reads and 2 kTileZ FMAs per source, and
// the whole tile is written once (no atomics; for a given plan the result is
// deterministic).  A crowded tile (more than kSpreadSplit sources) is split
// into parts, one workgroup each: the first stores like any tile, the others
// (a second launch) add their sums atomically on top (float atomics: the
// rounding order of those cells varies from run to run).  The tile's sub-problem, corner and source list come from
// one plan-time descriptor (the binning), each source's value and footprint
// from the pre-phase pass.  NR data rows share one evaluation of the kernel
// weights (row r's grid is the r-th copy of the batch workspace, ws_stride
// complex elements apart).
template <typename T, int NR>
__global__ __launch_bounds__(256) void k_spread(const PairDev *__restrict__ pairs,
                                                const SpreadTile *__restrict__ tiles,
                                                const int32_t *__restrict__ records,
                                                const StagedSrc<T> *__restrict__ staged,
                                                const cplx<T> *__restrict__ xval, int64_t xstride,
                                                cplx<T> *__restrict__ ws, int64_t ws_stride, int w, T beta,
                                                T two_over_w, float rwk)
{
    static_assert(kTileZ == 8, "the z weights of a source are read as 8 values");
    // per staged source: kTileZ z values in the tile's frame, then w x and w y
    // values in the source's frame (rows a multiple of 16 bytes)
    constexpr int kKv = kTileZ + 2 * kWMax;
    static_assert(kKv % 4 == 0, "16-byte rows");
    __shared__ __align__(16) T kv[kSpreadBatch][kKv];
    __shared__ T frac[kSpreadBatch][3];
    __shared__ cplx<T> val[NR][kSpreadBatch];
    __shared__ int org[kSpreadBatch][3];
    const int tid = threadIdx.x;
    const SpreadTile tile = tiles[blockIdx.x];
    const int ox = tile.org[0], oy = tile.org[1], oz = tile.org[2];
    // each wavefront owns an 8 x 8 patch of columns (x fastest): a w-wide
    // footprint meets one or two of the four wavefronts instead of all of them
    static_assert(kTileX == 32 && kTileY == 8, "8 x 8 column patches per wavefront");
    const int x = (tid & 7) + 8 * (tid >> 6), y = (tid >> 3) & 7;
    const int wk = 2 * w + kTileZ;   // kernel values per staged source
    T accr[NR][kTileZ], acci[NR][kTileZ];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int z = 0; z < kTileZ; ++z) accr[r][z] = acci[r][z] = T(0);

    for (int base = 0; base < tile.cnt; base += kSpreadBatch) {
        const int cnt = min(kSpreadBatch, tile.cnt - base);
        __syncthreads();
        if (tid < cnt) {
            const int32_t rec = records[tile.r0 + base + tid];
            const StagedSrc<T> sc = staged[rec];
            for (int d = 0; d < 3; ++d) frac[tid][d] = sc.frac[d];
            org[tid][0] = sc.c0[0] - ox;
            org[tid][1] = sc.c0[1] - oy;
            org[tid][2] = sc.c0[2] - oz;
            val[0][tid] = mk<T>(sc.v[0], sc.v[1]);
#pragma unroll
            for (int r = 1; r < NR; ++r) val[r][tid] = xval[(r - 1) * xstride + rec];
        }
        __syncthreads();
        // one branch-free evaluation per entry: z entries take their offset
        // from the tile, x and y entries from the footprint origin
        for (int i = tid; i < cnt * wk; i += 256) {
            const int j = small_div(i, rwk), r = i - __mul24(j, wk);
            const int rr = r - kTileZ;
            const int d = r < kTileZ ? 2 : (rr >= w ? 1 : 0);
            const int q = r < kTileZ ? r - (&org[0][0])[__mul24(j, 3) + 2] : rr - (d ? w : 0);
            const T k = es_kernel(((&frac[0][0])[__mul24(j, 3) + d] + T(q)) * two_over_w, beta);
            (&kv[0][0])[__mul24(j, kKv) + r] = (unsigned)q < (unsigned)w ? k : T(0);
        }
        __syncthreads();
        for (int j = 0; j < cnt; ++j) {
            const int qx = x - org[j][0], qy = y - org[j][1];
            if ((unsigned)qx >= (unsigned)w || (unsigned)qy >= (unsigned)w) continue;
            const T kxy = kv[j][kTileZ + qx] * kv[j][kTileZ + w + qy];
            T kz[kTileZ];
            load8(kv[j], kz);
            // the kernel weights of this source serve every data row
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const T vr = val[r][j].x * kxy, vi = val[r][j].y * kxy;
#pragma unroll
                for (int z = 0; z < kTileZ; ++z) {
                    accr[r][z] += vr * kz[z];
                    acci[r][z] += vi * kz[z];
                }
            }
        }
    }
    const PairDev &P = pairs[tile.pair];
    const int gx = ox + x, gy = oy + y;
    if (gx < P.n1[0] && gy < P.n1[1]) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            cplx<T> *grid = ws + r * ws_stride + P.bufG;   // row r's copy of the batch workspace
            if (tile.flags & kSpreadAdd) {
#pragma unroll
                for (int z = 0; z < kTileZ; ++z) {
                    const int gz = oz + z;
                    if (gz < P.n1[2]) {
                        T *c = reinterpret_cast<T *>(grid + ((int64_t)gz * P.n1[1] + gy) * P.n1[0] + gx);
                        atomicAdd(c, accr[r][z]);
                        atomicAdd(c + 1, acci[r][z]);
                    }
                }
            } else {
#pragma unroll
                for (int z = 0; z < kTileZ; ++z) {
                    const int gz = oz + z;
                    if (gz < P.n1[2])
                        grid[((int64_t)gz * P.n1[1] + gy) * P.n1[0] + gx] = mk<T>(accr[r][z], acci[r][z]);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// FFT passes (type-3 step 2: pre-correction + zero-padded FFT on grid 2).
// ---------------------------------------------------------------------------
// exp(2 pi i k / R) as (cos, sin), evaluated by the compiler: the angle is
// folded into [0, pi/4] with the quarter-turn and complement symmetries
// (integer arithmetic, exact) and the Taylor series summed there (eleven terms
// at |x| <= pi/4 leave a truncation below 1e-22).
constexpr double kPiRoots = 3.14159265358979323846;
constexpr double taylor_sin(double x)
{
    double t = x, s = x;
    for (int i = 1; i < 12; ++i) { t *= -x * x / ((2.0 * i) * (2.0 * i + 1.0)); s += t; }
    return s;
}
constexpr double taylor_cos(double x)
{
    double t = 1.0, s = 1.0;
    for (int i = 1; i < 12; ++i) { t *= -x * x / ((2.0 * i - 1.0) * (2.0 * i)); s += t; }
    return s;
}
template <int R> struct Roots {
    double c[R], s[R];
    constexpr Roots() : c(), s()
    {
        for (int k = 0; k < R; ++k) {
            const int q = (4 * k) / R, r = 4 * k - q * R;   // angle (pi/2)(q + r/R), 0 <= r < R
            double cr = 0.0, sr = 0.0;
            if (2 * r <= R) { const double x = kPiRoots / 2 * r / R; cr = taylor_cos(x); sr = taylor_sin(x); }
            else { const double x = kPiRoots / 2 * (R - r) / R; cr = taylor_sin(x); sr = taylor_cos(x); }
            for (int i = 0; i < q; ++i) { const double t = cr; cr = -sr; sr = t; }   // q quarter turns
            c[k] = cr;
            s[k] = sr;
        }
    }
};

template <typename T, int R> __device__ __forceinline__ void dft_small(cplx<T> *u, T s);

// R1 R2-point DFT in registers (Cooley-Tukey, one level): input q = R2 q1 + q2,
// output m = m1 + R1 m2.  An R1-point DFT over q1 for every q2, the twiddle
// w^(q2 m1) with w = exp(s 2 pi i / (R1 R2)), then an R2-point DFT over q2 for
// every m1.
template <typename T, int R1, int R2>
__device__ __forceinline__ void dft_two_factor(cplx<T> *u, T s)
{
    constexpr int R = R1 * R2;
    constexpr Roots<R> W{};
    cplx<T> t[R2][R1];
#pragma unroll
    for (int q2 = 0; q2 < R2; ++q2) {
#pragma unroll
        for (int q1 = 0; q1 < R1; ++q1) t[q2][q1] = u[R2 * q1 + q2];
        dft_small<T, R1>(t[q2], s);
#pragma unroll
        for (int m1 = 1; m1 < R1; ++m1) {
            const int k = (q2 * m1) % R;
            if (k == 0) continue;
            if ((4 * k) % R == 0) {   // a quarter turn: exact
                const int qt = 4 * k / R;
                t[q2][m1] = qt == 1 ? cmuli<T>(t[q2][m1], s)
                          : qt == 2 ? mk<T>(-t[q2][m1].x, -t[q2][m1].y) : cmuli<T>(t[q2][m1], -s);
            } else {
                const T c = T(W.c[k]), sn = s * T(W.s[k]);
                const cplx<T> a = t[q2][m1];
                t[q2][m1] = mk<T>(a.x * c - a.y * sn, a.y * c + a.x * sn);
            }
        }
    }
#pragma unroll
    for (int m1 = 0; m1 < R1; ++m1) {
        cplx<T> b[R2];
#pragma unroll
        for (int q2 = 0; q2 < R2; ++q2) b[q2] = t[q2][m1];
        dft_small<T, R2>(b, s);
#pragma unroll
        for (int m2 = 0; m2 < R2; ++m2) u[m1 + R1 * m2] = b[m2];
    }
}

// In-place R-point DFT u_m <- sum_q u_q exp(s 2 pi i q m / R), s = +-1.
template <typename T, int R>
__device__ __forceinline__ void dft_small(cplx<T> *u, T s)
{
    if constexpr (R == 2) {
        cplx<T> a = u[0], b = u[1];
        u[0] = cadd<T>(a, b);
        u[1] = csub<T>(a, b);
    } else if constexpr (R == 3) {
        const T h = T(0.86602540378443864676);
        cplx<T> t1 = cadd<T>(u[1], u[2]), t2 = csub<T>(u[1], u[2]);
        cplx<T> m = mk<T>(u[0].x - T(0.5) * t1.x, u[0].y - T(0.5) * t1.y);
        cplx<T> r = cmuli<T>(cscale<T>(t2, h), s);
        u[0] = cadd<T>(u[0], t1);
        u[1] = cadd<T>(m, r);
        u[2] = csub<T>(m, r);
    } else if constexpr (R == 4) {
        cplx<T> a = cadd<T>(u[0], u[2]), b = csub<T>(u[0], u[2]);
        cplx<T> c = cadd<T>(u[1], u[3]), d = csub<T>(u[1], u[3]);
        cplx<T> id = cmuli<T>(d, s);
        u[0] = cadd<T>(a, c);
        u[2] = csub<T>(a, c);
        u[1] = cadd<T>(b, id);
        u[3] = csub<T>(b, id);
    } else if constexpr (R == 8) {
        // two 4-point DFTs (even and odd inputs) joined with w^m, w = exp(s 2 pi i / 8)
        const T h = T(0.70710678118654752440);
        cplx<T> e[4] = {u[0], u[2], u[4], u[6]}, o[4] = {u[1], u[3], u[5], u[7]};
        dft_small<T, 4>(e, s);
        dft_small<T, 4>(o, s);
        const cplx<T> o1 = mk<T>(h * (o[1].x - s * o[1].y), h * (o[1].y + s * o[1].x));    // w^1 = (1 + i s)/sqrt2
        const cplx<T> o2 = cmuli<T>(o[2], s);                                              // w^2 = i s
        const cplx<T> o3 = mk<T>(-h * (o[3].x + s * o[3].y), h * (s * o[3].x - o[3].y));   // w^3 = (-1 + i s)/sqrt2
        u[0] = cadd<T>(e[0], o[0]);
        u[4] = csub<T>(e[0], o[0]);
        u[1] = cadd<T>(e[1], o1);
        u[5] = csub<T>(e[1], o1);
        u[2] = cadd<T>(e[2], o2);
        u[6] = csub<T>(e[2], o2);
        u[3] = cadd<T>(e[3], o3);
        u[7] = csub<T>(e[3], o3);
    } else if constexpr (R == 9) {
        dft_two_factor<T, 3, 3>(u, s);
    } else {
        static_assert(R == 5, "radix");
        const T c1 = T(0.30901699437494742410), c2 = T(-0.80901699437494742410);
        const T s1 = T(0.95105651629515357212), s2 = T(0.58778525229247312917);
        cplx<T> t1 = cadd<T>(u[1], u[4]), t2 = cadd<T>(u[2], u[3]);
        cplx<T> t3 = csub<T>(u[1], u[4]), t4 = csub<T>(u[2], u[3]);
        cplx<T> a1 = mk<T>(u[0].x + c1 * t1.x + c2 * t2.x, u[0].y + c1 * t1.y + c2 * t2.y);
        cplx<T> a2 = mk<T>(u[0].x + c2 * t1.x + c1 * t2.x, u[0].y + c2 * t1.y + c1 * t2.y);
        cplx<T> b1 = cmuli<T>(mk<T>(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y), s);
        cplx<T> b2 = cmuli<T>(mk<T>(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y), s);
        u[0] = cadd<T>(u[0], cadd<T>(t1, t2));
        u[1] = cadd<T>(a1, b1);
        u[4] = csub<T>(a1, b1);
        u[2] = cadd<T>(a2, b2);
        u[3] = csub<T>(a2, b2);
    }
}

// One Stockham stage of radix R on nl lines of length n held in LDS, in
// place: every thread first reads and transforms its butterflies into
// registers, then (after a barrier) writes them back in autosorted order.
// Butterfly i of a line: k = i mod p, inputs x[i + q n/R] twiddled by
// w^(k q n / (p R)), outputs at (i - k) R + k + m p.  The first stage
// (FIRST, p = 1) has k = 0: no twiddles.
template <typename T, int R, int NT, bool FIRST>
__device__ __forceinline__ void fft_stage(cplx<T> *lds, int nl, int n, int ls, int p, const cplx<T> *tw, T s)
{
    constexpr int MAXB = (fft_elems(NT) / R + NT - 1) / NT;
    const int nbf = n / R;
    const int total = nl * nbf;
    const int twstep = FIRST ? 0 : small_div(n, small_rcp(p * R));   // exact: p R divides n
    const int pR = p * R;
    const float rnbf = small_rcp(nbf), rp = FIRST ? 1.0f : small_rcp(p);
    cplx<T> v[MAXB][R];
    int obase[MAXB];
    // the thread index, opaque to the optimiser: otherwise the butterfly
    // indices of every radix case are hoisted out of the loop over stages and
    // held in registers across it (64 VGPRs, which halved the occupancy)
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
#pragma unroll
    for (int c = 0; c < MAXB; ++c) {
        const int b = tid + c * NT;
        obase[c] = -1;
        if (b < total) {
            const int j = small_div(b, rnbf), i = b - __mul24(j, nbf);
            const int g = FIRST ? i : small_div(i, rp), k = FIRST ? 0 : i - __mul24(g, p);
            const int lb = __mul24(j, ls);   // line j starts at j * ls in LDS
            obase[c] = lb + __mul24(g, pR) + k;
            const int tk = __mul24(k, twstep);
#pragma unroll
            for (int q = 0; q < R; ++q) {
                cplx<T> u = lds[lb + i + __mul24(q, nbf)];
                // exponent q k twstep < n; the LDS table holds exp(s 2 pi i j/n), j < n
                if (!FIRST && q > 0) u = cmul<T>(u, tw[__mul24(q, tk)]);
                v[c][q] = u;
            }
            dft_small<T, R>(v[c], s);
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < MAXB; ++c) {
        if (obase[c] >= 0) {
#pragma unroll
            for (int m = 0; m < R; ++m) lds[obase[c] + __mul24(m, p)] = v[c][m];
        }
    }
    __syncthreads();
}

// A stage of any of the planner's radices (2, 3, 4, 5, 8, 9).
template <typename T, int NT, bool FIRST>
__device__ __forceinline__ void fft_stage_radix(int R, cplx<T> *lds, int nl, int n, int ls, int p, const cplx<T> *tw, T s)
{
    switch (R) {
    case 9: fft_stage<T, 9, NT, FIRST>(lds, nl, n, ls, p, tw, s); break;
    case 8: fft_stage<T, 8, NT, FIRST>(lds, nl, n, ls, p, tw, s); break;
    case 5: fft_stage<T, 5, NT, FIRST>(lds, nl, n, ls, p, tw, s); break;
    case 4: fft_stage<T, 4, NT, FIRST>(lds, nl, n, ls, p, tw, s); break;
    case 3: fft_stage<T, 3, NT, FIRST>(lds, nl, n, ls, p, tw, s); break;
    default: fft_stage<T, 2, NT, FIRST>(lds, nl, n, ls, p, tw, s); break;
    }
}

// One axis pass for every sub-problem of a batch.  Element e of an input
// line is mode l = e - nin/2, placed at FFT slot l mod n (zero elsewhere: the
// zero padding of grid 1 into grid 2 is never stored).  The x and y passes
// read contiguous lines; the z pass reads its lines strided (line j of the
// plane is element j of every z-slab, so consecutive lines sit in adjacent
// lanes).  The x pass also applies the separable pre-correction
// 1/Phi_hat(l/n2) of all three axes (the (y, z) factor once per line) and
// reads grid-1 tiles that hold no source as zeros.  The second grid
// dimension runs over the data rows of the pass.  Output
// q of the kept window is FFT index (wstart + q) mod n, written line-major:
// out[line][q].
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_fft_pass(const PairDev *__restrict__ pairs, const int64_t *__restrict__ prefix,
                                                 int npairs, int pass, cplx<T> *__restrict__ ws,
                                                 const cplx<T> *__restrict__ twtab, const T *__restrict__ precor,
                                                 const uint32_t *__restrict__ occ, int tw_off, T s,
                                                 int64_t ws_stride)
{
    static_assert(kTileX == 32, "a grid-1 tile spans 32 cells of an x line");
    ws += (int64_t)blockIdx.y * ws_stride;   // data row blockIdx.y: its copy of the batch workspace
    extern __shared__ unsigned char smem_raw[];
    cplx<T> *lds = reinterpret_cast<cplx<T> *>(smem_raw);
    cplx<T> *ltw = lds + tw_off;              // exp(s 2 pi i j/n), j < n, after the lines
    __shared__ T lfac[kFftMaxLines];
    __shared__ uint32_t lmask[kFftMaxLines][kOccWords];   // x pass: occupancy bits of each line's tile row
    __shared__ int lbit0[kFftMaxLines];
    const int p = (int)find_segment(prefix, npairs, blockIdx.x);
    const PairDev &P = pairs[p];
    const int64_t tile = (int64_t)blockIdx.x - prefix[p];
    const int n = P.n2[pass], nin = P.n1[pass];
    const int wst = P.wstart[pass], wcnt = P.wcount[pass];
    int64_t lines;
    const cplx<T> *src;
    cplx<T> *dst;
    if (pass == 0) { lines = (int64_t)P.n1[2] * P.n1[1]; src = ws + P.bufG; dst = ws + P.bufB; }
    else if (pass == 1) { lines = (int64_t)P.n1[2] * P.wcount[0]; src = ws + P.bufA; dst = ws + P.bufB; }
    else { lines = (int64_t)P.wcount[0] * P.wcount[1]; src = ws + P.bufB; dst = ws + P.bufA; }
    const int L = P.lines_per_tile[pass];
    const int64_t line0 = tile * L;
    const int nl = (int)min((int64_t)L, lines - line0);
    const int half_in = nin / 2, half_n = n / 2;
    const int ls = fft_lds_stride(n);   // LDS line stride

    {
        // twiddles of this line length, staged with the data (sign s applied here)
        const cplx<T> *tw = twtab + P.tw[pass];
        for (int j = threadIdx.x; j < n; j += NT) {
            cplx<T> t = tw[j];
            t.y *= -s;   // table holds exp(-2 pi i j/n); s = -1 keeps it, +1 conjugates
            ltw[j] = t;
        }
    }
    if (pass == 0) {
        if ((int)threadIdx.x < nl) {
            const int64_t li = line0 + threadIdx.x;
            const int64_t lz = li / P.n1[1], ly = li - lz * P.n1[1];
            lfac[threadIdx.x] = precor[P.precor[1] + ly] * precor[P.precor[2] + lz];
            // tiles of this line's row: bit rowbit + tx is tile (tx, ly / 8, lz / 8) of the pair;
            // a tile without sources was never written and reads as zeros (no bitmap: all read)
            const int64_t rowbit = P.tile0 + ((lz / kTileZ) * P.ntile[1] + ly / kTileY) * P.ntile[0];
            lbit0[threadIdx.x] = (int)(rowbit & 31);
            for (int q = 0; q < kOccWords; ++q) lmask[threadIdx.x][q] = occ ? occ[(rowbit >> 5) + q] : ~0u;
        }
        __syncthreads();
    }
    // every thread loads its (at most) fft_elems(NT) / NT elements into
    // registers first, so the global loads are all in flight together, then
    // writes them to LDS
    constexpr int EPT = fft_elems(NT) / NT;
    static_assert(fft_elems(NT) % NT == 0, "FFT workgroup elements");
    const int ne = nl * n;
    cplx<T> v[EPT];
    if (pass < 2) {
        const cplx<T> *sb = src + line0 * nin;
        const T *px = precor + P.precor[0] + half_in;
        const float rn = small_rcp(n);
        T fx[EPT];             // x pre-correction (pass x), applied after all loads are issued
        int jl[EPT], slot[EPT];
#pragma unroll
        for (int c = 0; c < EPT; ++c) {
            const int e = threadIdx.x + c * NT;
            v[c] = mk<T>(T(0), T(0));
            fx[c] = T(1);
            jl[c] = 0;
            slot[c] = 0;
            if (e < ne) {
                const int j = small_div(e, rn), f = e - __mul24(j, n);
                const int l = f < half_n ? f : f - n;
                jl[c] = j;
                slot[c] = __mul24(j, ls) + f;
                bool take = l >= -half_in && l < half_in;
                if (pass == 0 && take) {
                    const int b = lbit0[j] + ((l + half_in) >> 5);
                    take = (lmask[j][b >> 5] >> (b & 31)) & 1u;
                }
                if (take) {
                    v[c] = sb[__mul24(j, nin) + l + half_in];
                    if (pass == 0) fx[c] = px[l];
                }
            }
        }
#pragma unroll
        for (int c = 0; c < EPT; ++c) {
            const int e = threadIdx.x + c * NT;
            if (e < ne) lds[slot[c]] = pass == 0 ? cscale<T>(v[c], fx[c] * lfac[jl[c]]) : v[c];
        }
    } else {
        const cplx<T> *sb = src + line0;
        const float rl = small_rcp(nl);
        int slot[EPT];
#pragma unroll
        for (int c = 0; c < EPT; ++c) {
            const int e = threadIdx.x + c * NT;
            v[c] = mk<T>(T(0), T(0));
            slot[c] = -1;
            if (e < ne) {
                const int f = small_div(e, rl), j = e - __mul24(f, nl);
                const int l = f < half_n ? f : f - n;
                slot[c] = __mul24(j, ls) + f;
                if (l >= -half_in && l < half_in) v[c] = sb[(int64_t)(l + half_in) * lines + j];
            }
        }
#pragma unroll
        for (int c = 0; c < EPT; ++c)
            if (slot[c] >= 0) lds[slot[c]] = v[c];
    }
    __syncthreads();
    int pc = 1;
    for (int st = 0; st < P.nrad[pass]; ++st) {
        const int R = P.radix[pass][st];
        if (st == 0) fft_stage_radix<T, NT, true>(R, lds, nl, n, ls, pc, ltw, s);
        else fft_stage_radix<T, NT, false>(R, lds, nl, n, ls, pc, ltw, s);
        pc *= R;
    }
    // kept window: wstart is 0 (whole line) or -R with 2R < n, so wstart + q lies in (-n, n)
    cplx<T> *out = dst + line0 * wcnt;
    const float rw = small_rcp(wcnt);
    for (int e = threadIdx.x; e < nl * wcnt; e += NT) {
        const int j = small_div(e, rw), q = e - __mul24(j, wcnt);
        int m = wst + q;
        if (m < 0) m += n;
        out[e] = lds[__mul24(j, ls) + m];
    }
}

// Transpose of the x-pass output for the y pass: per z-slab, B[y][x'] ->
// A[x'][y], through a padded LDS tile so reads and writes are both coalesced.
template <typename T>
__global__ __launch_bounds__(256) void k_transpose(const PairDev *__restrict__ pairs, const int64_t *__restrict__ prefix,
                                                   int npairs, cplx<T> *__restrict__ ws, int64_t ws_stride)
{
    __shared__ cplx<T> tile[kTransposeTile][kTransposeTile + 1];
    ws += (int64_t)blockIdx.y * ws_stride;   // data row blockIdx.y
    const int p = (int)find_segment(prefix, npairs, blockIdx.x);
    const PairDev &P = pairs[p];
    const int64_t local = (int64_t)blockIdx.x - prefix[p];
    const int R = P.n1[1], C = P.wcount[0];
    const int tr = (R + kTransposeTile - 1) / kTransposeTile, tc = (C + kTransposeTile - 1) / kTransposeTile;
    const int64_t z = local / ((int64_t)tr * tc);
    const int rem = (int)(local - z * tr * tc);
    const int ti = rem / tc, tj = rem - ti * tc;
    const cplx<T> *in = ws + P.bufB + z * (int64_t)R * C;
    cplx<T> *out = ws + P.bufA + z * (int64_t)R * C;
    const int tx = threadIdx.x % kTransposeTile, ty = threadIdx.x / kTransposeTile;
    constexpr int rows_per_pass = 256 / kTransposeTile;
#pragma unroll
    for (int k = 0; k < kTransposeTile; k += rows_per_pass) {
        const int r = ti * kTransposeTile + ty + k, c = tj * kTransposeTile + tx;
        if (r < R && c < C) tile[ty + k][tx] = in[(int64_t)r * C + c];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kTransposeTile; k += rows_per_pass) {
        const int c = tj * kTransposeTile + ty + k, r = ti * kTransposeTile + tx;
        if (r < R && c < C) out[(int64_t)c * R + r] = tile[tx][ty + k];
    }
}

// ---------------------------------------------------------------------------
// exp(2 pi i t) with t in revolutions, t reduced in float64 (phases of the
// interpolation epilogue and of the direct sum).
// ---------------------------------------------------------------------------
// exp(2 pi i t) for the float32 plan: fractional part in float64, then the
// hardware sine / cosine, whose argument is in revolutions.
__device__ __forceinline__ void cis_rev(double t, float &c, float &s)
{
    const float r = static_cast<float>(__builtin_amdgcn_fract(t));
    s = __builtin_amdgcn_sinf(r);
    c = __builtin_amdgcn_cosf(r);
}

// exp(2 pi i t) for the float64 plan: reduce t to the nearest quarter turn,
// t = q/4 + f with |f| <= 1/8, evaluate sin and cos of theta = 2 pi f by their
// Maclaurin series through theta^13 / theta^14 (truncation below 3e-14 on
// |theta| <= pi/4), then rotate by q quarter turns.
__device__ __forceinline__ void cis_rev(double t, double &c, double &s)
{
    const double q = rint(4.0 * t);
    const double f = fma(q, -0.25, t);
    const double th = 6.283185307179586476925287 * f;
    const double z = th * th;
    double ps = 1.0 / 6227020800.0;                 // 1/13!
    ps = fma(ps, -z, 1.0 / 39916800.0);             // 1/11!
    ps = fma(ps, -z, 1.0 / 362880.0);               // 1/9!
    ps = fma(ps, -z, 1.0 / 5040.0);                 // 1/7!
    ps = fma(ps, -z, 1.0 / 120.0);                  // 1/5!
    ps = fma(ps, -z, 1.0 / 6.0);                    // 1/3!
    const double sn = fma(-ps * z, th, th);
    double pc = 1.0 / 87178291200.0;                // 1/14!
    pc = fma(pc, -z, 1.0 / 479001600.0);            // 1/12!
    pc = fma(pc, -z, 1.0 / 3628800.0);              // 1/10!
    pc = fma(pc, -z, 1.0 / 40320.0);                // 1/8!
    pc = fma(pc, -z, 1.0 / 720.0);                  // 1/6!
    pc = fma(pc, -z, 1.0 / 24.0);                   // 1/4!
    pc = fma(pc, -z, 0.5);                          // 1/2!
    const double cs = fma(-pc, z, 1.0);
    const int k = static_cast<int>(q) & 3;
    const double s1 = (k & 1) ? cs : sn;
    const double c1 = (k & 1) ? sn : cs;
    s = (k & 2) ? -s1 : s1;
    c = (k == 1 || k == 2) ? -c1 : c1;
}

// exp(2 pi i t) in float64 from a table of exp(2 pi i k / kCisTab) (float64,
// filled on the host) and the Taylor terms of the remainder: with u =
// kCisTab t, k = rint(u) and f = u - k in [-1/2, 1/2], exp(2 pi i t) =
// tab[k mod kCisTab] exp(i theta), theta = 2 pi f / kCisTab, |theta| <= pi /
// kCisTab; sin theta ~ theta - theta^3 / 6 and cos theta ~ 1 - theta^2 / 2 +
// theta^4 / 24 leave a truncation below theta^5 / 120 = 2.3e-15 (kCisTab =
// 1024), the scale 2 pi / kCisTab folded into the coefficients.  k comes from
// one add of 1.5 2^52, which rounds u to an integer in round-to-nearest and
// leaves k + 2^51 in the low bits of the sum's mantissa (|u| < 2^51, i.e.
// |t| < 2^41 turns); the scaling by a power of two and the split u = k + f
// are exact.
__device__ __forceinline__ void cis_tab(double t, const double2 *tab, double &c, double &s)
{
    static_assert((kCisTab & (kCisTab - 1)) == 0, "power-of-two table");
    constexpr double kRound = 6755399441055744.0;                 // 1.5 * 2^52
    constexpr double a1 = 6.283185307179586476925287 / kCisTab;   // theta = a1 f
    constexpr double a3 = -a1 * a1 * a1 / 6.0, b2 = -a1 * a1 / 2.0, b4 = a1 * a1 * a1 * a1 / 24.0;
    double u, m;
    {
        // separate multiply and add (no contraction): a fused form would need the
        // 1.5 2^52 addend in a vector register per term
#pragma clang fp contract(off)
        u = t * static_cast<double>(kCisTab);
        m = u + kRound;
    }
    const double f = u - (m - kRound);                             // [-1/2, 1/2]
    const double2 e = tab[__double2loint(m) & (kCisTab - 1)];       // k + 2^51 = k mod kCisTab
    const double f2 = f * f;
    const double sn = f * fma(f2, a3, a1);
    const double cs = fma(f2, fma(f2, b4, b2), 1.0);
    c = fma(e.x, cs, -e.y * sn);
    s = fma(e.y, cs, e.x * sn);
}

// ---------------------------------------------------------------------------
// interpolation + deconvolution + post-phase (type-3 steps 3-4):
//   f_k += exp(2 pi i iota s_k.x_c) / prod Psi_hat(.) * sum_m G_m prod_d ES((m_d - tau_kd) 2/w)
// A group of kInterpLanes lanes per target (four targets per wavefront,
// kInterpTargets targets of one sub-problem per workgroup);
// the lanes cover the (y, z) pairs of its w^3 window (z fastest, as the
// grid), loop over x, and reduce across the group.  Accumulation is float64
// (cross-sub-problem sums stay in double precision).  NR data rows share the
// kernel weights, addresses and post-phase of each target (row r reads the
// r-th copy of the batch workspace and adds into accumulator row r).
// ---------------------------------------------------------------------------
template <typename T, int NR>
__global__ __launch_bounds__(256) void k_interp(const PairDev *__restrict__ pairs, const int64_t *__restrict__ bprefix,
                                                int npairs, int64_t block0, const double *__restrict__ xyz,
                                                int64_t ntgt, const double *__restrict__ deconv,
                                                const cplx<T> *__restrict__ ws, int64_t ws_stride,
                                                double *__restrict__ acc, int64_t acc_stride, int w, T beta,
                                                double iota, int det)
{
    __shared__ T ker[kInterpTargets][3 * kWMax];
    const int sub = threadIdx.x & (kInterpLanes - 1), slot = threadIdx.x / kInterpLanes;
    const T two_over_w = T(2) / T(w);
    // every workgroup serves kInterpTargets consecutive targets of one sub-problem
    const int64_t blk = block0 + blockIdx.x;
    const int p = (int)find_segment(bprefix, npairs, blk);
    const PairDev &P = pairs[p];
    const int64_t local = (blk - bprefix[p]) * kInterpTargets + slot;
    const bool active = local < P.tgt_cnt;
    const int64_t k = P.tgt_off + (active ? local : 0);
    double s_k[3];
    int m0[3];
    for (int d = 0; d < 3; ++d) {
        s_k[d] = xyz[d * ntgt + k];
        const double tau = (s_k[d] - P.sc[d]) * P.tscale[d];
        m0[d] = (int)ceil(tau - 0.5 * w);
        for (int q = sub; q < w; q += kInterpLanes)
            ker[slot][d * w + q] = es_kernel(T((double)(m0[d] + q) - tau) * two_over_w, beta);
    }
    __syncthreads();
    T ar[NR], ai[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) ar[r] = ai[r] = T(0);
    if (active) {
        const int wx = P.wcount[0], wy = P.wcount[1], wz = P.wcount[2];
        const bool fx = wx == P.n2[0], fy = wy == P.n2[1], fz = wz == P.n2[2];   // whole (periodic) axis kept
        const int n2x = P.n2[0], n2y = P.n2[1], n2z = P.n2[2];
        const int sx = P.wstart[0], sy = P.wstart[1], sz = P.wstart[2];
        const cplx<T> *grid = ws + P.bufA;          // [wx][wy][wz], z fastest; row r at r * ws_stride
        const int xstride = wy * wz;
        // x cells eight at a time (the offsets and weights of a chunk shared by every
        // (y, z) row of the target and every data row); cells beyond the kernel support
        // or outside the kept window get weight 0 and the address of a cell the target
        // reads anyway (its last column, clamped into the window), so the loads carry
        // no branches and fetch no line the window does not need.  Each lane takes two
        // (y, z) rows per step, sixteen loads in flight per data row.
        auto column = [&](int e, T &kyz) -> const cplx<T> * {
            const int dy = e / w, dz = e - dy * w;
            int qy = m0[1] + dy - sy, qz = m0[2] + dz - sz;
            if (fy) { qy %= n2y; if (qy < 0) qy += n2y; }
            if (fz) { qz %= n2z; if (qz < 0) qz += n2z; }
            const bool ok = qy >= 0 && qy < wy && qz >= 0 && qz < wz;
            kyz = ok ? ker[slot][w + dy] * ker[slot][2 * w + dz] : T(0);
            return grid + (ok ? qy * wz + qz : 0);
        };
        for (int dx0 = 0; dx0 < w; dx0 += 8) {
            int64_t xo[8];
            T kx[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int dx = min(dx0 + u, w - 1);
                int qx = m0[0] + dx - sx;
                if (fx) { qx %= n2x; if (qx < 0) qx += n2x; }
                const bool okx = dx0 + u < w && qx >= 0 && qx < wx;
                kx[u] = okx ? ker[slot][dx] : T(0);
                xo[u] = (int64_t)min(max(qx, 0), wx - 1) * xstride;
            }
            for (int e0 = sub; e0 < w * w; e0 += 2 * kInterpLanes) {
                const int e1 = e0 + kInterpLanes;
                const bool has1 = e1 < w * w;
                T kyz0, kyz1;
                const cplx<T> *col0 = column(e0, kyz0);
                const cplx<T> *col1 = column(has1 ? e1 : e0, kyz1);   // no second row: a repeat, weight 0
                if (!has1) kyz1 = T(0);
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const cplx<T> *c0 = col0 + r * ws_stride, *c1 = col1 + r * ws_stride;
                    cplx<T> g0[8], g1[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        g0[u] = c0[xo[u]];
                        g1[u] = c1[xo[u]];
                    }
                    T s0r = T(0), s0i = T(0), s1r = T(0), s1i = T(0);
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        s0r += g0[u].x * kx[u];
                        s0i += g0[u].y * kx[u];
                        s1r += g1[u].x * kx[u];
                        s1i += g1[u].y * kx[u];
                    }
                    ar[r] += s0r * kyz0 + s1r * kyz1;
                    ai[r] += s0i * kyz0 + s1i * kyz1;
                }
            }
        }
    }
    // reduce over the target's lane group (xor offsets below the group size stay inside it)
#pragma unroll
    for (int r = 0; r < NR; ++r)
        for (int off = kInterpLanes / 2; off > 0; off >>= 1) {
            ar[r] += __shfl_xor(ar[r], off, 64);
            ai[r] += __shfl_xor(ai[r], off, 64);
        }
    if (active && sub == 0) {
        // post-phase exp(2 pi i iota s_k.x_c) in float64 in both precisions
        double ph = 0.0;
        for (int d = 0; d < 3; ++d) ph += s_k[d] * P.xc[d];
        double er, ei;
        cis_rev(iota * ph, er, ei);
        const double dk = deconv[k];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            double *a = acc + r * acc_stride;
            const double vr = (double)ar[r] * dk, vi = (double)ai[r] * dk;
            if (det) {
                // deterministic plans: no other workgroup of this launch adds into target k
                a[2 * k] += vr * er - vi * ei;
                a[2 * k + 1] += vr * ei + vi * er;
            } else {
                atomicAdd(a + 2 * k, vr * er - vi * ei);
                atomicAdd(a + 2 * k + 1, vr * ei + vi * er);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// direct evaluation of a sub-problem block (Sect. 3.1, last bullet; the
// eps = 0 mode of Sect. 4):  f_k += sum_n c_n exp(2 pi i iota s_k.x_n).
// A workgroup of 256 threads owns <= 512 targets (two per thread) and
// <= kDirectSeg sources, staged 256 at a time in LDS, for NT data rows at
// once (the phase factors are computed once and applied to every row).  Per source tile with reference
// point x_S and target-tile reference s_T,
//   s_k.x_n = s_k.x_S + s_T.(x_n - x_S) + (s_k - s_T).(x_n - x_S):
// the first two terms are evaluated once per (target, tile) and
// (source, tile); only the small third term is evaluated per (target,
// source) pair.  Every phase is reduced to a fraction of a turn in float64
// and its sine / cosine taken in the plan's precision for the per-pair term
// (cis_rev), in float64 for the per-tile reference terms.  The sign iota
// multiplies the target offsets and the reference phases, so the inner loop
// always accumulates c exp(+2 pi i t).  Phases are float64 (full rate on CDNA).
// ---------------------------------------------------------------------------

template <typename T, int NT>
__device__ __forceinline__ void direct_item(const DirectItem it, const double *__restrict__ sxyz, int64_t nsrc,
                                            const double *__restrict__ txyz, int64_t ntgt,
                                            const int32_t *__restrict__ perm, const cplx<T> *__restrict__ in,
                                            int64_t in_stride, double *__restrict__ acc, int64_t acc_stride,
                                            double iota, int det, double *lx, double *ly, double *lz,
                                            cplx<T> (*lc)[kDirectSrcTile], const double2 *ltab)
{
    const int tid = threadIdx.x;
    // two targets per thread: each staged source is read from LDS once for both
    const bool has0 = tid < it.tgt_cnt, has1 = tid + kDirectThreads < it.tgt_cnt;
    const int64_t k0 = it.tgt_off + (has0 ? tid : 0);
    const int64_t k1 = it.tgt_off + (has1 ? tid + kDirectThreads : 0);
    double sT[3], sk0[3], sk1[3], sp0[3], sp1[3];
    for (int d = 0; d < 3; ++d) {
        sT[d] = txyz[d * ntgt + it.tgt_off];
        sk0[d] = txyz[d * ntgt + k0];
        sk1[d] = txyz[d * ntgt + k1];
        sp0[d] = iota * (sk0[d] - sT[d]);        // the sign enters through the phase
        sp1[d] = iota * (sk1[d] - sT[d]);
    }
    double a0r[NT], a0i[NT], a1r[NT], a1i[NT];
#pragma unroll
    for (int r = 0; r < NT; ++r) a0r[r] = a0i[r] = a1r[r] = a1i[r] = 0.0;
    for (int s0 = 0; s0 < it.src_cnt; s0 += kDirectSrcTile) {
        const int64_t nS = it.src_off + s0;
        double xS[3];
        for (int d = 0; d < 3; ++d) xS[d] = sxyz[d * nsrc + nS];
        const int cnt = min(kDirectSrcTile, it.src_cnt - s0);
        __syncthreads();
        if (tid < cnt) {
            const int64_t n = nS + tid;
            double dxv[3];
            double ph = 0.0;
            for (int d = 0; d < 3; ++d) {
                dxv[d] = sxyz[d * nsrc + n] - xS[d];
                ph += sT[d] * dxv[d];
            }
            lx[tid] = dxv[0];
            ly[tid] = dxv[1];
            lz[tid] = dxv[2];
            double ec, es;
            cis_rev(iota * ph, ec, es);   // exp(2 pi i iota ph), float64
            const int64_t u = perm ? perm[n] : n;
#pragma unroll
            for (int r = 0; r < NT; ++r) {
                const cplx<T> c = in[r * in_stride + u];
                lc[r][tid] = mk<T>(T(c.x * ec - c.y * es), T(c.x * es + c.y * ec));
            }
        }
        __syncthreads();
        T b0r[NT], b0i[NT], b1r[NT], b1i[NT];
#pragma unroll
        for (int r = 0; r < NT; ++r) b0r[r] = b0i[r] = b1r[r] = b1i[r] = T(0);
#pragma unroll 4
        for (int j = 0; j < cnt; ++j) {
            const double xj = lx[j], yj = ly[j], zj = lz[j];
            const double t0 = fma(sp0[0], xj, fma(sp0[1], yj, sp0[2] * zj));
            const double t1 = fma(sp1[0], xj, fma(sp1[1], yj, sp1[2] * zj));
            T c0, s0v, c1, s1v;
            if constexpr (sizeof(T) == 8) {   // float64 plan: the LDS phase table
                cis_tab(t0, ltab, c0, s0v);
                cis_tab(t1, ltab, c1, s1v);
            } else {                          // float32 plan: the hardware sine / cosine
                cis_rev(t0, c0, s0v);
                cis_rev(t1, c1, s1v);
            }
            // one phase factor per (target, source), applied to every row
#pragma unroll
            for (int r = 0; r < NT; ++r) {
                const cplx<T> c = lc[r][j];
                b0r[r] = fma(c.x, c0, fma(-c.y, s0v, b0r[r]));
                b0i[r] = fma(c.x, s0v, fma(c.y, c0, b0i[r]));
                b1r[r] = fma(c.x, c1, fma(-c.y, s1v, b1r[r]));
                b1i[r] = fma(c.x, s1v, fma(c.y, c1, b1i[r]));
            }
        }
        double ph0 = 0.0, ph1 = 0.0;
        for (int d = 0; d < 3; ++d) {
            ph0 += sk0[d] * xS[d];
            ph1 += sk1[d] * xS[d];
        }
        double e0c, e0s, e1c, e1s;   // tile reference phases, float64
        cis_rev(iota * ph0, e0c, e0s);
        cis_rev(iota * ph1, e1c, e1s);
        const double2 e0 = make_double2(e0c, e0s), e1 = make_double2(e1c, e1s);
#pragma unroll
        for (int r = 0; r < NT; ++r) {
            a0r[r] += (double)b0r[r] * e0.x - (double)b0i[r] * e0.y;
            a0i[r] += (double)b0r[r] * e0.y + (double)b0i[r] * e0.x;
            a1r[r] += (double)b1r[r] * e1.x - (double)b1i[r] * e1.y;
            a1i[r] += (double)b1r[r] * e1.y + (double)b1i[r] * e1.x;
        }
    }
#pragma unroll
    for (int r = 0; r < NT; ++r) {
        double *ar = acc + r * acc_stride;
        if (det) {
            // deterministic plans launch items sharing no target together (one layer)
            if (has0) { ar[2 * k0] += a0r[r]; ar[2 * k0 + 1] += a0i[r]; }
            if (has1) { ar[2 * k1] += a1r[r]; ar[2 * k1 + 1] += a1i[r]; }
        } else {
            if (has0) {
                atomicAdd(ar + 2 * k0, a0r[r]);
                atomicAdd(ar + 2 * k0 + 1, a0i[r]);
            }
            if (has1) {
                atomicAdd(ar + 2 * k1, a1r[r]);
                atomicAdd(ar + 2 * k1 + 1, a1i[r]);
            }
        }
    }
}

// One workgroup per work item, or (persistent launches, grid smaller than
// the item count) each workgroup loops over items blockIdx.x, + gridDim.x,
// ...: a capped grid leaves room on every CU for the kernels of the NUFFT
// sub-problems running beside the direct sum on another stream.  Items stay
// source-segment-major across consecutive workgroups either way.
template <typename T, int NT>
__global__ __launch_bounds__(kDirectThreads) void k_direct(const DirectItem *__restrict__ items, int64_t nitems,
                                                           const double *__restrict__ sxyz, int64_t nsrc,
                                                           const double *__restrict__ txyz, int64_t ntgt,
                                                           const int32_t *__restrict__ perm,
                                                           const cplx<T> *__restrict__ in, int64_t in_stride,
                                                           double *__restrict__ acc, int64_t acc_stride, double iota,
                                                           int det, const double2 *__restrict__ ctab)
{
    static_assert(kDirectSrcTile == kDirectThreads && kDirectTile == 2 * kDirectThreads, "direct tiling");
    __shared__ double lx[kDirectSrcTile], ly[kDirectSrcTile], lz[kDirectSrcTile];
    __shared__ cplx<T> lc[NT][kDirectSrcTile];
    __shared__ double2 ltab[sizeof(T) == 8 ? kCisTab : 1];   // float64 plans: the phase table
    if constexpr (sizeof(T) == 8) {
        for (int i = threadIdx.x; i < kCisTab; i += kDirectThreads) ltab[i] = ctab[i];
        // the first item's staging barrier orders these writes before any read
    }
    for (int64_t w = blockIdx.x; w < nitems; w += gridDim.x) {
        if (w != blockIdx.x) __syncthreads();   // the previous item's last tile is read before restaging
        direct_item<T, NT>(items[w], sxyz, nsrc, txyz, ntgt, perm, in, in_stride, acc, acc_stride, iota, det, lx, ly,
                           lz, lc, ltab);
    }
}

// ---------------------------------------------------------------------------
// epilogue: cast the float64 accumulator to the plan's precision and scatter
// to user order (the inverse of the chunk-order gather, Sect. 4 Fig. 5).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_finalize(const double *__restrict__ acc, int64_t n, const int32_t *__restrict__ perm,
                           cplx<T> *__restrict__ out, int real_only)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    out[perm ? perm[k] : k] = mk<T>(T(acc[2 * k]), real_only ? T(0) : T(acc[2 * k + 1]));
}

// ---------------------------------------------------------------------------
// direction-dependent gains in separable form A_k(r_n) = sum_t a[t][k] b[t][n]:
// the rows a transform takes (scale) and the sum of the transformed rows
// (combine).  out[t][i] = w'[t][i] x[i] and out[i] = sum_t w'[t][i] y[t][i],
// w' = w or conj(w); the combination accumulates in float64.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_dde_scale(const cplx<T> *__restrict__ w, const cplx<T> *__restrict__ x, cplx<T> *__restrict__ out,
                            int64_t n, int terms, int conj_w)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const cplx<T> v = x[i];
    for (int t = 0; t < terms; ++t) {
        cplx<T> g = w[(int64_t)t * n + i];
        if (conj_w) g.y = -g.y;
        out[(int64_t)t * n + i] = cmul<T>(g, v);
    }
}

template <typename T>
__global__ void k_dde_combine(const cplx<T> *__restrict__ w, const cplx<T> *__restrict__ y, cplx<T> *__restrict__ out,
                              int64_t n, int terms, int conj_w, int real_only)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double re = 0.0, im = 0.0;
    for (int t = 0; t < terms; ++t) {
        const cplx<T> g = w[(int64_t)t * n + i], v = y[(int64_t)t * n + i];
        const double gi = conj_w ? -(double)g.y : (double)g.y;
        re += (double)g.x * v.x - gi * v.y;
        im += (double)g.x * v.y + gi * v.x;
    }
    out[i] = mk<T>(T(re), real_only ? T(0) : T(im));
}

// ---------------------------------------------------------------------------
// launch wrappers (host)
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(int64_t n, int per, int64_t cap)
{
    int64_t b = (n + per - 1) / per;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return static_cast<unsigned>(b);
}

hipError_t launch_zero(double *p, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3(blocks_for(n, 256 * 8, 65536)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_deconv(const double *xyz, int64_t n, const int32_t *chunk_of, const double *ctr,
                         const double *hscale, const double *zq, const double *aq, int nq, int w, double *out,
                         hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_deconv, dim3(blocks_for(n, 256, INT32_MAX)), dim3(256), 0, st, xyz, n, chunk_of, ctr,
                       hscale, zq, aq, nq, w, out);
    return hipGetLastError();
}

hipError_t launch_bin(const PairDev *pairs, const int64_t *prefix, int npairs, int64_t total, const double *xyz,
                      int64_t nsrc, int w, int32_t *counts, unsigned long long *cursor, int32_t *records,
                      hipStream_t st)
{
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bin_points, dim3(blocks_for(total, 256, INT32_MAX)), dim3(256), 0, st, pairs, prefix, npairs,
                       total, xyz, nsrc, w, counts, cursor, records);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prephase(const PairDev *pairs, const int64_t *pprefix, int npairs, int64_t total, const double *xyz,
                           int64_t nsrc, const int32_t *perm, const void *in, int64_t in_stride, int rows, void *stage,
                           void *xval, int64_t xstride, double iota, int w, hipStream_t st)
{
    if (total <= 0) return hipSuccess;
    if (rows < 1 || rows > kRowBatch) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_prephase<T>, dim3(blocks_for(total, 256, INT32_MAX)), dim3(256), 0, st, pairs, pprefix,
                       npairs, total, xyz, nsrc, perm, static_cast<const cplx<T> *>(in), in_stride, rows,
                       static_cast<StagedSrc<T> *>(stage), static_cast<cplx<T> *>(xval), xstride, iota, w);
    return hipGetLastError();
}

template <typename T, int NR>
static void spread_rows(const PairDev *pairs, const SpreadTile *tiles, int64_t ntiles, const int32_t *records,
                        const void *stage, const void *xval, int64_t xstride, void *ws, int64_t ws_stride, int w,
                        double beta, hipStream_t st)
{
    hipLaunchKernelGGL((k_spread<T, NR>), dim3(static_cast<unsigned>(ntiles)), dim3(256), 0, st, pairs, tiles, records,
                       static_cast<const StagedSrc<T> *>(stage), static_cast<const cplx<T> *>(xval), xstride,
                       static_cast<cplx<T> *>(ws), ws_stride, w, T(beta), T(2.0 / w),
                       1.0f / static_cast<float>(2 * w + kTileZ));
}

template <typename T>
hipError_t launch_spread(const PairDev *pairs, const SpreadTile *tiles, int64_t ntiles, const int32_t *records,
                         const void *stage, const void *xval, int64_t xstride, int rows, void *ws, int64_t ws_stride,
                         int w, double beta, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    switch (rows) {
    case 1: spread_rows<T, 1>(pairs, tiles, ntiles, records, stage, xval, xstride, ws, ws_stride, w, beta, st); break;
    case 2: spread_rows<T, 2>(pairs, tiles, ntiles, records, stage, xval, xstride, ws, ws_stride, w, beta, st); break;
    case 3: spread_rows<T, 3>(pairs, tiles, ntiles, records, stage, xval, xstride, ws, ws_stride, w, beta, st); break;
    case 4: spread_rows<T, 4>(pairs, tiles, ntiles, records, stage, xval, xstride, ws, ws_stride, w, beta, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fft(const PairDev *pairs, const int64_t *prefix, int npairs, int64_t tiles, int pass, void *ws,
                      const void *tw, const void *precor, const uint32_t *occ, int lds_elems, int max_len, double sign,
                      int rows, int64_t ws_stride, hipStream_t st)
{
    if (tiles <= 0) return hipSuccess;
    if (rows < 1 || rows > kRowBatch) return hipErrorInvalidValue;
    // dynamic LDS: the lines of one workgroup, then the twiddle table of the longest line
    size_t lds = static_cast<size_t>(lds_elems + max_len) * sizeof(cplx<T>);
    const T *pc = static_cast<const T *>(precor);
    const dim3 grid(static_cast<unsigned>(tiles), static_cast<unsigned>(rows));
    // workgroup size from the longest line of the batch (lines up to kFftSmallLen: 256 threads)
    if (fft_threads(max_len) == kFftThreadsSmall)
        hipLaunchKernelGGL((k_fft_pass<T, kFftThreadsSmall>), grid, dim3(kFftThreadsSmall), lds, st, pairs, prefix,
                           npairs, pass, static_cast<cplx<T> *>(ws), static_cast<const cplx<T> *>(tw), pc, occ,
                           lds_elems, T(sign), ws_stride);
    else
        hipLaunchKernelGGL((k_fft_pass<T, kFftThreads>), grid, dim3(kFftThreads), lds, st, pairs, prefix, npairs, pass,
                           static_cast<cplx<T> *>(ws), static_cast<const cplx<T> *>(tw), pc, occ, lds_elems, T(sign),
                           ws_stride);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_transpose(const PairDev *pairs, const int64_t *prefix, int npairs, int64_t tiles, void *ws,
                            int rows, int64_t ws_stride, hipStream_t st)
{
    if (tiles <= 0) return hipSuccess;
    if (rows < 1 || rows > kRowBatch) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_transpose<T>, dim3(static_cast<unsigned>(tiles), static_cast<unsigned>(rows)), dim3(256), 0,
                       st, pairs, prefix, npairs, static_cast<cplx<T> *>(ws), ws_stride);
    return hipGetLastError();
}

template <typename T, int NR>
static hipError_t interp_rows(const PairDev *pairs, const int64_t *bprefix, int npairs, int64_t blocks,
                              const double *xyz, int64_t ntgt, const double *deconv, const void *ws,
                              int64_t ws_stride, double *acc, int64_t acc_stride, int w, double beta, double iota,
                              int det, hipStream_t st)
{
    for (int64_t b0 = 0; b0 < blocks; b0 += kMaxLaunchBlocks) {
        const int64_t nb = std::min<int64_t>(kMaxLaunchBlocks, blocks - b0);
        hipLaunchKernelGGL((k_interp<T, NR>), dim3(static_cast<unsigned>(nb)), dim3(256), 0, st, pairs, bprefix,
                           npairs, b0, xyz, ntgt, deconv, static_cast<const cplx<T> *>(ws), ws_stride, acc,
                           acc_stride, w, T(beta), iota, det);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T>
hipError_t launch_interp(const PairDev *pairs, const int64_t *bprefix, int npairs, int64_t blocks, const double *xyz,
                         int64_t ntgt, const double *deconv, const void *ws, int64_t ws_stride, double *acc,
                         int64_t acc_stride, int rows, int w, double beta, double iota, int det, hipStream_t st)
{
    if (blocks <= 0) return hipSuccess;
    switch (rows) {
    case 1: return interp_rows<T, 1>(pairs, bprefix, npairs, blocks, xyz, ntgt, deconv, ws, ws_stride, acc,
                                     acc_stride, w, beta, iota, det, st);
    case 2: return interp_rows<T, 2>(pairs, bprefix, npairs, blocks, xyz, ntgt, deconv, ws, ws_stride, acc,
                                     acc_stride, w, beta, iota, det, st);
    case 3: return interp_rows<T, 3>(pairs, bprefix, npairs, blocks, xyz, ntgt, deconv, ws, ws_stride, acc,
                                     acc_stride, w, beta, iota, det, st);
    case 4: return interp_rows<T, 4>(pairs, bprefix, npairs, blocks, xyz, ntgt, deconv, ws, ws_stride, acc,
                                     acc_stride, w, beta, iota, det, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, int NT>
static hipError_t launch_direct_rows(const DirectItem *items, int64_t nitems, const double *sxyz, int64_t nsrc,
                                     const double *txyz, int64_t ntgt, const int32_t *perm, const void *in,
                                     int64_t in_stride, double *acc, int64_t acc_stride, double iota, int det,
                                     int64_t grid_cap, const void *ctab, hipStream_t st)
{
    const double2 *tab = static_cast<const double2 *>(ctab);
    if (grid_cap > 0) {
        // persistent: at most grid_cap workgroups looping over the items
        const int64_t nb = std::min<int64_t>(std::min<int64_t>(grid_cap, nitems), kMaxLaunchBlocks);
        hipLaunchKernelGGL((k_direct<T, NT>), dim3(static_cast<unsigned>(nb)), dim3(kDirectThreads), 0, st, items,
                           nitems, sxyz, nsrc, txyz, ntgt, perm, static_cast<const cplx<T> *>(in), in_stride, acc,
                           acc_stride, iota, det, tab);
        return hipGetLastError();
    }
    // one workgroup per item, in launches of at most kMaxLaunchBlocks workgroups
    // (a dispatch counts its work-items in 32 bits)
    for (int64_t i0 = 0; i0 < nitems; i0 += kMaxLaunchBlocks) {
        const int64_t nb = std::min<int64_t>(kMaxLaunchBlocks, nitems - i0);
        hipLaunchKernelGGL((k_direct<T, NT>), dim3(static_cast<unsigned>(nb)), dim3(kDirectThreads), 0, st,
                           items + i0, nb, sxyz, nsrc, txyz, ntgt, perm, static_cast<const cplx<T> *>(in), in_stride,
                           acc, acc_stride, iota, det, tab);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T>
hipError_t launch_direct(const DirectItem *items, int64_t nitems, const double *sxyz, int64_t nsrc,
                         const double *txyz, int64_t ntgt, const int32_t *perm, const void *in, int64_t in_stride,
                         double *acc, int64_t acc_stride, int rows, double iota, int det, int64_t grid_cap,
                         const void *ctab, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    if (sizeof(T) == 8 && ctab == nullptr) return hipErrorInvalidValue;   // float64: the phase table
    switch (rows) {
    case 1: return launch_direct_rows<T, 1>(items, nitems, sxyz, nsrc, txyz, ntgt, perm, in, in_stride, acc,
                                            acc_stride, iota, det, grid_cap, ctab, st);
    case 2: return launch_direct_rows<T, 2>(items, nitems, sxyz, nsrc, txyz, ntgt, perm, in, in_stride, acc,
                                            acc_stride, iota, det, grid_cap, ctab, st);
    case 3: return launch_direct_rows<T, 3>(items, nitems, sxyz, nsrc, txyz, ntgt, perm, in, in_stride, acc,
                                            acc_stride, iota, det, grid_cap, ctab, st);
    case 4: return launch_direct_rows<T, 4>(items, nitems, sxyz, nsrc, txyz, ntgt, perm, in, in_stride, acc,
                                            acc_stride, iota, det, grid_cap, ctab, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_finalize(const double *acc, int64_t n, const int32_t *perm, void *out, int real_only,
                           hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize<T>, dim3(blocks_for(n, 256, INT32_MAX)), dim3(256), 0, st, acc, n, perm,
                       static_cast<cplx<T> *>(out), real_only);
    return hipGetLastError();
}

template hipError_t launch_prephase<float>(const PairDev *, const int64_t *, int, int64_t, const double *, int64_t,
                                           const int32_t *, const void *, int64_t, int, void *, void *, int64_t, double,
                                           int, hipStream_t);
template hipError_t launch_prephase<double>(const PairDev *, const int64_t *, int, int64_t, const double *, int64_t,
                                            const int32_t *, const void *, int64_t, int, void *, void *, int64_t,
                                            double, int, hipStream_t);
template hipError_t launch_spread<float>(const PairDev *, const SpreadTile *, int64_t, const int32_t *, const void *,
                                         const void *, int64_t, int, void *, int64_t, int, double, hipStream_t);
template hipError_t launch_spread<double>(const PairDev *, const SpreadTile *, int64_t, const int32_t *, const void *,
                                          const void *, int64_t, int, void *, int64_t, int, double, hipStream_t);
template hipError_t launch_fft<float>(const PairDev *, const int64_t *, int, int64_t, int, void *, const void *,
                                      const void *, const uint32_t *, int, int, double, int, int64_t, hipStream_t);
template hipError_t launch_fft<double>(const PairDev *, const int64_t *, int, int64_t, int, void *, const void *,
                                       const void *, const uint32_t *, int, int, double, int, int64_t, hipStream_t);
template hipError_t launch_transpose<float>(const PairDev *, const int64_t *, int, int64_t, void *, int, int64_t,
                                            hipStream_t);
template hipError_t launch_transpose<double>(const PairDev *, const int64_t *, int, int64_t, void *, int, int64_t,
                                             hipStream_t);
template hipError_t launch_interp<float>(const PairDev *, const int64_t *, int, int64_t, const double *, int64_t,
                                         const double *, const void *, int64_t, double *, int64_t, int, int, double,
                                         double, int, hipStream_t);
template hipError_t launch_interp<double>(const PairDev *, const int64_t *, int, int64_t, const double *, int64_t,
                                          const double *, const void *, int64_t, double *, int64_t, int, int, double,
                                          double, int, hipStream_t);
template hipError_t launch_direct<float>(const DirectItem *, int64_t, const double *, int64_t, const double *, int64_t,
                                         const int32_t *, const void *, int64_t, double *, int64_t, int, double, int,
                                         int64_t, const void *, hipStream_t);
template hipError_t launch_direct<double>(const DirectItem *, int64_t, const double *, int64_t, const double *, int64_t,
                                          const int32_t *, const void *, int64_t, double *, int64_t, int, double, int,
                                          int64_t, const void *, hipStream_t);
template <typename T>
hipError_t launch_dde_scale(const void *w, const void *x, void *out, int64_t n, int terms, int conj_w, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_dde_scale<T>, dim3(blocks_for(n, 256, INT32_MAX)), dim3(256), 0, st,
                       static_cast<const cplx<T> *>(w), static_cast<const cplx<T> *>(x), static_cast<cplx<T> *>(out), n,
                       terms, conj_w);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_dde_combine(const void *w, const void *y, void *out, int64_t n, int terms, int conj_w, int real_only,
                              hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_dde_combine<T>, dim3(blocks_for(n, 256, INT32_MAX)), dim3(256), 0, st,
                       static_cast<const cplx<T> *>(w), static_cast<const cplx<T> *>(y), static_cast<cplx<T> *>(out), n,
                       terms, conj_w, real_only);
    return hipGetLastError();
}

template hipError_t launch_dde_scale<float>(const void *, const void *, void *, int64_t, int, int, hipStream_t);
template hipError_t launch_dde_scale<double>(const void *, const void *, void *, int64_t, int, int, hipStream_t);
template hipError_t launch_dde_combine<float>(const void *, const void *, void *, int64_t, int, int, int, hipStream_t);
template hipError_t launch_dde_combine<double>(const void *, const void *, void *, int64_t, int, int, int,
                                               hipStream_t);
template hipError_t launch_finalize<float>(const double *, int64_t, const int32_t *, void *, int, hipStream_t);
template hipError_t launch_finalize<double>(const double *, int64_t, const int32_t *, void *, int, hipStream_t);

}  // namespace hvox
