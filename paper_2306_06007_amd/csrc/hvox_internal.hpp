// Internal definitions shared by the host planner, the executor and the HIP
// kernels of the HVOX library.  Not part of the public ABI (include/hvox.h).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hvox.h"

namespace hvox {

// ---- compile-time limits -------------------------------------------------
constexpr int kWMax = 24;            // largest kernel support handled by the kernels
constexpr int kFftThreads = 512;     // threads of an FFT workgroup for lines longer than kFftSmallLen
constexpr int kFftThreadsSmall = 256;   // threads of an FFT workgroup when every line is <= kFftSmallLen
constexpr int kFftSmallLen = 2048;
constexpr int kTransposeTile = 32;   // square tile of the transpose kernel
constexpr int kFftElems = 4096;      // complex elements (lines x length) held in LDS by one workgroup (at most)
// elements of a workgroup of nt threads (eight per thread), and the workgroup
// size and lines per workgroup used for an FFT length n
constexpr int fft_elems(int nt) { return 8 * nt; }
constexpr int fft_threads(int n) { return n <= kFftSmallLen ? kFftThreadsSmall : kFftThreads; }
constexpr int kFftMaxLen = 4096;     // longest 1D FFT (one line must fit a workgroup)
constexpr int kFftMaxLines = 64;     // lines per FFT workgroup
constexpr int fft_lines(int n)
{
    return n >= fft_elems(fft_threads(n)) ? 1 : (fft_elems(fft_threads(n)) / n < kFftMaxLines ? fft_elems(fft_threads(n)) / n : kFftMaxLines);
}
// lines of an FFT workgroup sit in LDS one element apart (line stride n + 1):
// lines loaded across lanes (the z pass) and even lengths would otherwise map
// every lane of an access to one or two banks
constexpr int fft_lds_stride(int n) { return n + 1; }
constexpr int fft_lds_elems(int lines, int n) { return lines * fft_lds_stride(n); }
constexpr int kDirectThreads = 256;  // threads of a direct-sum workgroup
constexpr int kDirectTile = 512;     // targets per direct-sum workgroup (two per thread)
constexpr int kDirectSrcTile = 256;  // sources staged in LDS at a time
constexpr int kDirectSeg = 8192;     // longest source segment of a direct-sum work item
constexpr int64_t kDirectMinItems = 4096;   // shorter segments while a plan has fewer direct work items
constexpr int kDirectWgPerCu = 8;    // direct-sum workgroups per CU while NUFFT work runs beside it
constexpr int kCisTab = 1024;        // entries exp(2 pi i k / kCisTab) of the float64 direct sum's phase table
constexpr int kRowBatch = 4;         // data rows (ntrans) per direct-sum launch, most per NUFFT pass, accumulator rows
constexpr int kInterpLanes = 16;     // interp: lanes per target
constexpr int kInterpTargets = 256 / kInterpLanes;   // interp: targets per 256-thread workgroup
constexpr int kMaxStages = 16;       // radix stages per FFT length
// workgroups per launch of the kernels whose grid grows with the problem (direct,
// interp): a dispatch counts its work-items in 32 bits
constexpr int64_t kMaxLaunchBlocks = int64_t(1) << 22;
// occupancy words of a tile row staged per FFT line: a row of at most
// kFftMaxLen / kTileX tiles starting at any bit
constexpr int kOccWords = (kFftMaxLen / 32 + 31) / 32 + 1;
// spreading by grid-1 tile: one 256-thread workgroup per tile of
// kTileX x kTileY x kTileZ cells, a column of kTileZ cells per thread; points
// touching the tile are staged kSpreadBatch at a time
constexpr int kTileX = 32, kTileY = 8, kTileZ = 8;
constexpr int kSpreadBatch = 64;
// sources of one batch of sub-problems (bounds the staging buffer; staged
// indices fit 32 bits)
constexpr int64_t kMaxBatchPts = int64_t(1) << 25;

// A source of a NUFFT sub-problem as the pre-phase pass leaves it for the
// spreading kernel: the pre-phased value, and the footprint of its kernel on
// grid 1 (first cell c0 per dimension and the offset frac = (c0 - n1/2) - t of
// that cell from the source's grid-1 coordinate t, in the plan's precision).
template <typename T>
struct alignas(16) StagedSrc {
    T v[2];
    T frac[3];
    int32_t c0[3];
};
static_assert(sizeof(StagedSrc<float>) == 32 && sizeof(StagedSrc<double>) == 64, "staged source layout");

// ---- one type-3 sub-problem (source chunk -> target chunk) on the device ---
// FFT passes: x reads grid 1 (contiguous lines) and writes its kept window
// line-major; a tiled transpose makes the y lines contiguous; y writes
// line-major; z reads its (short) lines strided, consecutive lines in
// adjacent lanes, and writes line-major, leaving a z-fastest grid.
// Sub-problem math (Sect. 3, the four type-3 steps; centring as in the
// published type-3 method the paper builds on):
//   f_k = e^{2 pi i iota s_k.x_c} sum_n [c_n e^{2 pi i iota s_c.x'_n}] e^{2 pi i iota s'_k.x'_n}
// with x' = x - x_c, s' = s - s_c.  Sources spread on grid 1 at
// t = x' * kscale (kscale = 2 sigma S, S = target half-width), grid 1 is
// pre-corrected and FFT'd on the upsampled grid 2, targets interpolate at
// tau = s' * tscale (tscale = n2 / (2 sigma S)) and are deconvolved.
struct PairDev {
    int64_t src_off, src_cnt;    // chunk-order range of the sources
    int64_t tgt_off, tgt_cnt;    // chunk-order range of the targets
    double xc[3];                // source chunk centre
    double sc[3];                // target chunk centre
    double kscale[3];            // grid-1 coordinate scale of the sources
    double tscale[3];            // grid-2 coordinate scale of the targets
    int32_t n1[3];               // grid-1 size (modes -n1/2 .. n1/2-1)
    int32_t n2[3];               // grid-2 (FFT) size
    int32_t wstart[3];           // first kept FFT output index (may be negative: periodic)
    int32_t wcount[3];           // kept FFT outputs per dimension
    int32_t nrad[3];             // radix stages per dimension
    int32_t lines_per_tile[3];   // FFT lines per workgroup, per pass
    int64_t bufG, bufA, bufB;    // complex-element offsets of the grid buffers in the workspace:
                                 //   G: grid 1 [n1z][n1y][n1x] (spread output, x-pass input)
                                 //   A: x-pass output transposed [n1z][wx][n1y] -> z-pass output
                                 //      [wx][wy][wz] (read by the interpolation)
                                 //   B: x-pass output [n1z][n1y][wx] -> y-pass output [n1z][wx][wy]
    int64_t tile0;               // index of the pair's first grid-1 tile among the direction's tiles
    int32_t ntile[3];            // grid-1 tiles per dimension
    int32_t pad_;
    int64_t precor[3];           // offsets into the pre-correction table (n1[d] entries each)
    int64_t tw[3];               // offsets into the twiddle table (n2[d] entries each)
    uint8_t radix[3][kMaxStages];
};

// ---- one grid-1 tile of a batch handed to the spreading kernel ------------
// Plan-time descriptor: a single load gives the workgroup its sub-problem,
// its cells and its source list.
struct SpreadTile {
    int64_t r0;                  // first of the tile's records (source indices) in the direction's list
    int32_t cnt;                 // records of the tile (of this part of it, see flags)
    int32_t pair;                // sub-problem, as an index into its batch's pairs
    int16_t org[3];              // grid-1 cell of the tile's first corner
    int16_t flags;               // kSpreadAdd: a further part of a crowded tile (adds atomically)
};
constexpr int16_t kSpreadAdd = 1;
// a tile with more sources is split into parts of at most this many, one
// workgroup each: the first stores, the others add on top in a later launch
// (dense sub-problems would otherwise leave most CUs idle behind a few long tiles)
constexpr int32_t kSpreadSplit = 256;
static_assert(sizeof(SpreadTile) == 24, "spreading tile descriptor layout");
static_assert(kFftMaxLen < 32768, "tile corners are stored in 16 bits");

// ---- direct-sum work item: <= kDirectTile targets x <= kDirectSeg sources --
struct DirectItem {
    int64_t tgt_off;             // chunk-order index of the first target
    int64_t src_off;             // chunk-order index of the first source
    int32_t tgt_cnt;
    int32_t src_cnt;
};

// ---- host-side plan pieces -------------------------------------------------
struct ChunkSet {
    int64_t n = 0;
    int32_t nc = 0;
    std::vector<int32_t> label;      // [n] chunk id of each user-order point
    std::vector<int32_t> perm;       // [n] user index of each chunk-order point
    std::vector<int64_t> off;        // [nc + 1] chunk start in chunk order
    std::vector<double> lo, hi;      // [nc * 3] tight boxes
    std::vector<double> ctr, half;   // [nc * 3] centres and half-widths
};

struct Batch {
    int64_t pair0 = 0, npairs = 0;       // range in the direction's PairDev array
    int64_t pts = 0, tgts = 0;           // spread points, interp targets
    int64_t iblocks = 0;                 // interp workgroups (kInterpTargets targets of one pair each)
    int64_t tiles[3] = {0, 0, 0};        // FFT workgroups per pass
    int64_t stiles = 0;                  // spreading tiles (workgroups)
    int64_t pre_stiles = 0;              // offset of the batch's tile prefix array
    int64_t ttiles = 0;                  // transpose tiles (workgroups)
    int64_t g_cnt = 0;                   // complex elements of the batch's grid-1 region (starts at 0)
    int64_t list_off = 0, list_cnt = 0;  // the batch's spreading tiles (those holding sources) in the
                                         //   direction's descriptor list
    int64_t pre_ttiles = 0;              // offset of the batch's transpose-tile prefix array
    int64_t ws_end = 0;                  // end of the batch's workspace use (complex elements)
    int64_t pre_pts = 0, pre_tgts = 0;   // offsets into the prefix arrays (pre_tgts: interp workgroups)
    int64_t pre_tiles[3] = {0, 0, 0};
    int32_t lds_elems[3] = {0, 0, 0};    // largest LDS need per pass (complex elements)
    int32_t max_pass_len[3] = {0, 0, 0};
};

struct DirPlan {                         // one direction (synthesis or analysis)
    std::vector<PairDev> pairs;          // NUFFT sub-problems, batch-contiguous
    std::vector<Batch> batches;
    std::vector<int64_t> pre_pts, pre_tgts, pre_tiles[3];   // per batch: npairs+1 prefix sums (points,
                                                            // interp workgroups, FFT workgroups)
    std::vector<int64_t> pre_stiles;     // per batch: npairs+1 prefix sums of spreading tiles
    std::vector<int64_t> pre_ttiles;     // per batch: npairs+1 prefix sums of transpose tiles
    int64_t tiles_total = 0;             // spreading tiles over all batches
    // one bit per grid-1 tile (index tile0 + local tile): set when the tile holds sources.
    // Only those tiles are spread; the x pass reads the others as zeros.
    std::vector<uint32_t> occ_bits;
    std::vector<SpreadTile> spread_tiles;   // spreading tiles of every batch (built with the binning)
    std::vector<DirectItem> direct;
    // direct items in launch order: [direct_layer_off[l], direct_layer_off[l + 1]) is launch l.
    // One launch of every item unless the plan is deterministic: then layer l holds the l-th
    // source segment of every target tile, so the items of a launch never share a target and
    // add into the accumulator without atomics, layer after layer.
    std::vector<int64_t> direct_layer_off;
    double grid_cells = 0.0, direct_terms = 0.0;
    int64_t occ_tiles[2] = {0, 0}, occ_xlines[2] = {0, 0}, occ_zplanes[2] = {0, 0};   // filled by the binning
    double est_seconds = 0.0;
    double est_direct_seconds = 0.0;     // the direct sub-problems' share of est_seconds
    double alg_bytes[HVOX_K_COUNT] = {0};
    double alg_flops[HVOX_K_COUNT] = {0};
};

struct Params {
    int dtype = HVOX_F32;
    double eps = 1e-4;
    double eps_sub = 0.0;          // accuracy each sub-problem's kernels are sized for (0: eps)
    double sigma = 1.25;           // upsampling of the spreading stage (grid 1 vs the Heisenberg box)
    int w = 8;                     // spreading kernel support (grid-1 cells)
    double beta = 0.0;
    double sigma_opt = 0.0;        // caller's spreading upsampling (0: automatic)
    double sigma2_opt = 0.0;       // caller's inner-FFT upsampling (0: automatic)
    double sigma2 = 1.25;          // upsampling of the inner FFT stage (grid 2 vs grid 1)
    int w2 = 8;                    // interpolation kernel support (grid-2 cells)
    double beta2 = 0.0;
    bool all_direct = false;
    double direct_threshold = -1.0;
    int ntrans_hint = 1;           // rows per call the cost model weighs
    double max_fft_bytes = 500e6;
    double alpha = 1.0;
    double ws_cap = 4.0 * 1024 * 1024 * 1024;
    int flags = 0;
    bool deterministic() const { return (flags & HVOX_DETERMINISTIC) != 0; }
};

struct HostPlan {
    Params prm;
    int64_t n_vis = 0, n_pix = 0;
    std::vector<double> uvw, xyz;        // user order, [n][3]
    ChunkSet vis, sky;
    double h[3] = {0, 0, 0}, eta[3] = {0, 0, 0};
    DirPlan syn, ana;                    // syn: sky -> vis (iota = -1); ana: vis -> sky (iota = +1)
    int64_t ws_elems = 0;                // workspace size (complex elements): rows copies of ws_row
    int64_t max_pair_ws = 0;
    // data rows per NUFFT pass (the ntrans rows of Sect. 4, at most kRowBatch, from the
    // caller's ntrans hint): the rows of a pass share the spreading and interpolation
    // weights, and each takes its own copy of the batch workspace, ws_row elements apart
    int rows = 1;
    int64_t ws_row = 0;
    int64_t max_pts = 0;                 // spread points of the largest batch
    // unique FFT-length tables: (n1, n2) pre-correction tables and n2 twiddles
    std::vector<double> precor_nu;       // nu = l / n2 of every pre-correction entry
    std::vector<int32_t> tw_len;         // lengths with a twiddle table
    std::vector<int64_t> tw_off;         // offsets (complex elements) of each table
    int64_t tw_total = 0;
    // deconvolution: per chunk S_eff (target scale) for each direction
    std::vector<double> syn_tgt_scale;   // [n_vis_chunks * 3]: 1 / (2 sigma S_eff) for vis targets
    std::vector<double> ana_tgt_scale;   // [n_sky_chunks * 3]
};

// ---- planner entry points (planner.cpp, host only) ------------------------
int es_params(double eps, double sigma, int *w, double *beta);
int choose_kernels(Params *p, double eps_sub);
int alg1(const double B[3], const double P[3], double v_max, double alpha, double h[3], double eta[3]);
int64_t partition(const double *x, int64_t n, const double h[3], int32_t *labels);
int make_host_plan(const double *uvw, int64_t n_vis, const double *xyz, int64_t n_pix,
                   const Params &prm, const int32_t *vis_chunk, const int32_t *sky_chunk,
                   HostPlan *hp, std::string *err);
int32_t smooth_even(int64_t n);
// bytes of the staged sources of one batch: the footprint records (with row 0's
// values), rounded up to 256 bytes, then the values of rows 1 .. rows-1
inline void stage_layout(const HostPlan &hp, int64_t *rec_bytes, int64_t *val_bytes)
{
    const bool f64 = hp.prm.dtype == HVOX_F64;
    const int64_t rec = (f64 ? sizeof(StagedSrc<double>) : sizeof(StagedSrc<float>)) * hp.max_pts;
    *rec_bytes = (rec + 255) / 256 * 256;
    *val_bytes = (f64 ? 16 : 8) * static_cast<int64_t>(hp.rows - 1) * hp.max_pts;
}

// upper bound of the device bytes of a plan (resident tables + workspace), from the host plan
int64_t device_bytes_bound(const HostPlan &hp);
// complex elements a single sub-problem region may hold: kernels index within one
// region in 32-bit arithmetic
constexpr int64_t kMaxRegionElems = (int64_t(1) << 31) - 1;
int factor_radices(int32_t n, uint8_t *radix);
void gauss_legendre(int n, std::vector<double> *x, std::vector<double> *w);

}  // namespace hvox
