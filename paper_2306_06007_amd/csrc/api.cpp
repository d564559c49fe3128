// C ABI of the HVOX library (include/hvox.h): plan creation (host planner +
// device uploads), the stream-ordered executor of synthesis / analysis, and
// per-kernel HIP-event statistics.  No exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "hvox_internal.hpp"

namespace hvox {

hipError_t launch_zero(double *p, int64_t n, hipStream_t st);
hipError_t launch_deconv(const double *xyz, int64_t n, const int32_t *chunk_of, const double *ctr,
                         const double *hscale, const double *zq, const double *aq, int nq, int w, double *out,
                         hipStream_t st);
hipError_t launch_bin(const PairDev *pairs, const int64_t *prefix, int npairs, int64_t total, const double *xyz,
                      int64_t nsrc, int w, int32_t *counts, unsigned long long *cursor, int32_t *records,
                      hipStream_t st);
template <typename T>
hipError_t launch_prephase(const PairDev *, const int64_t *, int, int64_t, const double *, int64_t, const int32_t *,
                           const void *, int64_t, int, void *, void *, int64_t, double, int, hipStream_t);
template <typename T>
hipError_t launch_spread(const PairDev *, const SpreadTile *, int64_t, const int32_t *, const void *, const void *,
                         int64_t, int, void *, int64_t, int, double, hipStream_t);
template <typename T>
hipError_t launch_fft(const PairDev *, const int64_t *, int, int64_t, int, void *, const void *, const void *,
                      const uint32_t *, int, int, double, int, int64_t, hipStream_t);
template <typename T>
hipError_t launch_transpose(const PairDev *, const int64_t *, int, int64_t, void *, int, int64_t, hipStream_t);
template <typename T>
hipError_t launch_interp(const PairDev *, const int64_t *, int, int64_t, const double *, int64_t, const double *,
                         const void *, int64_t, double *, int64_t, int, int, double, double, int, hipStream_t);
template <typename T>
hipError_t launch_direct(const DirectItem *, int64_t, const double *, int64_t, const double *, int64_t,
                         const int32_t *, const void *, int64_t, double *, int64_t, int, double, int, int64_t,
                         const void *, hipStream_t);
template <typename T>
hipError_t launch_finalize(const double *, int64_t, const int32_t *, void *, int, hipStream_t);
template <typename T>
hipError_t launch_dde_scale(const void *, const void *, void *, int64_t, int, int, hipStream_t);
template <typename T>
hipError_t launch_dde_combine(const void *, const void *, void *, int64_t, int, int, int, hipStream_t);

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

struct DevDir {
    PairDev *pairs = nullptr;
    int64_t *pre_pts = nullptr, *pre_tgts = nullptr, *pre_tiles[3] = {nullptr, nullptr, nullptr};
    DirectItem *direct = nullptr;
    double *deconv = nullptr;        // per chunk-order target
    int64_t *pre_ttiles = nullptr;   // per batch: transpose-tile prefix over its pairs
    int32_t *records = nullptr;      // source indices listed per tile (plan-resident binning)
    SpreadTile *spread_tiles = nullptr;   // spreading tiles of every batch (descriptor per workgroup)
    uint32_t *occ = nullptr;         // one bit per grid-1 tile: holds sources (read by the x pass)
    // per batch: descriptors of the further parts of crowded tiles, after the batch's
    // list_cnt first parts (a second launch adds them once the first has stored)
    std::vector<int64_t> spread_add_cnt;
};

struct TimedLaunch {
    int kind;
    hipEvent_t a, b;
};

}  // namespace
}  // namespace hvox

struct hvox_plan_s {
    hvox::HostPlan hp;
    bool host_only = false;
    int device = 0;
    size_t resident_bytes = 0;
    size_t device_bytes = 0;                            // every live device block of the plan
    std::vector<std::pair<void *, size_t>> allocations;
    hvox_alloc_fn alloc_hook = nullptr;                 // caller's device-memory hooks (or NULL)
    hvox_free_fn free_hook = nullptr;
    void *alloc_ctx = nullptr;
    double oom_limit = -1.0;                            // HVOX_FORCE_OOM_BYTES at plan creation (< 0: none)
    size_t alloc_peak = 0;                              // device bytes obtained so far (incl. temporaries)
    double *vis_xyz = nullptr, *sky_xyz = nullptr;     // SoA [3][n], chunk order
    int32_t *vis_perm = nullptr, *sky_perm = nullptr;
    void *precor = nullptr;                             // pre-correction tables in the plan's precision
    void *tw = nullptr;
    void *cis_tab = nullptr;                            // float64 plans: exp(2 pi i k / kCisTab), the direct sum's table
    hvox::DevDir syn, ana;
    void *ws = nullptr;
    void *stage = nullptr;                              // staged sources of one batch (value and footprint)
    double *acc = nullptr;
    hipStream_t last_stream = nullptr;
    // a second stream (default priority) the direct sum runs on while the NUFFT
    // batches run on the caller's stream, forked and joined with two events
    hipStream_t side = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    // workgroups of a direct-sum launch beside NUFFT work (persistent grid; 0: one per item)
    int64_t direct_grid_cap = 0;
    double plan_seconds = 0.0;
    // timing
    std::vector<hvox::TimedLaunch> pending;
    std::vector<hipEvent_t> spare_events;
    hvox_stats_t stats{};
};

namespace hvox {
namespace {

// One device block through the caller's hooks or hipMalloc, refused beyond the
// HVOX_FORCE_OOM_BYTES limit (fault injection).  Temporaries are handed back
// with raw_free; plan blocks are listed and released with the plan.
hipError_t raw_alloc(hvox_plan_s *pl, size_t bytes, void **dst, hipStream_t st)
{
    *dst = nullptr;
    if (pl->oom_limit >= 0.0 && static_cast<double>(pl->device_bytes + bytes) > pl->oom_limit)
        return hipErrorOutOfMemory;
    if (pl->alloc_hook) {
        *dst = pl->alloc_hook(bytes, pl->alloc_ctx, st);
        if (!*dst) return hipErrorOutOfMemory;
    } else {
        hipError_t e = hipMalloc(dst, bytes);
        if (e != hipSuccess) { *dst = nullptr; return e; }
    }
    pl->device_bytes += bytes;
    pl->alloc_peak = std::max(pl->alloc_peak, pl->device_bytes);
    return hipSuccess;
}

void raw_free(hvox_plan_s *pl, void *p, size_t bytes, hipStream_t st)
{
    if (!p) return;
    if (pl->free_hook) pl->free_hook(p, bytes, pl->alloc_ctx, st);
    else (void)hipFree(p);
    pl->device_bytes -= bytes;
}

hipError_t dev_alloc(hvox_plan_s *pl, size_t bytes, void **dst, bool resident, hipStream_t st)
{
    *dst = nullptr;
    if (bytes == 0) return hipSuccess;
    hipError_t e = raw_alloc(pl, bytes, dst, st);
    if (e != hipSuccess) return e;
    pl->allocations.emplace_back(*dst, bytes);
    if (resident) pl->resident_bytes += bytes;
    return hipSuccess;
}

template <typename V>
hipError_t upload(hvox_plan_s *pl, const std::vector<V> &v, V **dst, hipStream_t st)
{
    *dst = nullptr;
    if (v.empty()) return hipSuccess;
    void *p = nullptr;
    hipError_t e = dev_alloc(pl, v.size() * sizeof(V), &p, true, st);
    if (e != hipSuccess) return e;
    *dst = static_cast<V *>(p);
    return hipMemcpyAsync(p, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice, st);
}

void release(hvox_plan_s *pl)
{
    if (pl->side) { (void)hipStreamSynchronize(pl->side); (void)hipStreamDestroy(pl->side); pl->side = nullptr; }
    if (pl->fork_ev) { (void)hipEventDestroy(pl->fork_ev); pl->fork_ev = nullptr; }
    if (pl->join_ev) { (void)hipEventDestroy(pl->join_ev); pl->join_ev = nullptr; }
    for (auto &a : pl->allocations) raw_free(pl, a.first, a.second, pl->last_stream);
    pl->allocations.clear();
    pl->resident_bytes = 0;
    for (auto &t : pl->pending) { (void)hipEventDestroy(t.a); (void)hipEventDestroy(t.b); }
    pl->pending.clear();
    for (hipEvent_t e : pl->spare_events) (void)hipEventDestroy(e);
    pl->spare_events.clear();
}

std::vector<double> soa(const std::vector<double> &aos, const std::vector<int32_t> &perm)
{
    const size_t n = perm.size();
    std::vector<double> out(3 * n);
    for (size_t j = 0; j < n; ++j)
        for (int d = 0; d < 3; ++d) out[d * n + j] = aos[3 * static_cast<size_t>(perm[j]) + d];
    return out;
}

std::vector<int32_t> chunk_of_order(const ChunkSet &cs)
{
    std::vector<int32_t> out(cs.n);
    for (int32_t c = 0; c < cs.nc; ++c)
        for (int64_t j = cs.off[c]; j < cs.off[c + 1]; ++j) out[j] = c;
    return out;
}

// ---- timing -----------------------------------------------------------------
hipEvent_t take_event(hvox_plan_s *pl)
{
    if (!pl->spare_events.empty()) {
        hipEvent_t e = pl->spare_events.back();
        pl->spare_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

hipError_t resolve_timing(hvox_plan_s *pl)
{
    for (auto &t : pl->pending) {
        hipError_t e = hipEventSynchronize(t.b);
        if (e != hipSuccess) return e;
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, t.a, t.b);
        if (e != hipSuccess) return e;
        pl->stats.ms[t.kind] += ms;
        pl->spare_events.push_back(t.a);
        pl->spare_events.push_back(t.b);
    }
    pl->pending.clear();
    return hipSuccess;
}

// Launch f(), bracketed by HIP events on st when the plan times its kernels and
// the caller allows it (the allocation-free entry point never creates events).
template <class F>
hipError_t timed(hvox_plan_s *pl, bool may_time, int kind, hipStream_t st, F &&f)
{
    pl->stats.launches[kind] += 1;
    if (!may_time || !(pl->hp.prm.flags & HVOX_TIMING)) return f();
    hipEvent_t a = take_event(pl), b = take_event(pl);
    if (!a || !b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(a, st);
    if (e == hipSuccess) e = f();
    if (e == hipSuccess) e = hipEventRecord(b, st);
    pl->pending.push_back({kind, a, b});
    if (e == hipSuccess && pl->pending.size() >= 2048) e = resolve_timing(pl);
    return e;
}

// Device buffers a transform works in besides its inputs and outputs: the
// grid workspace, the staged sources of one batch, and the float64
// accumulator rows (kRowBatch rows of the larger domain).
struct Scratch {
    void *ws;
    void *stage;
    double *acc;
    void *xval;   // staged values of rows 1 .. rows-1 of a NUFFT pass
};

// ---- executor -----------------------------------------------------------------
// largest estimated direct-sum share of a direction's time at which the overlapped
// direct sum runs on a capped persistent grid (measured on one MI355X: SKA-like cap,
// direct share 0.75, 609 ms capped vs 624 ms uncapped; LOFAR-like wide field, share
// 0.93, 14.39 s capped vs 12.71 s uncapped)
constexpr double kCappedDirectShare = 0.85;
template <typename T>
int run_direction(hvox_plan_s *pl, bool synthesis, const void *in, void *out, int32_t ntrans, hipStream_t st,
                  const Scratch &sc, bool may_time, bool allow_real = true)
{
    const HostPlan &hp = pl->hp;
    const Params &p = hp.prm;
    const DirPlan &dp = synthesis ? hp.syn : hp.ana;
    const DevDir &dd = synthesis ? pl->syn : pl->ana;
    const int64_t n_src = synthesis ? hp.n_pix : hp.n_vis;
    const int64_t n_tgt = synthesis ? hp.n_vis : hp.n_pix;
    const double *sxyz = synthesis ? pl->sky_xyz : pl->vis_xyz;
    const double *txyz = synthesis ? pl->vis_xyz : pl->sky_xyz;
    // data already in chunk order: no gather / scatter through the permutations
    const bool pre = (p.flags & HVOX_PREORDERED) != 0;
    const int32_t *sperm = pre ? nullptr : (synthesis ? pl->sky_perm : pl->vis_perm);
    const int32_t *tperm = pre ? nullptr : (synthesis ? pl->vis_perm : pl->sky_perm);
    const double iota = synthesis ? -1.0 : 1.0;
    const int real_only = (allow_real && !synthesis && (p.flags & HVOX_REAL_SKY)) ? 1 : 0;
    const int det = p.deterministic() ? 1 : 0;
    using C = typename std::conditional<sizeof(T) == 4, float2, double2>::type;
    hipError_t e = hipSuccess;
#define HVOX_TRY(expr)                                                                             \
    do {                                                                                           \
        e = (expr);                                                                                \
        if (e != hipSuccess) return fail(HVOX_ERR_HIP, std::string("HIP: ") + hipGetErrorString(e)); \
    } while (0)

    // the direct blocks run on the plan's second stream, overlapping the NUFFT
    // batches (VALU-bound direct sum beside memory-bound grid passes; both add
    // into the accumulator atomically), unless the plan is deterministic (its
    // direct layers add after the batches, in order) or the call may not
    // create work outside the caller's stream.
    // Calls that time every kernel (HVOX_TIMING) run serialised, so that each
    // kernel's HIP-event time is its own and not a share of the GPU.
    const bool overlap = may_time && !(p.flags & HVOX_TIMING) && !det && pl->side && !dp.batches.empty() &&
                         !dp.direct.empty();
    hipStream_t dst = overlap ? pl->side : st;
    // beside a sizeable NUFFT share the direct sum takes a persistent grid capped per
    // CU, leaving room for the NUFFT kernels; when it is nearly the whole estimated
    // time (wide fields) it takes one workgroup per item, every CU full of its waves
    const double direct_share = dp.est_seconds > 0.0 ? dp.est_direct_seconds / dp.est_seconds : 1.0;
    const int64_t direct_cap = direct_share <= kCappedDirectShare ? pl->direct_grid_cap : 0;
    // rows in groups of up to kRowBatch: the NUFFT sub-problems run in passes of
    // up to hp.rows rows into the group's accumulator rows, the direct sum covers
    // all rows of the group in one launch (its phase factors are shared by the rows)
    for (int32_t t0 = 0; t0 < ntrans; t0 += kRowBatch) {
        const int nb = static_cast<int>(std::min<int32_t>(kRowBatch, ntrans - t0));
        if (n_tgt == 0) continue;
        HVOX_TRY(timed(pl, may_time, HVOX_K_ZERO, st, [&] { return launch_zero(sc.acc, 2 * n_tgt * nb, st); }));
        if (overlap) {
            // fork: the direct sum starts once the accumulator is clear
            HVOX_TRY(hipEventRecord(pl->fork_ev, st));
            HVOX_TRY(hipStreamWaitEvent(pl->side, pl->fork_ev, 0));
            for (size_t l = 0; l + 1 < dp.direct_layer_off.size(); ++l) {
                const int64_t i0 = dp.direct_layer_off[l], i1 = dp.direct_layer_off[l + 1];
                HVOX_TRY(timed(pl, may_time, HVOX_K_DIRECT, dst, [&] {
                    return launch_direct<T>(dd.direct + i0, i1 - i0, sxyz, n_src, txyz, n_tgt, sperm,
                                            static_cast<const C *>(in) + static_cast<int64_t>(t0) * n_src, n_src,
                                            sc.acc, 2 * n_tgt, nb, iota, det, direct_cap, pl->cis_tab, dst);
                }));
            }
            HVOX_TRY(hipEventRecord(pl->join_ev, pl->side));
        }
        // NUFFT sub-problems: passes of up to hp.rows data rows, each pass sharing the
        // spreading and interpolation weights over its rows (row r in the r-th
        // workspace copy and accumulator row)
        for (int r0 = 0; r0 < nb; r0 += hp.rows) {
            const int nr = std::min(hp.rows, nb - r0);
            const C *in_t = static_cast<const C *>(in) + static_cast<int64_t>(t0 + r0) * n_src;
            double *acc_r = sc.acc + 2 * n_tgt * r0;
            for (const Batch &b : dp.batches) {
                const PairDev *pairs = dd.pairs + b.pair0;
                const int np = static_cast<int>(b.npairs);
                const int64_t *pprefix = dd.pre_pts + b.pre_pts;
                HVOX_TRY(timed(pl, may_time, HVOX_K_PREPHASE, st, [&] {
                    return launch_prephase<T>(pairs, pprefix, np, b.pts, sxyz, n_src, sperm, in_t, n_src, nr, sc.stage,
                                              sc.xval, hp.max_pts, iota, p.w, st);
                }));
                HVOX_TRY(timed(pl, may_time, HVOX_K_SPREAD, st, [&] {
                    return launch_spread<T>(pairs, dd.spread_tiles + b.list_off, b.list_cnt, dd.records, sc.stage,
                                            sc.xval, hp.max_pts, nr, sc.ws, hp.ws_row, p.w, p.beta, st);
                }));
                const int64_t n_add = dd.spread_add_cnt[&b - dp.batches.data()];
                if (n_add > 0)
                    HVOX_TRY(timed(pl, may_time, HVOX_K_SPREAD, st, [&] {
                        return launch_spread<T>(pairs, dd.spread_tiles + b.list_off + b.list_cnt, n_add, dd.records,
                                                sc.stage, sc.xval, hp.max_pts, nr, sc.ws, hp.ws_row, p.w, p.beta, st);
                    }));
                for (int pass = 0; pass < 3; ++pass) {
                    HVOX_TRY(timed(pl, may_time, HVOX_K_FFT_X + pass, st, [&] {
                        return launch_fft<T>(pairs, dd.pre_tiles[pass] + b.pre_tiles[pass], np, b.tiles[pass], pass,
                                             sc.ws, pl->tw, pl->precor, dd.occ, b.lds_elems[pass],
                                             b.max_pass_len[pass], iota, nr, hp.ws_row, st);
                    }));
                    if (pass == 0)
                        HVOX_TRY(timed(pl, may_time, HVOX_K_TRANSPOSE, st, [&] {
                            return launch_transpose<T>(pairs, dd.pre_ttiles + b.pre_ttiles, np, b.ttiles, sc.ws, nr,
                                                       hp.ws_row, st);
                        }));
                }
                HVOX_TRY(timed(pl, may_time, HVOX_K_INTERP, st, [&] {
                    return launch_interp<T>(pairs, dd.pre_tgts + b.pre_tgts, np, b.iblocks, txyz, n_tgt, dd.deconv,
                                            sc.ws, hp.ws_row, acc_r, 2 * n_tgt, nr, p.w2, p.beta2, iota, det, st);
                }));
            }
        }
        // direct blocks (unless already on the second stream): one launch, or
        // (deterministic plans) one launch per layer of items that share no
        // target, in a fixed order
        if (overlap) HVOX_TRY(hipStreamWaitEvent(st, pl->join_ev, 0));   // join before the finalize
        else for (size_t l = 0; l + 1 < dp.direct_layer_off.size(); ++l) {
            const int64_t i0 = dp.direct_layer_off[l], i1 = dp.direct_layer_off[l + 1];
            HVOX_TRY(timed(pl, may_time, HVOX_K_DIRECT, st, [&] {
                return launch_direct<T>(dd.direct + i0, i1 - i0, sxyz, n_src, txyz, n_tgt, sperm,
                                        static_cast<const C *>(in) + static_cast<int64_t>(t0) * n_src, n_src, sc.acc,
                                        2 * n_tgt, nb, iota, det, 0, pl->cis_tab, st);
            }));
        }
        for (int r = 0; r < nb; ++r) {
            C *out_t = static_cast<C *>(out) + static_cast<int64_t>(t0 + r) * n_tgt;
            HVOX_TRY(timed(pl, may_time, HVOX_K_FINAL, st, [&] {
                return launch_finalize<T>(sc.acc + 2 * n_tgt * r, n_tgt, tperm, out_t, real_only, st);
            }));
        }
        for (int k = 0; k < HVOX_K_COUNT; ++k) {
            pl->stats.alg_bytes[k] += dp.alg_bytes[k] * nb;
            pl->stats.alg_flops[k] += dp.alg_flops[k] * nb;
        }
    }
#undef HVOX_TRY
    pl->last_stream = st;
    return HVOX_OK;
}

// the plan's own scratch: workspace, staged sources (footprint records, then
// the further rows' values) and accumulator rows
Scratch plan_scratch(const hvox_plan_s *pl)
{
    int64_t rec_b, val_b;
    stage_layout(pl->hp, &rec_b, &val_b);
    void *xval = pl->stage && val_b > 0 ? static_cast<char *>(pl->stage) + rec_b : nullptr;
    return Scratch{pl->ws, pl->stage, pl->acc, xval};
}

int transform(hvox_plan_s *pl, bool synthesis, const void *in, void *out, int32_t ntrans, void *stream)
{
    if (!pl) return fail(HVOX_ERR_STATE, "NULL plan");
    if (pl->host_only) return fail(HVOX_ERR_STATE, "host-only plan cannot run transforms (hvox_plan_upload first)");
    if (ntrans < 1) return fail(HVOX_ERR_ARG, "ntrans must be >= 1");
    const int64_t n_in = synthesis ? pl->hp.n_pix : pl->hp.n_vis;
    const int64_t n_out = synthesis ? pl->hp.n_vis : pl->hp.n_pix;
    if ((n_in > 0 && !in) || (n_out > 0 && !out)) return fail(HVOX_ERR_ARG, "NULL data pointer");
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return fail(HVOX_ERR_HIP, "hipGetDevice failed");
    if (cur != pl->device) return fail(HVOX_ERR_STATE, "the plan's device is not the current device");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Scratch sc = plan_scratch(pl);
    if (pl->hp.prm.dtype == HVOX_F64) return run_direction<double>(pl, synthesis, in, out, ntrans, st, sc, true);
    return run_direction<float>(pl, synthesis, in, out, ntrans, st, sc, true);
}

// Direction-dependent gains A_k(r_n) = sum_t a[t][k] b[t][n]: per data row, the
// n_terms rows of the transform's input (gain-weighted), one transform of
// n_terms rows, and the gain-weighted sum of its output rows.
template <typename T>
int run_dde(hvox_plan_s *pl, bool synthesis, const void *in, void *out, const void *a, const void *b, int32_t terms,
            int32_t ntrans, void *work, hipStream_t st)
{
    const HostPlan &hp = pl->hp;
    const int64_t n_in = synthesis ? hp.n_pix : hp.n_vis, n_out = synthesis ? hp.n_vis : hp.n_pix;
    // synthesis: rows b[t] * sky, combined with a[t]; analysis: rows conj(a[t]) * vis, combined with conj(b[t])
    const void *w_in = synthesis ? b : a, *w_out = synthesis ? a : b;
    const int conj = synthesis ? 0 : 1;
    const int real_only = (!synthesis && (hp.prm.flags & HVOX_REAL_SKY)) ? 1 : 0;
    using C = typename std::conditional<sizeof(T) == 4, float2, double2>::type;
    C *X = static_cast<C *>(work);
    C *Y = X + static_cast<int64_t>(terms) * std::max(hp.n_vis, hp.n_pix);
    const Scratch sc = plan_scratch(pl);
    for (int32_t r = 0; r < ntrans; ++r) {
        const C *x_r = static_cast<const C *>(in) + static_cast<int64_t>(r) * n_in;
        C *y_r = static_cast<C *>(out) + static_cast<int64_t>(r) * n_out;
        hipError_t e = launch_dde_scale<T>(w_in, x_r, X, n_in, terms, conj, st);
        if (e != hipSuccess) return fail(HVOX_ERR_HIP, std::string("HIP: ") + hipGetErrorString(e));
        const int rc = run_direction<T>(pl, synthesis, X, Y, terms, st, sc, true, false);
        if (rc) return rc;
        e = launch_dde_combine<T>(w_out, Y, y_r, n_out, terms, conj, real_only, st);
        if (e != hipSuccess) return fail(HVOX_ERR_HIP, std::string("HIP: ") + hipGetErrorString(e));
    }
    return HVOX_OK;
}

int transform_dde(hvox_plan_s *pl, bool synthesis, const void *in, void *out, const void *a, const void *b,
                  int32_t terms, int32_t ntrans, void *work, void *stream)
{
    if (!pl) return fail(HVOX_ERR_STATE, "NULL plan");
    if (pl->host_only) return fail(HVOX_ERR_STATE, "host-only plan cannot run transforms (hvox_plan_upload first)");
    if (ntrans < 1 || terms < 1) return fail(HVOX_ERR_ARG, "ntrans and n_terms must be >= 1");
    const int64_t n_in = synthesis ? pl->hp.n_pix : pl->hp.n_vis;
    const int64_t n_out = synthesis ? pl->hp.n_vis : pl->hp.n_pix;
    if ((n_in > 0 && !in) || (n_out > 0 && !out)) return fail(HVOX_ERR_ARG, "NULL data pointer");
    if ((pl->hp.n_vis > 0 && !a) || (pl->hp.n_pix > 0 && !b) || !work)
        return fail(HVOX_ERR_ARG, "NULL gain or work pointer");
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return fail(HVOX_ERR_HIP, "hipGetDevice failed");
    if (cur != pl->device) return fail(HVOX_ERR_STATE, "the plan's device is not the current device");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (pl->hp.prm.dtype == HVOX_F64) return run_dde<double>(pl, synthesis, in, out, a, b, terms, ntrans, work, st);
    return run_dde<float>(pl, synthesis, in, out, a, b, terms, ntrans, work, st);
}

int upload_dir(hvox_plan_s *pl, const DirPlan &dp, DevDir *dd, hipStream_t st)
{
    hipError_t e;
    if ((e = upload(pl, dp.pairs, &dd->pairs, st)) != hipSuccess) return HVOX_ERR_OOM;
    if ((e = upload(pl, dp.pre_pts, &dd->pre_pts, st)) != hipSuccess) return HVOX_ERR_OOM;
    if ((e = upload(pl, dp.pre_tgts, &dd->pre_tgts, st)) != hipSuccess) return HVOX_ERR_OOM;
    for (int q = 0; q < 3; ++q)
        if ((e = upload(pl, dp.pre_tiles[q], &dd->pre_tiles[q], st)) != hipSuccess) return HVOX_ERR_OOM;
    if ((e = upload(pl, dp.direct, &dd->direct, st)) != hipSuccess) return HVOX_ERR_OOM;
    if ((e = upload(pl, dp.pre_ttiles, &dd->pre_ttiles, st)) != hipSuccess) return HVOX_ERR_OOM;
    return HVOX_OK;
}

// Plan-time binning of every NUFFT sub-problem's sources to the grid-1 tiles
// their footprints touch (count, host prefix sum, scatter); the per-tile
// lists stay resident and drive the tiled spreading kernel.
int bin_direction(hvox_plan_s *pl, DirPlan &dp, DevDir *dd, const double *sxyz, int64_t n_src, hipStream_t st,
                  std::string *err)
{
    if (dp.tiles_total == 0) return HVOX_OK;
    const int w = pl->hp.prm.w;
    const bool det = pl->hp.prm.deterministic();
    const int64_t nt = dp.tiles_total;
    void *d_counts = nullptr, *d_cursor = nullptr;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(st);
        raw_free(pl, d_counts, sizeof(int32_t) * nt, st);
        raw_free(pl, d_cursor, sizeof(unsigned long long) * nt, st);
        d_counts = d_cursor = nullptr;
    };
    auto bad = [&](hipError_t e, const char *what) {
        cleanup();
        *err = std::string(what) + ": " + hipGetErrorString(e);
        return (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? HVOX_ERR_OOM : HVOX_ERR_HIP;
    };
    hipError_t e = raw_alloc(pl, sizeof(int32_t) * nt, &d_counts, st);
    if (e != hipSuccess) return bad(e, "binning counts");
    e = hipMemsetAsync(d_counts, 0, sizeof(int32_t) * nt, st);
    for (const Batch &b : dp.batches) {
        if (e != hipSuccess) break;
        e = launch_bin(dd->pairs + b.pair0, dd->pre_pts + b.pre_pts, static_cast<int>(b.npairs), b.pts, sxyz, n_src,
                       w, static_cast<int32_t *>(d_counts), nullptr, nullptr, st);
    }
    std::vector<int32_t> counts(nt);
    if (e == hipSuccess) e = hipMemcpyAsync(counts.data(), d_counts, sizeof(int32_t) * nt, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return bad(e, "binning count pass");
    std::vector<int64_t> off(nt + 1, 0);
    for (int64_t i = 0; i < nt; ++i) off[i + 1] = off[i] + counts[i];
    // Only tiles holding sources are spread (each written once, zeros of the cells
    // no footprint reaches included); the x pass reads the other tiles of grid 1
    // as zeros, from the occupancy bitmap, so they are never written or cleared.
    // A crowded tile (more than kSpreadSplit sources) becomes a first part, stored
    // with the batch's other tiles, and further parts that a second launch adds
    // atomically on top -- except in deterministic plans, whose tiles are never split.
    const int32_t split = det ? INT32_MAX : kSpreadSplit;
    dp.spread_tiles.clear();
    dd->spread_add_cnt.assign(dp.batches.size(), 0);
    std::vector<SpreadTile> adds;
    dp.occ_bits.assign(static_cast<size_t>((nt + 31) / 32 + kOccWords), 0u);   // padded: rows are read in whole words
    for (int64_t t = 0; t < nt; ++t)
        if (counts[t] > 0) dp.occ_bits[t >> 5] |= 1u << (t & 31);
    const double delta = pl->hp.prm.dtype == HVOX_F64 ? 16.0 : 8.0;
    for (Batch &b : dp.batches) {
        b.list_off = static_cast<int64_t>(dp.spread_tiles.size());
        adds.clear();
        for (int64_t i = 0; i < b.npairs; ++i) {
            const PairDev &pd = dp.pairs[b.pair0 + i];
            // occupancy statistics: tiles with sources, x lines and z planes they cover
            for (int32_t tz = 0; tz < pd.ntile[2]; ++tz) {
                bool layer = false;
                for (int32_t ty = 0; ty < pd.ntile[1]; ++ty) {
                    bool row = false;
                    for (int32_t tx = 0; tx < pd.ntile[0]; ++tx) {
                        const bool occ = counts[pd.tile0 + (static_cast<int64_t>(tz) * pd.ntile[1] + ty) * pd.ntile[0] + tx] > 0;
                        dp.occ_tiles[0] += occ;
                        row = row || occ;
                    }
                    layer = layer || row;
                    const int64_t lines = static_cast<int64_t>(std::min(kTileY, pd.n1[1] - ty * kTileY)) *
                                          std::min(kTileZ, pd.n1[2] - tz * kTileZ);
                    if (row) dp.occ_xlines[0] += lines;
                    dp.occ_xlines[1] += lines;
                }
                const int64_t planes = std::min(kTileZ, pd.n1[2] - tz * kTileZ);
                if (layer) dp.occ_zplanes[0] += planes;
                dp.occ_zplanes[1] += planes;
            }
            dp.occ_tiles[1] += static_cast<int64_t>(pd.ntile[0]) * pd.ntile[1] * pd.ntile[2];
            int64_t gt = pd.tile0;   // tiles are numbered x fastest, then y, then z
            for (int32_t tz = 0; tz < pd.ntile[2]; ++tz)
                for (int32_t ty = 0; ty < pd.ntile[1]; ++ty)
                    for (int32_t tx = 0; tx < pd.ntile[0]; ++tx, ++gt) {
                        if (counts[gt] == 0) {
                            // the x pass does not read this tile's cells
                            dp.alg_bytes[HVOX_K_FFT_X] -=
                                delta * static_cast<double>(std::min(kTileX, pd.n1[0] - tx * kTileX)) *
                                std::min(kTileY, pd.n1[1] - ty * kTileY) * std::min(kTileZ, pd.n1[2] - tz * kTileZ);
                            continue;
                        }
                        SpreadTile d{};
                        d.pair = static_cast<int32_t>(i);
                        d.org[0] = static_cast<int16_t>(tx * kTileX);
                        d.org[1] = static_cast<int16_t>(ty * kTileY);
                        d.org[2] = static_cast<int16_t>(tz * kTileZ);
                        d.r0 = off[gt];
                        d.cnt = std::min(counts[gt], split);
                        d.flags = 0;
                        dp.spread_tiles.push_back(d);
                        for (int32_t done = d.cnt; done < counts[gt]; done += split) {
                            SpreadTile a = d;
                            a.r0 = off[gt] + done;
                            a.cnt = std::min(counts[gt] - done, split);
                            a.flags = kSpreadAdd;
                            adds.push_back(a);
                        }
                    }
        }
        b.list_cnt = static_cast<int64_t>(dp.spread_tiles.size()) - b.list_off;
        dd->spread_add_cnt[&b - dp.batches.data()] = static_cast<int64_t>(adds.size());
        dp.spread_tiles.insert(dp.spread_tiles.end(), adds.begin(), adds.end());
    }
    {
        hipError_t eo = upload(pl, dp.occ_bits, &dd->occ, st);
        if (eo == hipSuccess) eo = hipStreamSynchronize(st);
        if (eo != hipSuccess) return bad(eo, "tile occupancy");
        dp.occ_bits.clear();
        dp.occ_bits.shrink_to_fit();
    }
    if (!dp.spread_tiles.empty()) {
        hipError_t el = upload(pl, dp.spread_tiles, &dd->spread_tiles, st);
        if (el == hipSuccess) el = hipStreamSynchronize(st);
        if (el != hipSuccess) return bad(el, "spreading tiles");
        dp.spread_tiles.clear();
        dp.spread_tiles.shrink_to_fit();
    }
    void *rec = nullptr;
    e = dev_alloc(pl, sizeof(int32_t) * std::max<int64_t>(off[nt], 1), &rec, true, st);
    if (e != hipSuccess) return bad(e, "tile records");
    dd->records = static_cast<int32_t *>(rec);
    e = raw_alloc(pl, sizeof(unsigned long long) * nt, &d_cursor, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_cursor, off.data(), sizeof(int64_t) * nt, hipMemcpyHostToDevice, st);
    for (const Batch &b : dp.batches) {
        if (e != hipSuccess) break;
        e = launch_bin(dd->pairs + b.pair0, dd->pre_pts + b.pre_pts, static_cast<int>(b.npairs), b.pts, sxyz, n_src,
                       w, nullptr, static_cast<unsigned long long *>(d_cursor), dd->records, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return bad(e, "binning scatter pass");
    if (det && off[nt] > 0) {
        // the scatter lists a tile's sources in the order its atomics land; deterministic
        // plans list them in index order, so every tile sums its sources in a fixed order
        std::vector<int32_t> recs(off[nt]);
        e = hipMemcpyAsync(recs.data(), rec, sizeof(int32_t) * off[nt], hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return bad(e, "tile records download");
        for (int64_t t = 0; t < nt; ++t) std::sort(recs.begin() + off[t], recs.begin() + off[t + 1]);
        e = hipMemcpyAsync(rec, recs.data(), sizeof(int32_t) * off[nt], hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return bad(e, "tile records upload");
    }
    cleanup();
    return HVOX_OK;
}

int build_device(hvox_plan_s *pl, hipStream_t st, std::string *err)
{
    HostPlan &hp = pl->hp;
    const Params &p = hp.prm;
    if (hipGetDevice(&pl->device) != hipSuccess) { *err = "hipGetDevice failed"; return HVOX_ERR_HIP; }
    std::vector<double> vx = soa(hp.uvw, hp.vis.perm), sx = soa(hp.xyz, hp.sky.perm);
    int rc = HVOX_OK;
    // on failure, wait for the uploads already enqueued before the host tables they read go away
    auto bail = [&](int r) {
        (void)hipStreamSynchronize(st);
        return r;
    };
    auto chk = [&](hipError_t e, const char *what) {
        if (e != hipSuccess && rc == HVOX_OK) {
            rc = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? HVOX_ERR_OOM : HVOX_ERR_HIP;
            *err = std::string(what) + ": " + hipGetErrorString(e);
        }
    };
    chk(upload(pl, vx, &pl->vis_xyz, st), "visibility coordinates");
    chk(upload(pl, sx, &pl->sky_xyz, st), "sky coordinates");
    chk(upload(pl, hp.vis.perm, &pl->vis_perm, st), "visibility permutation");
    chk(upload(pl, hp.sky.perm, &pl->sky_perm, st), "sky permutation");
    if (rc) return bail(rc);

    // Fourier transforms of the two ES kernels by Gauss-Legendre quadrature:
    // K_hat(nu) = (w/2) sum_q a_q cos(pi nu w z_q), a_q = weight_q ES(z_q).
    // Stage 1 (spreading, w/beta) deconvolves the targets; stage 2
    // (interpolation, w2/beta2) pre-corrects the modes 1 / Phi_hat(l / n2).
    const int nq = 2 * std::max(p.w, p.w2) + 60;
    std::vector<double> zq, wq;
    gauss_legendre(nq, &zq, &wq);
    std::vector<double> aq(nq), aq2(nq);
    for (int q = 0; q < nq; ++q) {
        const double root = std::sqrt(1.0 - zq[q] * zq[q]);
        aq[q] = wq[q] * std::exp(p.beta * (root - 1.0));
        aq2[q] = wq[q] * std::exp(p.beta2 * (root - 1.0));
    }
    std::vector<double> precor(hp.precor_nu.size());
    for (size_t i = 0; i < precor.size(); ++i) {
        double s = 0.0;
        for (int q = 0; q < nq; ++q) s += aq2[q] * std::cos(M_PI * hp.precor_nu[i] * p.w2 * zq[q]);
        precor[i] = 1.0 / (0.5 * p.w2 * s);
    }
    if (p.dtype == HVOX_F64) {
        double *d = nullptr;
        chk(upload(pl, precor, &d, st), "pre-correction tables");
        pl->precor = d;
    } else {
        std::vector<float> precor32(precor.begin(), precor.end());
        float *d = nullptr;
        chk(upload(pl, precor32, &d, st), "pre-correction tables");
        chk(hipStreamSynchronize(st), "pre-correction upload");   // precor32 is released on return
        pl->precor = d;
    }
    // twiddles exp(-2 pi i j / n); the host tables stay alive until the
    // stream synchronisation that ends the plan upload
    std::vector<double2> tw64, cis64;
    std::vector<float2> tw32;
    if (p.dtype == HVOX_F64) {
        tw64.resize(hp.tw_total);
        for (size_t t = 0; t < hp.tw_len.size(); ++t)
            for (int32_t j = 0; j < hp.tw_len[t]; ++j) {
                double a = 2.0 * M_PI * j / hp.tw_len[t];
                tw64[hp.tw_off[t] + j] = make_double2(std::cos(a), -std::sin(a));
            }
        double2 *d = nullptr;
        chk(upload(pl, tw64, &d, st), "twiddles");
        pl->tw = d;
        // the direct sum's phase table: exp(2 pi i k / kCisTab)
        cis64.resize(kCisTab);
        for (int k = 0; k < kCisTab; ++k) {
            const double a = 2.0 * M_PI * k / kCisTab;
            cis64[k] = make_double2(std::cos(a), std::sin(a));
        }
        double2 *dc = nullptr;
        chk(upload(pl, cis64, &dc, st), "phase table");
        pl->cis_tab = dc;
    } else {
        tw32.resize(hp.tw_total);
        for (size_t t = 0; t < hp.tw_len.size(); ++t)
            for (int32_t j = 0; j < hp.tw_len[t]; ++j) {
                double a = 2.0 * M_PI * j / hp.tw_len[t];
                tw32[hp.tw_off[t] + j] = make_float2(static_cast<float>(std::cos(a)), static_cast<float>(-std::sin(a)));
            }
        float2 *d = nullptr;
        chk(upload(pl, tw32, &d, st), "twiddles");
        pl->tw = d;
    }
    if (rc) return bail(rc);
    if (upload_dir(pl, hp.syn, &pl->syn, st) || upload_dir(pl, hp.ana, &pl->ana, st)) {
        *err = "device allocation of sub-problem tables failed";
        return bail(HVOX_ERR_OOM);
    }
    rc = bin_direction(pl, hp.syn, &pl->syn, pl->sky_xyz, hp.n_pix, st, err);
    if (rc == HVOX_OK) rc = bin_direction(pl, hp.ana, &pl->ana, pl->vis_xyz, hp.n_vis, st, err);
    if (rc) return bail(rc);

    // deconvolution factors of every target, per direction
    double *d_zq = nullptr, *d_aq = nullptr, *d_ctr_v = nullptr, *d_ctr_s = nullptr, *d_hs_v = nullptr,
           *d_hs_s = nullptr;
    int32_t *d_cov = nullptr, *d_cos = nullptr;
    chk(upload(pl, zq, &d_zq, st), "quadrature");
    chk(upload(pl, aq, &d_aq, st), "quadrature");
    chk(upload(pl, hp.vis.ctr, &d_ctr_v, st), "chunk centres");
    chk(upload(pl, hp.sky.ctr, &d_ctr_s, st), "chunk centres");
    chk(upload(pl, hp.syn_tgt_scale, &d_hs_v, st), "target scales");
    chk(upload(pl, hp.ana_tgt_scale, &d_hs_s, st), "target scales");
    std::vector<int32_t> cov = chunk_of_order(hp.vis), cos_ = chunk_of_order(hp.sky);
    chk(upload(pl, cov, &d_cov, st), "chunk ids");
    chk(upload(pl, cos_, &d_cos, st), "chunk ids");
    void *tmp = nullptr;
    chk(dev_alloc(pl, sizeof(double) * hp.n_vis, &tmp, true, st), "deconvolution");
    pl->syn.deconv = static_cast<double *>(tmp);
    chk(dev_alloc(pl, sizeof(double) * hp.n_pix, &tmp, true, st), "deconvolution");
    pl->ana.deconv = static_cast<double *>(tmp);
    if (rc) return bail(rc);
    chk(launch_deconv(pl->vis_xyz, hp.n_vis, d_cov, d_ctr_v, d_hs_v, d_zq, d_aq, nq, p.w, pl->syn.deconv, st),
        "deconvolution kernel");
    chk(launch_deconv(pl->sky_xyz, hp.n_pix, d_cos, d_ctr_s, d_hs_s, d_zq, d_aq, nq, p.w, pl->ana.deconv, st),
        "deconvolution kernel");
    // accumulator and workspace
    const size_t delta = p.dtype == HVOX_F64 ? 16 : 8;
    chk(dev_alloc(pl, 16 * static_cast<size_t>(kRowBatch) * static_cast<size_t>(std::max(hp.n_vis, hp.n_pix)), &tmp,
                  true, st),
        "accumulator");
    pl->acc = static_cast<double *>(tmp);
    chk(dev_alloc(pl, delta * static_cast<size_t>(hp.ws_elems), &pl->ws, false, st), "workspace");
    int64_t rec_b, val_b;
    stage_layout(hp, &rec_b, &val_b);
    if (hp.max_pts > 0)
        chk(dev_alloc(pl, static_cast<size_t>(rec_b + val_b), &pl->stage, true, st), "source staging");
    if (rc) return bail(rc);
    // the direct sum's stream and the fork / join events; its grid is capped at
    // kDirectWgPerCu workgroups per CU so the NUFFT kernels find room beside it
    // (HVOX_DIRECT_WG_PER_CU overrides the cap for tuning, 0 = uncapped)
    {
        int ncu = 0;
        chk(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, pl->device), "CU count");
        int per_cu = kDirectWgPerCu;
        if (const char *v = std::getenv("HVOX_DIRECT_WG_PER_CU")) per_cu = std::atoi(v);
        pl->direct_grid_cap = per_cu > 0 ? static_cast<int64_t>(per_cu) * ncu : 0;
    }
    chk(hipStreamCreateWithFlags(&pl->side, hipStreamNonBlocking), "direct-sum stream");
    chk(hipEventCreateWithFlags(&pl->fork_ev, hipEventDisableTiming), "fork event");
    chk(hipEventCreateWithFlags(&pl->join_ev, hipEventDisableTiming), "join event");
    if (rc) return bail(rc);
    chk(hipStreamSynchronize(st), "plan upload");
    return rc;
}

// ---- the static scratch of hvox_transform_noalloc ---------------------------------
// One buffer per GPU in the library's device code; host code reaches it only
// through the per-device address that hipGetSymbolAddress returns (the array's
// name is a host-side stand-in, not a device address).
static __device__ __align__(256) unsigned char scratch[HVOX_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// address of this GPU's copy of `scratch`, looked up once per device (the
// current device must be the plan's)
hipError_t static_scratch(int device, void **ptr)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
}

constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// bytes of the accumulator rows, staged sources and grid workspace a plan
// takes from the static scratch, each rounded up to 256 bytes
void static_scratch_layout(const HostPlan &hp, size_t *acc_b, size_t *stage_b, size_t *ws_b)
{
    const bool f64 = hp.prm.dtype == HVOX_F64;
    int64_t rec_b, val_b;
    stage_layout(hp, &rec_b, &val_b);
    *acc_b = align256(16 * static_cast<size_t>(kRowBatch) * static_cast<size_t>(std::max(hp.n_vis, hp.n_pix)));
    *stage_b = align256(static_cast<size_t>(rec_b + val_b));
    *ws_b = align256((f64 ? 16 : 8) * static_cast<size_t>(hp.ws_elems));
}

int transform_static(hvox_plan_s *pl, int32_t direction, const void *in, void *out, int32_t ntrans, void *stream)
{
    if (!pl) return fail(HVOX_ERR_STATE, "NULL plan");
    if (pl->host_only) return fail(HVOX_ERR_STATE, "host-only plan cannot run transforms (hvox_plan_upload first)");
    if (direction != 0 && direction != 1) return fail(HVOX_ERR_ARG, "direction must be 0 (synthesis) or 1 (analysis)");
    if (ntrans < 1) return fail(HVOX_ERR_ARG, "ntrans must be >= 1");
    const bool synthesis = direction == 0;
    const HostPlan &hp = pl->hp;
    const int64_t n_in = synthesis ? hp.n_pix : hp.n_vis;
    const int64_t n_out = synthesis ? hp.n_vis : hp.n_pix;
    if ((n_in > 0 && !in) || (n_out > 0 && !out)) return fail(HVOX_ERR_ARG, "NULL data pointer");
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return fail(HVOX_ERR_HIP, "hipGetDevice failed");
    if (cur != pl->device) return fail(HVOX_ERR_STATE, "the plan's device is not the current device");
    // scratch layout: accumulator rows, staged sources, grid workspace
    const bool f64 = hp.prm.dtype == HVOX_F64;
    size_t acc_b, stage_b, ws_b;
    static_scratch_layout(hp, &acc_b, &stage_b, &ws_b);
    if (acc_b + stage_b + ws_b > HVOX_STATIC_SCRATCH_BYTES)
        return fail(HVOX_ERR_OOM, "the plan needs " + std::to_string(acc_b + stage_b + ws_b) +
                                      " bytes of scratch; the static buffer holds " +
                                      std::to_string(static_cast<size_t>(HVOX_STATIC_SCRATCH_BYTES)));
    void *base = nullptr;
    const hipError_t e = static_scratch(cur, &base);
    if (e != hipSuccess) return fail(HVOX_ERR_HIP, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
    char *b = static_cast<char *>(base);
    int64_t rec_b, val_b;
    stage_layout(hp, &rec_b, &val_b);
    const Scratch sc{b + acc_b + stage_b, b + acc_b, reinterpret_cast<double *>(b),
                     val_b > 0 ? b + acc_b + rec_b : nullptr};
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (f64) return run_direction<double>(pl, synthesis, in, out, ntrans, st, sc, false);
    return run_direction<float>(pl, synthesis, in, out, ntrans, st, sc, false);
}

// HVOX_FORCE_OOM_BYTES: fault injection (a plan may not hold more device memory)
double forced_oom_limit()
{
    const char *v = std::getenv("HVOX_FORCE_OOM_BYTES");
    if (!v || !*v) return -1.0;
    char *end = nullptr;
    const double lim = std::strtod(v, &end);
    return (end != v && lim >= 0.0) ? lim : -1.0;
}

}  // namespace
}  // namespace hvox

using namespace hvox;

extern "C" {

int hvox_version(void) { return HVOX_VERSION; }

const char *hvox_error_string(int code)
{
    switch (code) {
        case HVOX_OK: return "success";
        case HVOX_ERR_ARG: return "invalid argument";
        case HVOX_ERR_EPS: return "accuracy out of range";
        case HVOX_ERR_OOM: return "out of device memory";
        case HVOX_ERR_HIP: return "HIP runtime error";
        case HVOX_ERR_STATE: return "invalid plan state";
        default: return "unknown error";
    }
}

const char *hvox_last_error(void) { return g_last_error.c_str(); }

int hvox_kernel_params(double eps, double sigma, int32_t *w, double *beta)
{
    if (!w || !beta) return fail(HVOX_ERR_ARG, "NULL output");
    int wi = 0;
    int rc = es_params(eps, sigma, &wi, beta);
    if (rc) return fail(rc, "no kernel for this eps / sigma");
    *w = wi;
    return HVOX_OK;
}

int hvox_alg1(const double B[3], const double P[3], double v_max, double alpha, double h[3], double eta[3])
{
    if (!B || !P || !h || !eta) return fail(HVOX_ERR_ARG, "NULL argument");
    int rc = alg1(B, P, v_max, alpha, h, eta);
    if (rc) return fail(rc, "Algorithm 1: widths and budget must be positive, alpha >= 1");
    return HVOX_OK;
}

int64_t hvox_partition(const double *x, int64_t n, const double h[3], int32_t *labels)
{
    if (!h) return fail(HVOX_ERR_ARG, "NULL h");
    try {
        int64_t r = partition(x, n, h, labels);
        if (r < 0) return fail(static_cast<int>(r), "Algorithm 2: bad points or box dimensions");
        return r;
    } catch (const std::bad_alloc &) {
        return fail(HVOX_ERR_OOM, "host allocation failed");
    }
}

int hvox_plan(const double *uvw, int64_t n_vis, const double *xyz, int64_t n_pix, double eps, int32_t dtype,
              const hvox_opts *opts, void *stream, hvox_plan_t *out)
{
    auto t0 = std::chrono::steady_clock::now();
    if (!out) return fail(HVOX_ERR_ARG, "NULL output plan pointer");
    *out = nullptr;
    if (n_vis < 0 || n_pix < 0) return fail(HVOX_ERR_ARG, "negative point count");
    if ((n_vis > 0 && !uvw) || (n_pix > 0 && !xyz)) return fail(HVOX_ERR_ARG, "NULL coordinates");
    if (n_vis > INT32_MAX || n_pix > INT32_MAX) return fail(HVOX_ERR_ARG, "more than 2^31-1 points");
    if (dtype != HVOX_F32 && dtype != HVOX_F64) return fail(HVOX_ERR_ARG, "dtype must be HVOX_F32 or HVOX_F64");
    if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(HVOX_ERR_EPS, "eps must be finite and >= 0");
    Params prm;
    prm.dtype = dtype;
    prm.eps = eps;
    hvox_opts o{};
    if (opts) o = *opts;
    prm.sigma_opt = o.upsampfac;
    prm.sigma2_opt = o.inner_upsampfac;
    if (prm.sigma_opt != 0.0 && !(prm.sigma_opt >= 1.25 && prm.sigma_opt <= 2.0))
        return fail(HVOX_ERR_ARG, "upsampfac must lie in [1.25, 2]");
    if (prm.sigma2_opt != 0.0 && !(prm.sigma2_opt >= 1.25 && prm.sigma2_opt <= 2.0))
        return fail(HVOX_ERR_ARG, "inner_upsampfac must lie in [1.25, 2]");
    prm.alpha = o.anisotropy == 0.0 ? 1.0 : o.anisotropy;
    if (!(prm.alpha >= 1.0) || !std::isfinite(prm.alpha)) return fail(HVOX_ERR_ARG, "anisotropy must be >= 1");
    prm.max_fft_bytes = o.max_fft_bytes == 0.0 ? 500e6 : o.max_fft_bytes;
    if (!(prm.max_fft_bytes > 0.0)) return fail(HVOX_ERR_ARG, "max_fft_bytes must be > 0");
    prm.ws_cap = o.workspace_bytes == 0.0 ? 4.0 * 1024 * 1024 * 1024 : o.workspace_bytes;
    if (!(prm.ws_cap > 0.0) || !std::isfinite(prm.ws_cap)) return fail(HVOX_ERR_ARG, "workspace_bytes must be > 0");
    prm.direct_threshold = o.direct_threshold;
    if (std::isnan(prm.direct_threshold)) return fail(HVOX_ERR_ARG, "direct_threshold is NaN");
    prm.flags = o.flags;
    if (o.ntrans_hint < 0) return fail(HVOX_ERR_ARG, "ntrans_hint must be >= 0");
    prm.ntrans_hint = o.ntrans_hint == 0 ? 1 : o.ntrans_hint;
    prm.all_direct = eps == 0.0 || std::isinf(prm.direct_threshold);
    if (eps > 0.0) {
        const double floor_eps = dtype == HVOX_F64 ? 1e-10 : 1e-5;
        if (eps < floor_eps) return fail(HVOX_ERR_EPS, "eps below the floor of this dtype");
        int rc = choose_kernels(&prm, eps);
        if (rc) return fail(rc, "no kernel for this eps");
    } else {
        prm.sigma = prm.sigma_opt > 0.0 ? prm.sigma_opt : 1.25;
        prm.sigma2 = prm.sigma2_opt > 0.0 ? prm.sigma2_opt : 1.5;
        prm.w = prm.w2 = 3;
        prm.beta = prm.beta2 = 1.0;
    }
    if ((o.dev_alloc == nullptr) != (o.dev_free == nullptr))
        return fail(HVOX_ERR_ARG, "dev_alloc and dev_free must be given together");
    auto *pl = new (std::nothrow) hvox_plan_s();
    if (!pl) return fail(HVOX_ERR_OOM, "host allocation failed");
    pl->host_only = (prm.flags & HVOX_PLAN_HOST_ONLY) != 0;
    pl->alloc_hook = o.dev_alloc;
    pl->free_hook = o.dev_free;
    pl->alloc_ctx = o.alloc_ctx;
    pl->oom_limit = forced_oom_limit();
    pl->last_stream = static_cast<hipStream_t>(stream);
    std::string err;
    int rc;
    try {
        rc = make_host_plan(uvw, n_vis, xyz, n_pix, prm, o.vis_chunk, o.sky_chunk, &pl->hp, &err);
        if (rc == HVOX_OK && pl->oom_limit >= 0.0 &&
            static_cast<double>(device_bytes_bound(pl->hp)) > pl->oom_limit) {
            // fault injection: a plan whose device memory could exceed the forced limit fails
            // before touching the device (host-only plans included)
            rc = HVOX_ERR_OOM;
            err = "device memory bound of the plan exceeds HVOX_FORCE_OOM_BYTES";
        }
        if (rc == HVOX_OK && !pl->host_only) rc = build_device(pl, static_cast<hipStream_t>(stream), &err);
    } catch (const std::bad_alloc &) {
        rc = HVOX_ERR_OOM;
        err = "host allocation failed";
    } catch (const std::exception &ex) {
        rc = HVOX_ERR_ARG;
        err = ex.what();
    }
    if (rc != HVOX_OK) {
        if (!pl->host_only) (void)hipStreamSynchronize(static_cast<hipStream_t>(stream));   // uploads in flight
        release(pl);
        delete pl;
        return fail(rc, err);
    }
    pl->plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = pl;
    return HVOX_OK;
}

int hvox_synthesis(hvox_plan_t plan, const void *sky, void *vis, int32_t ntrans, void *stream)
{
    try {
        return transform(plan, true, sky, vis, ntrans, stream);
    } catch (...) {
        return fail(HVOX_ERR_HIP, "unexpected failure in hvox_synthesis");
    }
}

int hvox_analysis(hvox_plan_t plan, const void *vis, void *sky, int32_t ntrans, void *stream)
{
    try {
        return transform(plan, false, vis, sky, ntrans, stream);
    } catch (...) {
        return fail(HVOX_ERR_HIP, "unexpected failure in hvox_analysis");
    }
}

int hvox_plan_upload(hvox_plan_t plan, void *stream)
{
    if (!plan) return fail(HVOX_ERR_ARG, "NULL plan");
    if (!plan->host_only) return fail(HVOX_ERR_STATE, "the plan already has its device part");
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = static_cast<hipStream_t>(stream);
    plan->last_stream = st;
    std::string err;
    int rc;
    try {
        rc = build_device(plan, st, &err);
    } catch (const std::bad_alloc &) {
        rc = HVOX_ERR_OOM;
        err = "host allocation failed";
    } catch (...) {
        rc = HVOX_ERR_HIP;
        err = "unexpected failure in hvox_plan_upload";
    }
    if (rc != HVOX_OK) {
        (void)hipStreamSynchronize(st);
        release(plan);
        plan->vis_xyz = plan->sky_xyz = nullptr;
        plan->vis_perm = plan->sky_perm = nullptr;
        plan->precor = plan->tw = plan->ws = plan->stage = plan->cis_tab = nullptr;
        plan->acc = nullptr;
        plan->syn = DevDir{};
        plan->ana = DevDir{};
        return fail(rc, err);
    }
    plan->host_only = false;
    plan->hp.prm.flags &= ~HVOX_PLAN_HOST_ONLY;
    plan->plan_seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return HVOX_OK;
}

int hvox_synthesis_dde(hvox_plan_t plan, const void *sky, void *vis, const void *a, const void *b, int32_t n_terms,
                       int32_t ntrans, void *work, void *stream)
{
    try {
        return transform_dde(plan, true, sky, vis, a, b, n_terms, ntrans, work, stream);
    } catch (...) {
        return fail(HVOX_ERR_HIP, "unexpected failure in hvox_synthesis_dde");
    }
}

int hvox_analysis_dde(hvox_plan_t plan, const void *vis, void *sky, const void *a, const void *b, int32_t n_terms,
                      int32_t ntrans, void *work, void *stream)
{
    try {
        return transform_dde(plan, false, vis, sky, a, b, n_terms, ntrans, work, stream);
    } catch (...) {
        return fail(HVOX_ERR_HIP, "unexpected failure in hvox_analysis_dde");
    }
}

int hvox_transform_noalloc(hvox_plan_t plan, int32_t direction, const void *in, void *out, int32_t ntrans,
                           void *stream)
{
    try {
        return transform_static(plan, direction, in, out, ntrans, stream);
    } catch (...) {
        return fail(HVOX_ERR_HIP, "unexpected failure in hvox_transform_noalloc");
    }
}

int hvox_free(hvox_plan_t plan)
{
    if (!plan) return HVOX_OK;
    if (!plan->host_only && plan->last_stream) (void)hipStreamSynchronize(plan->last_stream);
    release(plan);
    delete plan;
    return HVOX_OK;
}

int hvox_plan_info(hvox_plan_t plan, hvox_plan_info_t *out)
{
    if (!plan || !out) return fail(HVOX_ERR_ARG, "NULL argument");
    const HostPlan &hp = plan->hp;
    std::memset(out, 0, sizeof(*out));
    out->n_vis = hp.n_vis;
    out->n_pix = hp.n_pix;
    out->dtype = hp.prm.dtype;
    out->w = hp.prm.w;
    out->beta = hp.prm.beta;
    out->sigma = hp.prm.sigma;
    out->w2 = hp.prm.w2;
    out->beta2 = hp.prm.beta2;
    out->sigma2 = hp.prm.sigma2;
    out->eps = hp.prm.eps;
    out->eps_sub = hp.prm.eps_sub > 0.0 ? hp.prm.eps_sub : hp.prm.eps;
    for (int d = 0; d < 3; ++d) { out->h[d] = hp.h[d]; out->eta[d] = hp.eta[d]; }
    out->n_vis_chunks = hp.vis.nc;
    out->n_sky_chunks = hp.sky.nc;
    out->n_pairs_nufft = static_cast<int64_t>(hp.syn.pairs.size());
    out->n_pairs_direct = static_cast<int64_t>(hp.vis.nc) * hp.sky.nc - out->n_pairs_nufft;
    out->n_batches = static_cast<int64_t>(hp.syn.batches.size());
    const int64_t delta = hp.prm.dtype == HVOX_F64 ? 16 : 8;
    out->workspace_bytes = hp.ws_elems * delta;
    out->max_pair_workspace_bytes = hp.max_pair_ws * delta;
    if (plan->host_only) {
        // bound of what hvox_plan_upload allocates besides the workspace
        out->resident_bytes = device_bytes_bound(hp) - hp.ws_elems * delta;
    } else {
        out->resident_bytes = static_cast<int64_t>(plan->resident_bytes);
    }
    out->grid_cells = hp.syn.grid_cells;
    out->direct_terms = hp.syn.direct_terms;
    out->est_seconds = hp.syn.est_seconds + hp.ana.est_seconds;
    out->plan_seconds = plan->plan_seconds;
    out->device_bytes = plan->host_only ? device_bytes_bound(hp) : static_cast<int64_t>(plan->device_bytes);
    out->flags = hp.prm.flags;
    out->on_device = plan->host_only ? 0 : 1;
    out->n_direct_layers = static_cast<int64_t>(std::max<size_t>(hp.syn.direct_layer_off.size(), 1) - 1);
    size_t acc_b, stage_b, ws_b;
    static_scratch_layout(hp, &acc_b, &stage_b, &ws_b);
    out->noalloc_scratch_bytes = static_cast<int64_t>(acc_b + stage_b + ws_b);
    for (int q = 0; q < 2; ++q) {
        out->occ_tiles[q] = hp.syn.occ_tiles[q] + hp.ana.occ_tiles[q];
        out->occ_xlines[q] = hp.syn.occ_xlines[q] + hp.ana.occ_xlines[q];
        out->occ_zplanes[q] = hp.syn.occ_zplanes[q] + hp.ana.occ_zplanes[q];
    }
    out->nufft_rows = hp.rows;
    out->est_direct_seconds = hp.syn.est_direct_seconds + hp.ana.est_direct_seconds;
    return HVOX_OK;
}

int hvox_plan_permutation(hvox_plan_t plan, int32_t *vis_perm, int32_t *sky_perm)
{
    if (!plan) return fail(HVOX_ERR_ARG, "NULL plan");
    if (vis_perm) std::memcpy(vis_perm, plan->hp.vis.perm.data(), sizeof(int32_t) * plan->hp.n_vis);
    if (sky_perm) std::memcpy(sky_perm, plan->hp.sky.perm.data(), sizeof(int32_t) * plan->hp.n_pix);
    return HVOX_OK;
}

int hvox_plan_chunks(hvox_plan_t plan, int32_t *vis_chunk, int32_t *sky_chunk)
{
    if (!plan) return fail(HVOX_ERR_ARG, "NULL plan");
    if (vis_chunk) std::memcpy(vis_chunk, plan->hp.vis.label.data(), sizeof(int32_t) * plan->hp.n_vis);
    if (sky_chunk) std::memcpy(sky_chunk, plan->hp.sky.label.data(), sizeof(int32_t) * plan->hp.n_pix);
    return HVOX_OK;
}

int hvox_stats(hvox_plan_t plan, hvox_stats_t *out)
{
    if (!plan || !out) return fail(HVOX_ERR_ARG, "NULL argument");
    if (!plan->host_only) {
        hipError_t e = resolve_timing(plan);
        if (e != hipSuccess) return fail(HVOX_ERR_HIP, std::string("HIP: ") + hipGetErrorString(e));
    }
    *out = plan->stats;
    return HVOX_OK;
}

int hvox_set_timing(hvox_plan_t plan, int32_t on)
{
    if (!plan) return fail(HVOX_ERR_ARG, "NULL plan");
    if (on) plan->hp.prm.flags |= HVOX_TIMING;
    else plan->hp.prm.flags &= ~HVOX_TIMING;
    return HVOX_OK;
}

int hvox_stats_reset(hvox_plan_t plan)
{
    if (!plan) return fail(HVOX_ERR_ARG, "NULL plan");
    if (!plan->host_only) {
        hipError_t e = resolve_timing(plan);
        if (e != hipSuccess) return fail(HVOX_ERR_HIP, std::string("HIP: ") + hipGetErrorString(e));
    }
    plan->stats = hvox_stats_t{};
    return HVOX_OK;
}

}  // extern "C"

// ---- kernel-level test entry point (include/hvox_testing.h) ---------------------
#include "../../include/hvox_testing.h"

extern "C" int hvox_test_fft(int32_t dtype, int32_t n, int32_t nin, int32_t nlines, int32_t wstart, int32_t wcount,
                             int32_t sign, const void *in, void *out, void *stream)
{
    using namespace hvox;
    if ((dtype != HVOX_F32 && dtype != HVOX_F64) || n < 2 || n > kFftMaxLen || (n & 1) || nin < 2 || (nin & 1) ||
        nin > n || nlines < 1 || wcount < 1 || wcount > n || (sign != 1 && sign != -1) || !in || !out)
        return fail(HVOX_ERR_ARG, "bad FFT test arguments");
    if (smooth_even(n) != n) return fail(HVOX_ERR_ARG, "n must be 2-3-5 smooth");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t delta = dtype == HVOX_F64 ? 16 : 8;
    // one sub-problem whose x pass is exactly this transform: grid 1 is
    // [1][nlines][nin], pre-correction 1, output window along x only
    PairDev pd{};
    pd.n1[0] = nin; pd.n1[1] = nlines; pd.n1[2] = 1;
    pd.n2[0] = n; pd.n2[1] = nlines; pd.n2[2] = 1;
    pd.wstart[0] = wstart; pd.wcount[0] = wcount;
    pd.wstart[1] = 0; pd.wcount[1] = nlines; pd.wstart[2] = 0; pd.wcount[2] = 1;
    pd.nrad[0] = factor_radices(n, pd.radix[0]);
    pd.lines_per_tile[0] = fft_lines(n);
    const int64_t lines = nlines;
    const int64_t tiles = (lines + pd.lines_per_tile[0] - 1) / pd.lines_per_tile[0];
    const int64_t gin = static_cast<int64_t>(nin) * nlines, gout = static_cast<int64_t>(wcount) * nlines;
    pd.bufG = 0;
    pd.bufA = gin;
    pd.bufB = gin;
    pd.precor[0] = 0; pd.precor[1] = nin; pd.precor[2] = nin + nlines;
    pd.tw[0] = 0;
    std::vector<double> ones(nin + nlines + 1, 1.0);
    std::vector<float> ones32(nin + nlines + 1, 1.0f);
    std::vector<double2> tw64(n);
    std::vector<float2> tw32(n);
    for (int j = 0; j < n; ++j) {
        double a = 2.0 * M_PI * j / n;
        tw64[j] = make_double2(std::cos(a), -std::sin(a));
        tw32[j] = make_float2(static_cast<float>(std::cos(a)), static_cast<float>(-std::sin(a)));
    }
    std::vector<int64_t> prefix = {0, tiles};
    void *d_ws = nullptr, *d_tw = nullptr, *d_pd = nullptr, *d_pre = nullptr, *d_one = nullptr;
    auto cleanup = [&]() {
        for (void *p : {d_ws, d_tw, d_pd, d_pre, d_one}) if (p) (void)hipFree(p);
    };
    hipError_t e = hipMalloc(&d_ws, delta * (gin + gout));
    if (e == hipSuccess) e = hipMalloc(&d_tw, delta * n);
    if (e == hipSuccess) e = hipMalloc(&d_pd, sizeof(PairDev));
    if (e == hipSuccess) e = hipMalloc(&d_pre, sizeof(int64_t) * 2);
    if (e == hipSuccess) e = hipMalloc(&d_one, delta / 2 * ones.size());
    if (e == hipSuccess) e = hipMemcpyAsync(d_ws, in, delta * gin, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_tw, dtype == HVOX_F64 ? static_cast<const void *>(tw64.data()) : tw32.data(), delta * n,
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_pd, &pd, sizeof(PairDev), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_pre, prefix.data(), sizeof(int64_t) * 2, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_one, dtype == HVOX_F64 ? static_cast<const void *>(ones.data()) : ones32.data(),
                           delta / 2 * ones.size(), hipMemcpyHostToDevice, st);
    const int lds = fft_lds_elems(pd.lines_per_tile[0], n);
    if (e == hipSuccess)
        e = dtype == HVOX_F64
                ? launch_fft<double>(static_cast<PairDev *>(d_pd), static_cast<int64_t *>(d_pre), 1, tiles, 0, d_ws,
                                     d_tw, d_one, nullptr, lds, n, sign, 1, 0, st)
                : launch_fft<float>(static_cast<PairDev *>(d_pd), static_cast<int64_t *>(d_pre), 1, tiles, 0, d_ws,
                                    d_tw, d_one, nullptr, lds, n, sign, 1, 0, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, static_cast<char *>(d_ws) + delta * gin, delta * gout, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    cleanup();
    if (e != hipSuccess) return fail(HVOX_ERR_HIP, std::string("HIP: ") + hipGetErrorString(e));
    return HVOX_OK;
}

extern "C" int hvox_test_fft_radices(int32_t n, uint8_t *radix)
{
    using namespace hvox;
    if (!radix || n < 2 || n > kFftMaxLen || smooth_even(n) != n)
        return fail(HVOX_ERR_ARG, "n must be even, 2-3-5 smooth and at most the longest FFT line");
    uint8_t r[kMaxStages];
    const int ns = factor_radices(n, r);
    if (ns < 1) return fail(HVOX_ERR_ARG, "no radix plan for this length");
    for (int i = 0; i < ns; ++i) radix[i] = r[i];
    return ns;
}
