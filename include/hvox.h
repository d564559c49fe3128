/*
 * hvox.h -- C ABI of the MI355X (gfx950) HVOX library.
 *
 * HVOX (Kashani, Rue Queralt, Jarret, Simeoni, arXiv 2306.06007) evaluates
 * interferometric synthesis and its adjoint with a chunked 3D type-3 NUFFT.
 * The problem statement (Sect. 2, Eqs. 2-3, unit tesselation weights):
 *
 *   hvox_synthesis  (sky -> vis):  V_k = sum_n I_n exp(-2 pi i <p_k, r_n>)
 *   hvox_analysis   (vis -> sky):  I_n = sum_k V_k exp(+2 pi i <p_k, r_n>)
 *
 * p_k are uvw baselines in wavelengths, r_n points of an arbitrary sky mesh
 * (unit vectors; any finite 3-vectors are accepted).  The paper names the
 * sky->vis direction "analysis" (Eq. 2) and vis->sky "synthesis" (Eq. 3);
 * this library follows the names above and states each direction explicitly.
 *
 * Both sums are approximated to relative l2 accuracy eps (Sect. 3: the
 * NUFFT's error is controlled through the kernel support) by partitioning the
 * visibility and sky domains into chunks (Sect. 3.1, Eq. 8; Sect. 3.2,
 * Algorithms 1-2) and evaluating every (sky chunk, visibility chunk)
 * sub-problem either as a type-3 NUFFT (spread, 3D FFT, interpolate,
 * deconvolve; Sect. 3) or by direct summation (Sect. 3.1, last bullet).
 *
 * Conventions shared by every entry point
 *  - Coordinates are host arrays of float64, row-major [n][3]; they are
 *    copied, the plan keeps no caller pointer.
 *  - Data vectors are DEVICE pointers to interleaved complex values, complex64
 *    for HVOX_F32 plans and complex128 for HVOX_F64 plans, laid out as ntrans
 *    contiguous rows: sky is [ntrans][n_pix], vis is [ntrans][n_vis].
 *  - Outputs are overwritten, never accumulated into.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the default stream)
 *    and the call returns once it is enqueued.  A plan is immutable after
 *    creation, but owns one workspace: at most one call per plan may be in
 *    flight at a time; concurrent work needs distinct plans.
 *  - Every call returns 0 on success or a negative hvox error code; no C++
 *    exception crosses this boundary.  hvox_last_error() gives a message
 *    (thread-local) describing the most recent failure of this thread.
 */
#ifndef HVOX_H
#define HVOX_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HVOX_VERSION 200

/* error codes */
#define HVOX_OK          0
#define HVOX_ERR_ARG    (-1)  /* NULL pointer, negative size, ntrans < 1, non-finite coordinate, bad option */
#define HVOX_ERR_EPS    (-2)  /* eps < 0, or below the floor of the dtype / upsampling factor */
#define HVOX_ERR_OOM    (-3)  /* device allocation failed or the workspace would exceed its cap */
#define HVOX_ERR_HIP    (-4)  /* a HIP runtime call failed (message in hvox_last_error) */
#define HVOX_ERR_STATE  (-5)  /* freed / host-only plan used for a transform, or wrong call sequence */

typedef enum { HVOX_F32 = 0, HVOX_F64 = 1 } hvox_dtype;

/* option flags */
#define HVOX_REAL_SKY        0x1  /* analysis returns Re(A^H V) (imaginary part 0): a real-valued adjoint
                                     for real sky maps (Sect. 4, the `real` option of Listing 1) */
#define HVOX_PLAN_HOST_ONLY  0x2  /* plan on the host only (partition, pair sizes, costs); no device memory,
                                     transforms return HVOX_ERR_STATE.  For inspection and CPU tests */
#define HVOX_TIMING          0x4  /* record HIP events around every kernel launch; see hvox_stats */
#define HVOX_PREORDERED      0x8  /* data vectors are in the plan's chunk order (hvox_plan_permutation)
                                     instead of user order: the gather and scatter through the
                                     permutations are skipped.  Sect. 4 recommends re-ordering the data
                                     once when a plan is reused for repeated transforms. */
#define HVOX_DETERMINISTIC   0x10 /* bit-reproducible results: no floating-point atomics.  Spreading tiles
                                     are never split and list their sources in index order, sub-problems
                                     sharing a target chunk never run in the same launch, and direct-sum
                                     blocks add into the accumulator layer by layer in a fixed order.
                                     Slower on crowded grids and on plans with few target chunks. */

typedef struct hvox_plan_s *hvox_plan_t;

/* Device-memory hooks.  When both are set, every device allocation of a plan
 * (its tables, workspace, staging and accumulator, and the temporaries of plan
 * creation) goes through them, e.g. to a framework's caching allocator:
 *   dev_alloc(bytes, ctx, stream) returns a device pointer aligned to at least
 *     256 bytes, or NULL on failure (the plan call then fails with
 *     HVOX_ERR_OOM and every block it obtained is handed back);
 *   dev_free(ptr, bytes, ctx, stream) releases a block obtained from dev_alloc
 *     (stream: the plan's last stream, already synchronised).
 * Blocks are first used on the stream given to hvox_plan and later on the
 * streams of the transform calls.  Neither hook may be set alone. */
typedef void *(*hvox_alloc_fn)(size_t bytes, void *ctx, void *stream);
typedef void (*hvox_free_fn)(void *ptr, size_t bytes, void *ctx, void *stream);

/* Plan options.  A zero-initialised struct (or a NULL pointer) selects the
 * defaults noted on each field. */
typedef struct {
    double max_fft_bytes;     /* FFT memory budget B per sub-problem, bytes (Sect. 3.2, Algorithm 1).
                                 0 -> 500e6 (the paper's default partition size, Table 2);
                                 +INFINITY -> one chunk per domain (monolithic type-3, Sect. 3). */
    double anisotropy;        /* alpha >= 1 of Algorithm 1; 0 -> 1. */
    double upsampfac;         /* sigma, the upsampling of the spreading stage (grid 1 against the
                                 Heisenberg box); 0 -> automatic: 1.25 (the type-3 default discussed
                                 in Sect. 5.2) while its kernel support stays <= 8 (float32) or
                                 <= 12 (float64) cells, else 1.5, where 1.25 would cost digits of the
                                 working precision.  Range [1.25, 2]. */
    double inner_upsampfac;   /* sigma2, the upsampling of the inner FFT stage (grid 2 against grid 1);
                                 0 -> 1.5.  Accepted range [1.25, 2]. */
    double direct_threshold;  /* per-sub-problem choice between NUFFT and direct summation (Sect. 3.1):
                                 < 0  -> automatic (cost model);  0 -> never direct (forced NUFFT);
                                 +INFINITY -> always direct.  A positive finite value t makes a
                                 sub-problem direct when t * cost_direct <= cost_nufft. */
    double workspace_bytes;   /* cap on the workspace shared by concurrently executed sub-problems
                                 and the data rows of a NUFFT pass; 0 -> 4 GiB (raised to the
                                 largest single sub-problem, per row, if needed). */
    const int32_t *vis_chunk; /* optional custom partition (host, [n_vis] chunk ids >= 0), replacing
                                 Algorithm 2 on the visibility domain (Sect. 4, allocate()). */
    const int32_t *sky_chunk; /* same for the sky domain ([n_pix]). */
    int32_t flags;            /* HVOX_REAL_SKY | HVOX_PLAN_HOST_ONLY | HVOX_TIMING | HVOX_PREORDERED |
                                 HVOX_DETERMINISTIC */
    int32_t ntrans_hint;      /* data rows per call the plan is made for (Sect. 4, ntrans); 0 -> 1,
                                 negative -> HVOX_ERR_ARG.  The NUFFT sub-problems run in passes of
                                 min(4, ntrans_hint) rows that share the spreading and interpolation
                                 weights, each row in its own copy of the batch workspace (the
                                 workspace_bytes cap is split among them); the direct sum shares its
                                 phase factors among up to four rows and, with the larger per-row
                                 NUFFT cost, the choice between them is weighed for this many rows.
                                 Results depend on it only through rounding (with
                                 HVOX_DETERMINISTIC: not at all for an all-NUFFT plan). */
    hvox_alloc_fn dev_alloc;  /* optional device-memory hooks (see above); NULL -> hipMalloc / hipFree */
    hvox_free_fn  dev_free;
    void *alloc_ctx;          /* passed to both hooks */
} hvox_opts;

/* What a plan decided.  Sizes in bytes; counts of sub-problems are per
 * direction (the same (sky chunk, vis chunk) set serves both). */
typedef struct {
    int64_t n_vis, n_pix;
    int32_t dtype;            /* hvox_dtype */
    int32_t w;                /* spreading kernel support (grid-1 cells per dimension) */
    double  beta;             /* its exponential-of-semicircle shape parameter */
    double  sigma;            /* spreading-stage upsampling factor */
    int32_t w2;               /* interpolation kernel support (grid-2 cells) */
    int32_t pad0;
    double  beta2;            /* its shape parameter */
    double  sigma2;           /* inner FFT upsampling factor */
    double  eps;              /* requested accuracy */
    double  eps_sub;          /* accuracy the sub-problem kernels are sized for (eps / min(4, chunks)) */
    double  h[3], eta[3];     /* Algorithm 1 maximum box dimensions (visibility, sky) */
    int32_t n_vis_chunks, n_sky_chunks;
    int64_t n_pairs_nufft, n_pairs_direct;
    int64_t n_batches;        /* groups of NUFFT sub-problems sharing the workspace */
    int64_t resident_bytes;   /* device memory held by the plan besides the workspace */
    int64_t workspace_bytes;  /* device workspace (grids of concurrently executed sub-problems) */
    int64_t max_pair_workspace_bytes;
    double  grid_cells;       /* sum over NUFFT sub-problems of the grid-1 cell counts */
    double  direct_terms;     /* sum over direct sub-problems of N_src * N_tgt */
    double  est_seconds;      /* cost-model estimate of one synthesis + one analysis (of ntrans_hint rows) */
    double  plan_seconds;     /* host + device time spent in hvox_plan */
    int64_t device_bytes;     /* device memory the plan holds (resident + workspace); for a host-only
                                 plan an upper bound of what hvox_plan_upload will allocate (exact but
                                 for the tile lists, bounded by every source touching 2^3 tiles) */
    int32_t flags;            /* the plan's option flags */
    int32_t on_device;        /* 1 once the device part exists */
    int64_t n_direct_layers;  /* HVOX_DETERMINISTIC: launches of the direct sum per data-row group */
    int64_t noalloc_scratch_bytes;  /* static scratch hvox_transform_noalloc needs for this plan */
    /* occupancy of the NUFFT grids (both directions, device plans): grid-1 tiles (32 x 8 x 8 cells)
     * holding sources, x lines of grid 1 in tile rows holding sources, z planes in tile layers
     * holding sources; [0] occupied, [1] total */
    int64_t occ_tiles[2], occ_xlines[2], occ_zplanes[2];
    int32_t nufft_rows;       /* data rows per NUFFT pass (min(4, ntrans_hint)) */
    int32_t pad1;
    double  est_direct_seconds;   /* the direct sub-problems' part of est_seconds */
} hvox_plan_info_t;

/* Per-kernel statistics of the calls since the last reset (HVOX_TIMING plans). */
#define HVOX_K_ZERO     0   /* accumulator clears */
#define HVOX_K_SPREAD   1   /* spreading over the occupied grid-1 tiles */
#define HVOX_K_FFT_X    2
#define HVOX_K_FFT_Y    3
#define HVOX_K_FFT_Z    4
#define HVOX_K_INTERP   5
#define HVOX_K_DIRECT   6
#define HVOX_K_FINAL    7
#define HVOX_K_TRANSPOSE 8
#define HVOX_K_PREPHASE 9   /* gather + pre-phase of the sources of a batch of sub-problems */
#define HVOX_K_COUNT    10
typedef struct {
    int64_t launches[HVOX_K_COUNT];
    double  ms[HVOX_K_COUNT];           /* summed HIP-event durations */
    double  alg_bytes[HVOX_K_COUNT];    /* algorithmic HBM bytes moved (see the kernel documentation) */
    double  alg_flops[HVOX_K_COUNT];    /* algorithmic arithmetic (direct: terms) */
} hvox_stats_t;

/*
 * Create a plan for uvw [n_vis][3] (host, wavelengths) and xyz [n_pix][3]
 * (host, sky points) at accuracy eps for data of the given dtype.
 * Host work: boxes, kernel parameters, Algorithm 1 (maximum Heisenberg box
 * dimensions under the FFT budget, Sect. 3.2), Algorithm 2 on both domains,
 * chunk-order permutations (Sect. 4: inputs are re-ordered so that chunks are
 * contiguous), per-sub-problem sizes and NUFFT-or-direct choice.  Device work
 * (on `stream`, synchronised before return): coordinates, permutations,
 * deconvolution and FFT tables.
 * eps == 0 selects direct summation for every sub-problem (the paper's eps=0
 * case).  eps floors: 1e-5 for HVOX_F32, 1e-10 for HVOX_F64.
 * n_vis or n_pix may be 0 (outputs are then all zero / empty).
 * On success *out receives the plan, owned by the caller (hvox_free).
 * Out of memory (HVOX_ERR_OOM) leaves nothing allocated.  The environment
 * variable HVOX_FORCE_OOM_BYTES (a byte count) makes every plan whose device
 * memory would exceed it fail with HVOX_ERR_OOM, host-only plans included
 * (their device_bytes bound is checked): fault injection for tests.
 */
int hvox_plan(const double *uvw, int64_t n_vis, const double *xyz, int64_t n_pix,
              double eps, int32_t dtype, const hvox_opts *opts, void *stream,
              hvox_plan_t *out);

/* Create the device part of a plan made with HVOX_PLAN_HOST_ONLY (a host
 * plan, e.g. planned on a worker thread and admitted by its device_bytes):
 * uploads coordinates and tables and allocates the workspace on `stream`
 * (synchronised before return), exactly as hvox_plan would have.  The plan
 * then runs transforms; its flags lose HVOX_PLAN_HOST_ONLY.  On failure the
 * plan stays host-only and holds no device memory.  HVOX_ERR_STATE if the plan
 * already has its device part. */
int hvox_plan_upload(hvox_plan_t plan, void *stream);

/* sky -> vis:  vis[t][k] = sum_n sky[t][n] exp(-2 pi i <p_k, r_n>)   (Eq. 2)
 * sky: device [ntrans][n_pix] complex, vis: device [ntrans][n_vis] complex.
 * Rows are processed in groups of up to four: the direct sub-problems of a
 * group share their phase factors across its rows (one kernel launch), the
 * NUFFT sub-problems run in passes of up to min(4, ntrans_hint) rows that
 * share the spreading and interpolation weights (Sect. 4, ntrans). */
int hvox_synthesis(hvox_plan_t plan, const void *sky, void *vis, int32_t ntrans, void *stream);

/* vis -> sky:  sky[t][n] = sum_k vis[t][k] exp(+2 pi i <p_k, r_n>)   (Eq. 3, the adjoint)
 * With HVOX_REAL_SKY the imaginary part of sky is set to 0. */
int hvox_analysis(hvox_plan_t plan, const void *vis, void *sky, int32_t ntrans, void *stream);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * Runs synthesis (direction 0, as hvox_synthesis) or analysis (direction 1,
 * as hvox_analysis) of `plan` with the same kernels, but the grid workspace,
 * the staged sources and the float64 accumulator come from one static device
 * buffer of HVOX_STATIC_SCRATCH_BYTES per GPU (held from the first call on
 * that GPU until the process ends) instead of the plan's own.  The call
 * allocates nothing: no hipMalloc / hipFree, no events (HVOX_TIMING is
 * ignored).  Inputs and outputs are the caller's, as for hvox_synthesis.
 * Scratch need of a plan: 16 * 4 * max(n_vis, n_pix) accumulator bytes +
 * staged sources of its largest batch + its workspace_bytes, each rounded up
 * to 256 bytes; a plan needing more than the buffer fails with HVOX_ERR_OOM
 * (plan_info's workspace_bytes is bounded by the workspace_bytes option).
 * Every call on one GPU shares that GPU's buffer and it keeps the last call's
 * contents (each call clears what must start at zero): calls that overlap on
 * one GPU race, so serialise them (e.g. one stream). */
#define HVOX_STATIC_SCRATCH_BYTES (64u << 20)
int hvox_transform_noalloc(hvox_plan_t plan, int32_t direction, const void *in, void *out, int32_t ntrans,
                           void *stream);

/* Direction-dependent effects: beam shapes and DDEs, which the paper sets
 * aside in Sect. 2 (its measurement equation omits antenna beams) and names
 * as future work (Sect. 6).  Visibility k sees the sky through a gain
 * A_k(r) given in separable (low-rank) form over n_terms terms,
 *   A_k(r_n) = sum_t a[t][k] b[t][n],
 * e.g. a time-variable primary beam (a[t][k] = 1 when visibility k belongs
 * to snapshot t, b[t] the beam of that snapshot on the sky points) or a
 * low-rank expansion of per-station beams.
 *   hvox_synthesis_dde:  vis[r][k] = sum_n A_k(r_n) sky[r][n] exp(-2 pi i <p_k, r_n>)
 *   hvox_analysis_dde:   sky[r][n] = sum_k conj(A_k(r_n)) vis[r][k] exp(+2 pi i <p_k, r_n>)
 * (an adjoint pair).  Evaluated as n_terms rows of the plan's transform:
 * synthesis of the rows b[t] * sky[r], combined as sum_t a[t] * (row t);
 * analysis of the rows conj(a[t]) * vis[r], combined as sum_t conj(b[t]) *
 * (row t), float64 accumulation.  a: device [n_terms][n_vis], b: device
 * [n_terms][n_pix], complex of the plan's precision, in the data order of the
 * plan (user order, or chunk order with HVOX_PREORDERED).  work: caller's
 * device buffer of at least 2 * n_terms * max(n_vis, n_pix) complex values.
 * sky / vis as for hvox_synthesis (ntrans rows).  HVOX_REAL_SKY applies to
 * the combined analysis output.  HVOX_ERR_ARG for NULL pointers or
 * n_terms < 1. */
int hvox_synthesis_dde(hvox_plan_t plan, const void *sky, void *vis, const void *a, const void *b, int32_t n_terms,
                       int32_t ntrans, void *work, void *stream);
int hvox_analysis_dde(hvox_plan_t plan, const void *vis, void *sky, const void *a, const void *b, int32_t n_terms,
                      int32_t ntrans, void *work, void *stream);

/* Release every resource of the plan (device memory after synchronising the
 * plan's last stream).  NULL is a no-op. */
int hvox_free(hvox_plan_t plan);

/* Fill *out with the plan's decisions and memory footprint. */
int hvox_plan_info(hvox_plan_t plan, hvox_plan_info_t *out);

/* Chunk-order permutations (Sect. 4): vis_perm[j] is the user index of the
 * j-th visibility in chunk order, likewise sky_perm.  Host arrays of n_vis and
 * n_pix entries; either pointer may be NULL.  Supplying data already in this
 * order is what the paper recommends for repeated transforms. */
int hvox_plan_permutation(hvox_plan_t plan, int32_t *vis_perm, int32_t *sky_perm);

/* Chunk id of every point in user order (host arrays, either may be NULL). */
int hvox_plan_chunks(hvox_plan_t plan, int32_t *vis_chunk, int32_t *sky_chunk);

/* Kernel statistics of an HVOX_TIMING plan; hvox_stats_reset clears them.
 * Synchronises the plan's last stream. */
int hvox_stats(hvox_plan_t plan, hvox_stats_t *out);
int hvox_stats_reset(hvox_plan_t plan);

/* Switch per-launch HIP-event timing on (1) or off (0) for later calls of
 * this plan (the HVOX_TIMING flag sets the initial state).  Timing adds two
 * event records per kernel launch on the call's stream. */
int hvox_set_timing(hvox_plan_t plan, int32_t on);

/* ---- host-only helpers (no GPU needed) --------------------------------- */

/* Kernel parameters for accuracy eps at upsampling sigma: support w (cells)
 * and shape beta of the exponential-of-semicircle kernel
 * ES(z) = exp(beta (sqrt(1 - z^2) - 1)), |z| < 1 (the ES kernel named in
 * Sect. 2.1). */
int hvox_kernel_params(double eps, double sigma, int32_t *w, double *beta);

/* Algorithm 1 (Sect. 3.2): maximum box dimensions h (visibility) and eta
 * (sky) minimising the chunk count prod(B/h) prod(P/eta) subject to
 * prod(h eta) <= v_max, h <= B, eta <= P and the anisotropy bounds alpha.
 * B, P: full widths of the two domains (zero widths are floored so that the
 * dimension spans one grid cell). */
int hvox_alg1(const double B[3], const double P[3], double v_max, double alpha,
              double h[3], double eta[3]);

/* Algorithm 2 (Sect. 3.2): partition points x [n][3] (host) into chunks whose
 * boxes are at most h per dimension.  labels[n] receives chunk ids numbered
 * 0..n_chunks-1.  Returns the number of chunks (>= 0) or an error code. */
int64_t hvox_partition(const double *x, int64_t n, const double h[3], int32_t *labels);

/* Human-readable text of an error code, and the calling thread's last message. */
const char *hvox_error_string(int code);
const char *hvox_last_error(void);
int hvox_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HVOX_H */
