// Host planner of the HVOX library: Heisenberg boxes, kernel parameters,
// Algorithm 1 (maximum box dimensions under an FFT budget), Algorithm 2
// (lattice partition + fusion), chunk-order permutations, per-sub-problem grid
// sizes, the NUFFT-or-direct choice and the grouping of sub-problems that
// share the device workspace.
//
// Floating-point contraction is disabled in this file so that the partition
// decisions (box widths compared against h) are plain IEEE operations,
// independent of the compiler's FMA choices.
#pragma clang fp contract(off)

#include <algorithm>
#include <cmath>
#include <limits>
#include <map>
#include <numeric>
#include <string>
#include <thread>
#include <unordered_map>

#include "hvox_internal.hpp"

namespace hvox {

namespace {

constexpr double kPi = 3.14159265358979323846;

// Cost-model rates used to choose NUFFT or direct summation for each
// sub-problem, from MI355X kernel timings: the grid passes (FFT passes,
// transpose) sustain ~3e12 algorithmic bytes/s of the byte model
// below and the spreading / interpolation kernels ~4e11 kernel-cell updates/s
// in float32 and ~8e11 in float64 (its 14-wide footprints fill more lanes of
// a wavefront, and float64 FMAs issue at the float32 rate); the direct
// kernel 3.0e12 (float32) and 1.35e12 (float64) terms/s.  A sweep of the
// decision threshold on the SKA-like and dense DCOS workloads puts the
// fastest split at these rates (threshold 1).
struct Rates {
    double hbm_bytes_per_s;     // effective streaming rate of the grid passes
    double cells_per_s;         // spread/interp kernel-cell updates
    double terms_per_s;         // direct-sum terms
    double pair_overhead_s;     // fixed cost of a NUFFT sub-problem
};

Rates rates_for(int dtype)
{
    if (dtype == HVOX_F64) return {3.0e12, 8.0e11, 1.35e12, 4e-6};
    return {3.0e12, 4.0e11, 3.0e12, 4e-6};
}

}  // namespace

// Kernel support and shape from the accuracy target.  The ES kernel's
// aliasing error decays like exp(-pi w sqrt(1 - 1/sigma)) with
// beta = 0.97 pi w (1 - 1/(2 sigma)) (the published ES error analysis the
// paper cites for its kernels, Sect. 2.1); one extra cell covers the two
// approximation stages of the type-3 transform (spreading and the inner
// upsampled FFT + interpolation each contribute).
int es_params(double eps, double sigma, int *w, double *beta)
{
    if (!(eps > 0.0) || !(eps < 1.0) || !(sigma > 1.0) || !std::isfinite(sigma)) return HVOX_ERR_ARG;
    double ww = std::ceil(std::log(1.0 / eps) / (kPi * std::sqrt(1.0 - 1.0 / sigma))) + 1.0;
    int wi = std::max(3, static_cast<int>(ww));
    if (wi > kWMax) return HVOX_ERR_EPS;
    *w = wi;
    *beta = 0.97 * kPi * wi * (1.0 - 1.0 / (2.0 * sigma));
    return HVOX_OK;
}

// Upsampling factors and kernels for a per-sub-problem accuracy eps_sub.
// Both type-3 stages divide by a kernel transform that falls by
// ~exp(-c(sigma) beta) per dimension towards the edge of its band
// (c = 0.27 at sigma = 1.25, 0.14 at 1.5): targets near the corners of a box
// populated in all three dimensions, and the inner FFT's edge modes, are then
// recovered from sums that cancel by that factor cubed, which costs digits of
// the working precision as beta (i.e. w) grows.  Measured on chunked 3D
// sub-problems: the inner stage stays within eps at sigma2 = 1.5 for every
// supported eps; spreading at sigma = 1.25 stays within eps while w <= 8
// (float32) or w <= 12 (float64), and sigma = 1.5 is used beyond.
int choose_kernels(Params *p, double eps_sub)
{
    const double e = std::min(eps_sub, 0.5);
    p->sigma2 = p->sigma2_opt > 0.0 ? p->sigma2_opt : 1.5;
    int rc = es_params(e, p->sigma2, &p->w2, &p->beta2);
    if (rc) return rc;
    if (p->sigma_opt > 0.0) {
        p->sigma = p->sigma_opt;
        return es_params(e, p->sigma, &p->w, &p->beta);
    }
    const int wmax_125 = p->dtype == HVOX_F64 ? 12 : 8;
    p->sigma = 1.25;
    rc = es_params(e, p->sigma, &p->w, &p->beta);
    if (rc == HVOX_OK && p->w <= wmax_125) return HVOX_OK;
    p->sigma = 1.5;
    return es_params(e, p->sigma, &p->w, &p->beta);
}

// Smallest even n' >= n whose prime factors are 2, 3 and 5 only.
int32_t smooth_even(int64_t n)
{
    if (n < 2) n = 2;
    for (int64_t m = n;; ++m) {
        if (m & 1) continue;
        int64_t r = m;
        for (int p : {2, 3, 5})
            while (r % p == 0) r /= p;
        if (r == 1) return static_cast<int32_t>(std::min<int64_t>(m, std::numeric_limits<int32_t>::max()));
    }
}

// Radix stages of an n-point FFT (n = 2^a 3^b 5^c): the product of radices
// from {2, 3, 4, 5, 8, 9} with the least estimated VALU work per element,
// largest radix first (the first stage has no twiddles).  Every stage costs a
// butterfly of R elements ~35 instructions of index and LDS address
// arithmetic, two LDS operations per element, ~6 per twiddle product and the
// butterfly's own arithmetic (the radix-8 stage, 123 instructions in the
// gfx950 assembly, fixes the scale), so fewer, larger stages win.  Radices 6,
// 10, 12 and 16 measured slower: their butterflies' registers cost occupancy.
int factor_radices(int32_t n, uint8_t *radix)
{
    struct Rad { int r, e2, e3, e5, arith; };
    static const Rad rads[] = {{9, 0, 2, 0, 120}, {8, 3, 0, 0, 60}, {5, 0, 0, 1, 40},
                               {4, 2, 0, 0, 16},  {3, 0, 1, 0, 16}, {2, 1, 0, 0, 4}};
    constexpr int kRads = static_cast<int>(sizeof(rads) / sizeof(rads[0]));
    int a = 0, b = 0, c = 0;
    int32_t m = n;
    if (m < 1) return -1;
    while (m % 2 == 0) { m /= 2; ++a; }
    while (m % 3 == 0) { m /= 3; ++b; }
    while (m % 5 == 0) { m /= 5; ++c; }
    if (m != 1) return -1;
    // best[a][b][c]: least cost per element of a 2^a 3^b 5^c-point FFT, and the radix taken first
    const int A = a + 1, B = b + 1, C = c + 1;
    std::vector<double> best(static_cast<size_t>(A) * B * C, 1e300);
    std::vector<int> pick(best.size(), -1);
    auto at = [&](int x, int y, int z) { return (static_cast<size_t>(x) * B + y) * C + z; };
    best[at(0, 0, 0)] = 0.0;
    for (int x = 0; x <= a; ++x)
        for (int y = 0; y <= b; ++y)
            for (int z = 0; z <= c; ++z) {
                if (x + y + z == 0) continue;
                for (int i = 0; i < kRads; ++i) {
                    const Rad &q = rads[i];
                    if (q.e2 > x || q.e3 > y || q.e5 > z) continue;
                    const double rest = best[at(x - q.e2, y - q.e3, z - q.e5)];
                    const double cost = rest + (35.0 + 2.0 * q.r + 6.0 * (q.r - 1) + q.arith) / q.r;
                    if (cost < best[at(x, y, z)]) { best[at(x, y, z)] = cost; pick[at(x, y, z)] = i; }
                }
            }
    int ns = 0;
    for (int x = a, y = b, z = c; x + y + z > 0;) {
        if (ns >= kMaxStages) return -1;
        const Rad &q = rads[pick[at(x, y, z)]];
        radix[ns++] = static_cast<uint8_t>(q.r);
        x -= q.e2; y -= q.e3; z -= q.e5;
    }
    std::sort(radix, radix + ns, [](uint8_t u, uint8_t v) { return u > v; });
    for (int i = ns; i < kMaxStages; ++i) radix[i] = 0;
    return ns;
}

// n-point Gauss-Legendre rule on [-1, 1] (Newton iteration on the Legendre
// three-term recurrence).
void gauss_legendre(int n, std::vector<double> *x, std::vector<double> *w)
{
    x->assign(n, 0.0);
    w->assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        (*x)[i] = -z;
        (*x)[n - 1 - i] = z;
        (*w)[i] = (*w)[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Algorithm 1 (Sect. 3.2).  In log variables u_k = log(h_k/B_k),
// v_k = log(eta_k/P_k) the chunk count is exp(-(sum u + sum v)), the FFT
// memory bound is sum u + sum v <= log(v_max / prod(B P)), h <= B and
// eta <= P are u, v <= 0, and the anisotropy bounds limit pairwise
// differences of u and v to log(alpha).  The objective depends on the sum
// only, so the equal split u_k = v_k = min(0, c)/6 is optimal for every
// alpha >= 1 (it is feasible for alpha = 1 and the optimum value min(0, c)
// cannot be exceeded).  This is the point returned.
int alg1(const double B[3], const double P[3], double v_max, double alpha, double h[3], double eta[3])
{
    if (!(v_max > 0.0) || !(alpha >= 1.0)) return HVOX_ERR_ARG;
    double lsum = 0.0;
    for (int d = 0; d < 3; ++d) {
        if (!(B[d] > 0.0) || !(P[d] > 0.0) || !std::isfinite(B[d]) || !std::isfinite(P[d])) return HVOX_ERR_ARG;
        lsum += std::log(B[d]) + std::log(P[d]);
    }
    double c = std::isfinite(v_max) ? std::log(v_max) - lsum : 0.0;
    double t = c >= 0.0 ? 1.0 : std::exp(c / 6.0);
    for (int d = 0; d < 3; ++d) {
        h[d] = t * B[d];
        eta[d] = t * P[d];
    }
    return HVOX_OK;
}

// Algorithm 2 (Sect. 3.2), steps 1-4.  Readings of what the paper leaves
// open: lattice origin at the box minimum; K_d = max(1, ceil(W_d / h_d))
// cells; a point goes to cell min(K_d - 1, floor((x_d - lo_d) / h_d)); empty
// cells are dropped; fusion visits chunks in ascending cell key
// (key = c_x + K_x (c_y + K_y c_z)) and lets the visited chunk absorb, again
// and again, the admissible neighbour (union box <= h_d in every dimension)
// whose box centre is nearest in h-scaled distance (ties: smaller key).  A
// fused box is at most h wide, so it spans at most two cells per dimension
// and admissible neighbours own cells within one cell of its cell range.
int64_t partition(const double *x, int64_t n, const double hin[3], int32_t *labels)
{
    if (n < 0 || (n > 0 && (!x || !labels))) return HVOX_ERR_ARG;
    if (n == 0) return 0;
    double h[3], lo[3], hi[3];
    int64_t K[3];
    for (int d = 0; d < 3; ++d) {
        h[d] = hin[d];
        if (!(h[d] > 0.0) || !std::isfinite(h[d])) return HVOX_ERR_ARG;
        lo[d] = x[d];
        hi[d] = x[d];
    }
    for (int64_t i = 1; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], x[3 * i + d]);
            hi[d] = std::max(hi[d], x[3 * i + d]);
        }
    double cells_total = 1.0;
    for (int d = 0; d < 3; ++d) {
        double width = hi[d] - lo[d];
        double k = width > 0.0 ? std::max(1.0, std::ceil(width / h[d])) : 1.0;
        if (!(k < 4.0e18)) return HVOX_ERR_ARG;
        K[d] = static_cast<int64_t>(k);
        cells_total *= k;
    }
    if (!(cells_total < 9.0e18)) return HVOX_ERR_ARG;

    // steps 1-3: occupied cells with tight point boxes
    std::vector<int64_t> key(n);
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3];
        for (int d = 0; d < 3; ++d) {
            double q = std::floor((x[3 * i + d] - lo[d]) / h[d]);
            int64_t qi = q < 0.0 ? 0 : (q > static_cast<double>(K[d] - 1) ? K[d] - 1 : static_cast<int64_t>(q));
            c[d] = qi;
        }
        key[i] = c[0] + K[0] * (c[1] + K[1] * c[2]);
    }
    std::vector<int64_t> ukeys(key);
    std::sort(ukeys.begin(), ukeys.end());
    ukeys.erase(std::unique(ukeys.begin(), ukeys.end()), ukeys.end());
    const int64_t nc0 = static_cast<int64_t>(ukeys.size());
    std::unordered_map<int64_t, int64_t> cell_index;
    cell_index.reserve(static_cast<size_t>(nc0) * 2);
    for (int64_t j = 0; j < nc0; ++j) cell_index[ukeys[j]] = j;

    struct Chunk {
        bool alive = true;
        double lo[3], hi[3];
        std::vector<int64_t> cells;   // cell indices
    };
    std::vector<Chunk> ch(nc0);
    std::vector<uint8_t> seen(nc0, 0);
    std::vector<int64_t> cell_of(n);
    for (int64_t i = 0; i < n; ++i) {
        int64_t j = cell_index[key[i]];
        cell_of[i] = j;
        if (!seen[j]) {
            seen[j] = 1;
            for (int d = 0; d < 3; ++d) ch[j].lo[d] = ch[j].hi[d] = x[3 * i + d];
            ch[j].cells.push_back(j);
        } else {
            for (int d = 0; d < 3; ++d) {
                ch[j].lo[d] = std::min(ch[j].lo[d], x[3 * i + d]);
                ch[j].hi[d] = std::max(ch[j].hi[d], x[3 * i + d]);
            }
        }
    }
    std::vector<int64_t> owner(nc0);
    std::iota(owner.begin(), owner.end(), 0);

    auto coords = [&](int64_t k, int64_t c[3]) {
        c[0] = k % K[0];
        c[1] = (k / K[0]) % K[1];
        c[2] = k / (K[0] * K[1]);
    };

    // step 4: greedy fusion
    std::vector<int64_t> cand;
    for (int64_t a = 0; a < nc0; ++a) {
        if (!ch[a].alive) continue;
        for (;;) {
            Chunk &ca = ch[a];
            int64_t cmin[3] = {INT64_MAX, INT64_MAX, INT64_MAX}, cmax[3] = {-1, -1, -1};
            for (int64_t cj : ca.cells) {
                int64_t c[3];
                coords(ukeys[cj], c);
                for (int d = 0; d < 3; ++d) {
                    cmin[d] = std::min(cmin[d], c[d]);
                    cmax[d] = std::max(cmax[d], c[d]);
                }
            }
            cand.clear();
            for (int64_t cz = std::max<int64_t>(0, cmin[2] - 1); cz <= std::min(K[2] - 1, cmax[2] + 1); ++cz)
                for (int64_t cy = std::max<int64_t>(0, cmin[1] - 1); cy <= std::min(K[1] - 1, cmax[1] + 1); ++cy)
                    for (int64_t cx = std::max<int64_t>(0, cmin[0] - 1); cx <= std::min(K[0] - 1, cmax[0] + 1); ++cx) {
                        auto it = cell_index.find(cx + K[0] * (cy + K[1] * cz));
                        if (it == cell_index.end()) continue;
                        int64_t o = owner[it->second];
                        if (o != a) cand.push_back(o);
                    }
            std::sort(cand.begin(), cand.end());
            cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
            int64_t best = -1;
            double best_d = 0.0;
            for (int64_t b : cand) {
                const Chunk &cb = ch[b];
                bool ok = true;
                double dist = 0.0;
                for (int d = 0; d < 3; ++d) {
                    double ulo = std::min(ca.lo[d], cb.lo[d]);
                    double uhi = std::max(ca.hi[d], cb.hi[d]);
                    if (!(uhi - ulo <= h[d])) { ok = false; break; }
                    double ma = 0.5 * (ca.lo[d] + ca.hi[d]);
                    double mb = 0.5 * (cb.lo[d] + cb.hi[d]);
                    double t = (ma - mb) / h[d];
                    dist += t * t;
                }
                if (ok && (best < 0 || dist < best_d)) { best = b; best_d = dist; }
            }
            if (best < 0) break;
            Chunk &cb = ch[best];
            for (int64_t cj : cb.cells) owner[cj] = a;
            ca.cells.insert(ca.cells.end(), cb.cells.begin(), cb.cells.end());
            for (int d = 0; d < 3; ++d) {
                ca.lo[d] = std::min(ca.lo[d], cb.lo[d]);
                ca.hi[d] = std::max(ca.hi[d], cb.hi[d]);
            }
            cb.alive = false;
            cb.cells.clear();
        }
    }
    std::vector<int32_t> relabel(nc0, -1);
    int32_t next = 0;
    for (int64_t a = 0; a < nc0; ++a)
        if (ch[a].alive) relabel[a] = next++;
    for (int64_t i = 0; i < n; ++i) labels[i] = relabel[owner[cell_of[i]]];
    return next;
}

namespace {

uint32_t spread_bits10(uint32_t v)
{
    v &= 0x3ff;
    v = (v | (v << 16)) & 0x030000FF;
    v = (v | (v << 8)) & 0x0300F00F;
    v = (v | (v << 4)) & 0x030C30C3;
    v = (v | (v << 2)) & 0x09249249;
    return v;
}

// Chunk tables from per-point labels: chunks renumbered densely in ascending
// label order; inside a chunk points follow a Morton (Z-order) curve of their
// position in the chunk box, so that consecutive points are spatial
// neighbours (compact tiles for the kernels).
int build_chunkset(const double *x, int64_t n, const int32_t *labels, ChunkSet *cs, std::string *err)
{
    cs->n = n;
    cs->label.assign(labels, labels + n);
    if (n == 0) {
        cs->nc = 0;
        cs->off.assign(1, 0);
        return HVOX_OK;
    }
    int32_t mx = -1;
    for (int64_t i = 0; i < n; ++i) {
        if (labels[i] < 0) { *err = "chunk ids must be >= 0"; return HVOX_ERR_ARG; }
        mx = std::max(mx, labels[i]);
    }
    std::vector<int32_t> dense(static_cast<size_t>(mx) + 1, -1);
    for (int64_t i = 0; i < n; ++i) dense[labels[i]] = 0;
    int32_t nc = 0;
    for (auto &v : dense) if (v == 0) v = nc++;
    for (int64_t i = 0; i < n; ++i) cs->label[i] = dense[labels[i]];
    cs->nc = nc;
    cs->lo.assign(3 * nc, std::numeric_limits<double>::infinity());
    cs->hi.assign(3 * nc, -std::numeric_limits<double>::infinity());
    std::vector<int64_t> cnt(nc, 0);
    for (int64_t i = 0; i < n; ++i) {
        int32_t c = cs->label[i];
        cnt[c]++;
        for (int d = 0; d < 3; ++d) {
            cs->lo[3 * c + d] = std::min(cs->lo[3 * c + d], x[3 * i + d]);
            cs->hi[3 * c + d] = std::max(cs->hi[3 * c + d], x[3 * i + d]);
        }
    }
    cs->off.assign(nc + 1, 0);
    for (int32_t c = 0; c < nc; ++c) cs->off[c + 1] = cs->off[c] + cnt[c];
    cs->ctr.resize(3 * nc);
    cs->half.resize(3 * nc);
    for (int32_t c = 0; c < nc; ++c)
        for (int d = 0; d < 3; ++d) {
            cs->ctr[3 * c + d] = 0.5 * (cs->lo[3 * c + d] + cs->hi[3 * c + d]);
            cs->half[3 * c + d] = 0.5 * (cs->hi[3 * c + d] - cs->lo[3 * c + d]);
        }
    std::vector<uint32_t> code(n);
    for (int64_t i = 0; i < n; ++i) {
        int32_t c = cs->label[i];
        uint32_t q[3];
        for (int d = 0; d < 3; ++d) {
            double wd = cs->hi[3 * c + d] - cs->lo[3 * c + d];
            double f = wd > 0.0 ? (x[3 * i + d] - cs->lo[3 * c + d]) / wd : 0.0;
            q[d] = static_cast<uint32_t>(std::min(1023.0, std::max(0.0, std::floor(f * 1024.0))));
        }
        code[i] = spread_bits10(q[0]) | (spread_bits10(q[1]) << 1) | (spread_bits10(q[2]) << 2);
    }
    cs->perm.resize(n);
    std::vector<int64_t> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
        if (cs->label[a] != cs->label[b]) return cs->label[a] < cs->label[b];
        if (code[a] != code[b]) return code[a] < code[b];
        return a < b;
    });
    for (int64_t j = 0; j < n; ++j) cs->perm[j] = static_cast<int32_t>(idx[j]);
    return HVOX_OK;
}

struct PairGeom {
    int32_t n1[3], n2[3], wstart[3], wcount[3];
    double kscale[3], tscale[3];
    int64_t g1, bx, cy, dz, bufA, bufB;   // bufA, bufB exclude grid 1 (its own region)
    bool fits;
};

// Grid sizes of one sub-problem: source half-widths X, effective target
// half-widths S (> 0).  Grid 1 holds the spread footprint of sources at
// t = x' (2 sigma S), |t| <= T = 2 sigma S X, plus the kernel support w; grid
// 2 upsamples it by the inner factor sigma2 for the FFT; only the FFT
// outputs within n2/(2 sigma) + w2/2 of the origin are read by the
// interpolation (kernel support w2), so only that window is kept.
PairGeom pair_geometry(const double X[3], const double S[3], const Params &p)
{
    const double sigma = p.sigma, sigma2 = p.sigma2;
    const int w = p.w, w2 = p.w2;
    PairGeom g{};
    g.fits = true;
    for (int d = 0; d < 3; ++d) {
        double T = 2.0 * sigma * S[d] * X[d];
        double need1 = std::ceil(2.0 * T + w + 2.0);
        if (!(need1 < 1e9)) { g.fits = false; need1 = 1e9; }
        g.n1[d] = smooth_even(static_cast<int64_t>(need1));
        int64_t need2 = static_cast<int64_t>(std::ceil(sigma2 * g.n1[d]));
        g.n2[d] = smooth_even(std::max<int64_t>(need2, 2 * w2));
        if (g.n2[d] > kFftMaxLen) g.fits = false;
        int64_t R = static_cast<int64_t>(std::ceil(g.n2[d] / (2.0 * sigma) + 0.5 * w2)) + 1;
        if (2 * R + 1 >= g.n2[d]) { g.wstart[d] = 0; g.wcount[d] = g.n2[d]; }
        else { g.wstart[d] = static_cast<int32_t>(-R); g.wcount[d] = static_cast<int32_t>(2 * R + 1); }
        g.kscale[d] = 2.0 * sigma * S[d];
        g.tscale[d] = g.n2[d] / (2.0 * sigma * S[d]);
    }
    const int64_t n1x = g.n1[0], n1y = g.n1[1], n1z = g.n1[2];
    const int64_t wx = g.wcount[0], wy = g.wcount[1], wz = g.wcount[2];
    g.g1 = n1x * n1y * n1z;
    g.bx = wx * n1y * n1z;
    g.cy = wx * wy * n1z;
    g.dz = wx * wy * wz;
    g.bufA = std::max(g.bx, g.dz);
    g.bufB = std::max(g.bx, g.cy);
    // the kernels index inside one grid region with 32-bit arithmetic
    if (g.g1 > kMaxRegionElems || g.bufA > kMaxRegionElems || g.bufB > kMaxRegionElems) g.fits = false;
    return g;
}

// Zero widths are floored so that the dimension spans one grid cell
// (sigma * B * P = 1); both zero: each gets 1/sqrt(sigma).
void floor_widths(double B[3], double P[3], double sigma)
{
    for (int d = 0; d < 3; ++d) {
        if (!(B[d] > 0.0) && !(P[d] > 0.0)) { B[d] = P[d] = 1.0 / std::sqrt(sigma); }
        else if (!(B[d] > 0.0)) B[d] = 1.0 / (sigma * P[d]);
        else if (!(P[d] > 0.0)) P[d] = 1.0 / (sigma * B[d]);
    }
}

int64_t ws_of(const PairGeom &g) { return g.g1 + g.bufA + g.bufB; }

struct DirInputs {
    const ChunkSet *src, *tgt;
    double s_floor[3];          // minimum effective target half-width per dimension
};

double pair_nufft_seconds(const PairGeom &g, int64_t ns, int64_t nt, const Params &p, double *bytes)
{
    const Rates r = rates_for(p.dtype);
    const double delta = p.dtype == HVOX_F64 ? 16.0 : 8.0;
    // spread writes grid 1; x pass G1 -> Bx; transpose 2 Bx; y pass Bx -> Cy; z pass Cy -> Dz
    double b = delta * (2.0 * g.g1 + 4.0 * g.bx + 2.0 * g.cy + g.dz);
    if (bytes) *bytes = b;
    const double w3 = static_cast<double>(p.w) * p.w * p.w, w23 = static_cast<double>(p.w2) * p.w2 * p.w2;
    return b / r.hbm_bytes_per_s + (ns * w3 + nt * w23) / r.cells_per_s + r.pair_overhead_s;
}

// lower bound of pair_nufft_seconds (no grid passes): fixed overhead and cell updates
double nufft_seconds_floor(int64_t ns, int64_t nt, const Params &p)
{
    const Rates r = rates_for(p.dtype);
    const double w3 = static_cast<double>(p.w) * p.w * p.w, w23 = static_cast<double>(p.w2) * p.w2 * p.w2;
    return (ns * w3 + nt * w23) / r.cells_per_s + r.pair_overhead_s;
}

double pair_direct_seconds(int64_t ns, int64_t nt, int dtype)
{
    return static_cast<double>(ns) * static_cast<double>(nt) / rates_for(dtype).terms_per_s;
}

// Cost of `rows` data rows relative to one: the direct kernel evaluates each
// phase factor once for up to kRowBatch rows, so every further row of a group
// adds only its multiply-adds (about 2 of the 11 issue cycles of a float32
// term and 4 of the 22 of a float64 term, from the direct kernel's inner-loop
// instruction counts); a NUFFT sub-problem repeats every stage per row.
double direct_rows_factor(int rows, int dtype)
{
    const double extra = dtype == HVOX_F64 ? 4.0 / 22.25 : 2.0 / 11.125;
    double f = 0.0;
    for (int r = rows; r > 0; r -= kRowBatch) f += 1.0 + extra * (std::min(r, kRowBatch) - 1);
    return f;
}

void plan_direction(const HostPlan &hp, const DirInputs &in, DirPlan *dp,
                    std::map<std::pair<int32_t, int32_t>, int64_t> *precor_map,
                    std::vector<double> *precor_nu, std::map<int32_t, int64_t> *tw_map, int64_t *max_pair_ws)
{
    const Params &p = hp.prm;
    const ChunkSet &src = *in.src, &tgt = *in.tgt;
    const double delta = p.dtype == HVOX_F64 ? 16.0 : 8.0;
    const double w3 = static_cast<double>(p.w) * p.w * p.w;
    const double w23 = static_cast<double>(p.w2) * p.w2 * p.w2;
    struct Cand { int32_t i, j; PairGeom g; };
    std::vector<Cand> nufft;
    dp->direct.clear();
    dp->grid_cells = dp->direct_terms = dp->est_seconds = dp->est_direct_seconds = 0.0;
    for (auto &v : dp->alg_bytes) v = 0.0;
    for (auto &v : dp->alg_flops) v = 0.0;

    // Direct sub-problems are evaluated as work items of <= kDirectTile targets x
    // <= seg sources.  Per target chunk, its direct source chunks are merged into
    // contiguous source ranges (chunks are contiguous in chunk order), and
    // consecutive target chunks with the same ranges share one target range, so
    // items are cut from the merged rectangles rather than from every small pair.
    struct Group { int64_t t0, t1; std::vector<std::pair<int64_t, int64_t>> ranges; };
    std::vector<Group> groups;
    std::vector<std::pair<int64_t, int64_t>> ranges;
    for (int32_t j = 0; j < tgt.nc; ++j) {
        double S[3];
        for (int d = 0; d < 3; ++d) S[d] = std::max(tgt.half[3 * j + d], in.s_floor[d]);
        const int64_t nt = tgt.off[j + 1] - tgt.off[j];
        ranges.clear();
        for (int32_t i = 0; i < src.nc; ++i) {
            const int64_t ns = src.off[i + 1] - src.off[i];
            // per call of ntrans_hint rows
            const double t_dir = pair_direct_seconds(ns, nt, p.dtype) * direct_rows_factor(p.ntrans_hint, p.dtype);
            const double thr = p.direct_threshold < 0.0 ? 1.0 : p.direct_threshold;
            // a NUFFT sub-problem costs at least its fixed overhead and its kernel-cell
            // updates: a pair cheaper direct than that bound is direct whatever its grids
            // (wide fields with thousands of small chunks skip the grid sizing)
            const bool clearly_direct = p.all_direct ||
                (p.direct_threshold != 0.0 && thr * t_dir <= nufft_seconds_floor(ns, nt, p) * p.ntrans_hint);
            auto take_direct = [&]() {
                dp->est_seconds += t_dir;
                dp->est_direct_seconds += t_dir;
                dp->direct_terms += static_cast<double>(ns) * nt;
                if (ns == 0) return;
                if (!ranges.empty() && ranges.back().second == src.off[i]) ranges.back().second = src.off[i + 1];
                else ranges.emplace_back(src.off[i], src.off[i + 1]);
            };
            if (clearly_direct) {
                take_direct();
                continue;
            }
            PairGeom g = pair_geometry(&src.half[3 * i], S, p);
            const double t_nu = pair_nufft_seconds(g, ns, nt, p, nullptr) * p.ntrans_hint;
            bool direct;
            if (!g.fits) direct = true;
            else if (p.direct_threshold == 0.0) direct = false;
            else direct = thr * t_dir <= t_nu;
            if (direct) {
                take_direct();
            } else {
                dp->est_seconds += t_nu;
                nufft.push_back({i, j, g});
            }
        }
        if (nt == 0 || ranges.empty()) continue;
        if (!groups.empty() && groups.back().ranges == ranges && groups.back().t1 == tgt.off[j])
            groups.back().t1 = tgt.off[j + 1];
        else
            groups.push_back({tgt.off[j], tgt.off[j + 1], ranges});
    }
    // Segment length: the longest of kDirectSeg, kDirectSeg/2, ... (>= 2 LDS
    // tiles) that still gives enough items to fill the GPU.  Items are listed
    // source-segment-major: consecutive workgroups (spread over the XCDs) work on
    // the same source segment for different target tiles, so a segment is
    // fetched into each XCD's L2 once rather than once per tile.
    int64_t seg = kDirectSeg;
    for (; seg > 2 * kDirectSrcTile; seg /= 2) {
        int64_t items = 0;
        for (const Group &g : groups) {
            int64_t segs = 0;
            for (const auto &r : g.ranges) segs += (r.second - r.first + seg - 1) / seg;
            items += segs * ((g.t1 - g.t0 + kDirectTile - 1) / kDirectTile);
        }
        if (items >= kDirectMinItems) break;
    }
    // layer of an item: its source segment's position in its group's list (deterministic plans
    // launch layer by layer; other plans launch every item at once)
    std::vector<int64_t> layer_of;
    for (const Group &g : groups) {
        int64_t layer = 0;
        for (const auto &r : g.ranges)
            for (int64_t s0 = r.first; s0 < r.second; s0 += seg, ++layer)
                for (int64_t t0 = g.t0; t0 < g.t1; t0 += kDirectTile) {
                    DirectItem it;
                    it.tgt_off = t0;
                    it.src_off = s0;
                    it.tgt_cnt = static_cast<int32_t>(std::min<int64_t>(kDirectTile, g.t1 - t0));
                    it.src_cnt = static_cast<int32_t>(std::min<int64_t>(seg, r.second - s0));
                    dp->direct.push_back(it);
                    layer_of.push_back(layer);
                }
    }
    dp->direct_layer_off.assign(1, 0);
    if (p.deterministic() && !dp->direct.empty()) {
        const int64_t nl = *std::max_element(layer_of.begin(), layer_of.end()) + 1;
        std::vector<int64_t> cnt(nl + 1, 0);
        for (int64_t l : layer_of) cnt[l + 1]++;
        for (int64_t l = 0; l < nl; ++l) cnt[l + 1] += cnt[l];
        std::vector<DirectItem> sorted(dp->direct.size());
        std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
        for (size_t q = 0; q < dp->direct.size(); ++q) sorted[pos[layer_of[q]]++] = dp->direct[q];
        dp->direct.swap(sorted);
        dp->direct_layer_off.assign(cnt.begin() + 1, cnt.end());
        dp->direct_layer_off.insert(dp->direct_layer_off.begin(), 0);
    } else if (!dp->direct.empty()) {
        dp->direct_layer_off.push_back(static_cast<int64_t>(dp->direct.size()));
    }
    dp->alg_flops[HVOX_K_DIRECT] = dp->direct_terms;

    // Deterministic plans: sub-problems source-chunk-major, and a batch never holds two
    // sub-problems of one target chunk, so the interpolation of a batch adds into every
    // target at most once (plain read-modify-write, no atomics) and the batches add in order.
    if (p.deterministic())
        std::stable_sort(nufft.begin(), nufft.end(), [](const Cand &a, const Cand &b) {
            return a.i != b.i ? a.i < b.i : a.j < b.j;
        });
    // group NUFFT sub-problems into batches sharing the workspace
    dp->pairs.clear();
    dp->batches.clear();
    dp->pre_pts.clear();
    dp->pre_tgts.clear();
    dp->pre_stiles.clear();
    dp->pre_ttiles.clear();
    dp->spread_tiles.clear();
    dp->tiles_total = 0;
    for (int q = 0; q < 3; ++q) dp->pre_tiles[q].clear();
    // batches fill the caller's workspace cap, raised to the largest NUFFT sub-problem
    int64_t max_ws = 0;
    for (const Cand &c : nufft) max_ws = std::max(max_ws, ws_of(c.g));
    *max_pair_ws = max_ws;
    const int64_t cap = std::max(static_cast<int64_t>(hp.ws_elems), max_ws);
    size_t k = 0;
    while (k < nufft.size()) {
        Batch b;
        b.pair0 = static_cast<int64_t>(dp->pairs.size());
        int64_t sumG = 0, sumA = 0, sumB = 0, npts = 0;
        size_t k1 = k;
        std::vector<uint8_t> tgt_seen;          // deterministic plans: target chunks of this batch
        if (p.deterministic()) tgt_seen.assign(static_cast<size_t>(tgt.nc), 0);
        while (k1 < nufft.size()) {
            const int64_t gg = nufft[k1].g.g1, a = nufft[k1].g.bufA, bb = nufft[k1].g.bufB;
            const int64_t np = src.off[nufft[k1].i + 1] - src.off[nufft[k1].i];
            if (k1 > k && (sumG + sumA + sumB + gg + a + bb > cap || npts + np > kMaxBatchPts)) break;
            if (p.deterministic()) {
                if (tgt_seen[nufft[k1].j]) break;
                tgt_seen[nufft[k1].j] = 1;
            }
            npts += np;
            sumG += gg;
            sumA += a;
            sumB += bb;
            ++k1;
        }
        b.g_cnt = sumG;
        b.npairs = static_cast<int64_t>(k1 - k);
        b.pre_pts = static_cast<int64_t>(dp->pre_pts.size());
        b.pre_tgts = static_cast<int64_t>(dp->pre_tgts.size());
        b.pre_stiles = static_cast<int64_t>(dp->pre_stiles.size());
        dp->pre_stiles.push_back(0);
        b.pre_ttiles = static_cast<int64_t>(dp->pre_ttiles.size());
        dp->pre_ttiles.push_back(0);
        for (int q = 0; q < 3; ++q) b.pre_tiles[q] = static_cast<int64_t>(dp->pre_tiles[q].size());
        dp->pre_pts.push_back(0);
        dp->pre_tgts.push_back(0);
        for (int q = 0; q < 3; ++q) dp->pre_tiles[q].push_back(0);
        int64_t offG = 0, offA = sumG, offB = sumG + sumA;   // grid-1 region, then the A and B buffers
        for (size_t m = k; m < k1; ++m) {
            const Cand &c = nufft[m];
            const PairGeom &g = c.g;
            PairDev pd{};
            pd.src_off = src.off[c.i];
            pd.src_cnt = src.off[c.i + 1] - src.off[c.i];
            pd.tgt_off = tgt.off[c.j];
            pd.tgt_cnt = tgt.off[c.j + 1] - tgt.off[c.j];
            for (int d = 0; d < 3; ++d) {
                pd.xc[d] = src.ctr[3 * c.i + d];
                pd.sc[d] = tgt.ctr[3 * c.j + d];
                pd.kscale[d] = g.kscale[d];
                pd.tscale[d] = g.tscale[d];
                pd.n1[d] = g.n1[d];
                pd.n2[d] = g.n2[d];
                pd.wstart[d] = g.wstart[d];
                pd.wcount[d] = g.wcount[d];
                pd.nrad[d] = factor_radices(g.n2[d], pd.radix[d]);
                pd.lines_per_tile[d] = fft_lines(g.n2[d]);
                auto key = std::make_pair(g.n1[d], g.n2[d]);
                auto it = precor_map->find(key);
                if (it == precor_map->end()) {
                    int64_t off = static_cast<int64_t>(precor_nu->size());
                    for (int32_t l = -g.n1[d] / 2; l < g.n1[d] / 2; ++l)
                        precor_nu->push_back(static_cast<double>(l) / g.n2[d]);
                    it = precor_map->emplace(key, off).first;
                }
                pd.precor[d] = it->second;
                if (tw_map->find(g.n2[d]) == tw_map->end()) tw_map->emplace(g.n2[d], 0);
            }
            pd.bufG = offG;
            pd.bufA = offA;
            pd.bufB = offB;
            pd.ntile[0] = (g.n1[0] + kTileX - 1) / kTileX;
            pd.ntile[1] = (g.n1[1] + kTileY - 1) / kTileY;
            pd.ntile[2] = (g.n1[2] + kTileZ - 1) / kTileZ;
            const int64_t nst = static_cast<int64_t>(pd.ntile[0]) * pd.ntile[1] * pd.ntile[2];
            pd.tile0 = dp->tiles_total;
            dp->tiles_total += nst;
            b.stiles += nst;
            dp->pre_stiles.push_back(dp->pre_stiles.back() + nst);
            offG += g.g1;
            offA += g.bufA;
            offB += g.bufB;
            int64_t lines[3] = {static_cast<int64_t>(g.n1[2]) * g.n1[1],
                                static_cast<int64_t>(g.n1[2]) * g.wcount[0],
                                static_cast<int64_t>(g.wcount[0]) * g.wcount[1]};
            const int64_t ntt = static_cast<int64_t>(g.n1[2]) * ((g.n1[1] + kTransposeTile - 1) / kTransposeTile) *
                                ((g.wcount[0] + kTransposeTile - 1) / kTransposeTile);
            b.ttiles += ntt;
            dp->pre_ttiles.push_back(dp->pre_ttiles.back() + ntt);
            for (int q = 0; q < 3; ++q) {
                int64_t L = pd.lines_per_tile[q];
                int64_t tiles = (lines[q] + L - 1) / L;
                b.tiles[q] += tiles;
                dp->pre_tiles[q].push_back(dp->pre_tiles[q].back() + tiles);
                b.lds_elems[q] = std::max<int32_t>(b.lds_elems[q], fft_lds_elems(static_cast<int>(L), g.n2[q]));
                b.max_pass_len[q] = std::max(b.max_pass_len[q], g.n2[q]);
            }
            b.pts += pd.src_cnt;
            b.tgts += pd.tgt_cnt;
            const int64_t iblk = (pd.tgt_cnt + kInterpTargets - 1) / kInterpTargets;
            b.iblocks += iblk;
            dp->pre_pts.push_back(dp->pre_pts.back() + pd.src_cnt);
            dp->pre_tgts.push_back(dp->pre_tgts.back() + iblk);
            dp->grid_cells += static_cast<double>(g.g1);
            // algorithmic HBM bytes per kernel (see the kernel documentation)
            // gather + pre-phase: coordinates, permutation, input value read, staged source written
            const double staged = p.dtype == HVOX_F64 ? sizeof(StagedSrc<double>) : sizeof(StagedSrc<float>);
            dp->alg_bytes[HVOX_K_PREPHASE] += pd.src_cnt * (24.0 + 4.0 + delta + staged);
            // spreading (with the gather of A5): a source's coordinates (16 bytes) and value, and
            // every grid-1 cell its kernel touches written once, delta min(G1, N_s w^3)
            dp->alg_bytes[HVOX_K_SPREAD] += pd.src_cnt * (16.0 + delta) +
                                            delta * std::min(static_cast<double>(g.g1), pd.src_cnt * w3);
            dp->alg_bytes[HVOX_K_FFT_X] += delta * (static_cast<double>(g.g1) + g.bx);
            dp->alg_bytes[HVOX_K_TRANSPOSE] += delta * 2.0 * static_cast<double>(g.bx);
            dp->alg_bytes[HVOX_K_FFT_Y] += delta * (static_cast<double>(g.bx) + g.cy);
            dp->alg_bytes[HVOX_K_FFT_Z] += delta * (static_cast<double>(g.cy) + g.dz);
            // interpolation: a target's coordinates (16 bytes) and result, and every grid cell
            // its kernel reads once, delta min(G2 window, N_t w2^3)
            dp->alg_bytes[HVOX_K_INTERP] += pd.tgt_cnt * (16.0 + delta) +
                                            delta * std::min(static_cast<double>(g.dz), pd.tgt_cnt * w23);
            dp->alg_flops[HVOX_K_SPREAD] += pd.src_cnt * w3;
            dp->alg_flops[HVOX_K_INTERP] += pd.tgt_cnt * w23;
            dp->pairs.push_back(pd);
        }
        b.ws_end = offB;
        dp->batches.push_back(b);
        k = k1;
    }
    dp->alg_bytes[HVOX_K_FINAL] = tgt.n * (16.0 + 4.0 + delta);
    dp->alg_bytes[HVOX_K_ZERO] = 16.0 * tgt.n;   // accumulator clear
}

}  // namespace

// Upper bound of the device memory a plan allocates (tables, workspace, staging,
// accumulator, and the binning temporaries of plan creation).  Exact but for
// the tile lists: a source is counted under every tile its footprint can reach
// (ceil((w - 1) / tile) + 1 tiles per dimension), and every crowded tile part
// is counted as if each took a full descriptor.
int64_t device_bytes_bound(const HostPlan &hp)
{
    const Params &p = hp.prm;
    const int64_t nv = hp.n_vis, np = hp.n_pix;
    const int64_t delta = p.dtype == HVOX_F64 ? 16 : 8;
    const int64_t prec = p.dtype == HVOX_F64 ? 8 : 4;
    const int64_t staged = p.dtype == HVOX_F64 ? sizeof(StagedSrc<double>) : sizeof(StagedSrc<float>);
    int64_t b = 24 * (nv + np) + 4 * (nv + np) + 8 * (nv + np) + 4 * (nv + np);   // coords, perms, deconv, chunk ids
    b += 16 * static_cast<int64_t>(kRowBatch) * std::max(nv, np);                // accumulator
    b += prec * static_cast<int64_t>(hp.precor_nu.size()) + delta * hp.tw_total;
    if (p.dtype == HVOX_F64) b += 16 * kCisTab;                                 // direct-sum phase table
    const int nq = 2 * std::max(p.w, p.w2) + 60;
    b += 16 * nq + 48 * (static_cast<int64_t>(hp.vis.nc) + hp.sky.nc);          // quadrature, centres, scales
    const int per_dim[3] = {(p.w - 1 + kTileX - 1) / kTileX + 1, (p.w - 1 + kTileY - 1) / kTileY + 1,
                            (p.w - 1 + kTileZ - 1) / kTileZ + 1};
    const int64_t touch = static_cast<int64_t>(per_dim[0]) * per_dim[1] * per_dim[2];
    int64_t max_pts = 0, temp = 0;
    for (const DirPlan *dp : {&hp.syn, &hp.ana}) {
        b += static_cast<int64_t>(dp->pairs.size() * sizeof(PairDev));
        b += static_cast<int64_t>(dp->direct.size() * sizeof(DirectItem));
        b += 8 * static_cast<int64_t>(dp->pre_pts.size() + dp->pre_tgts.size() + dp->pre_ttiles.size() +
                                      dp->pre_tiles[0].size() + dp->pre_tiles[1].size() + dp->pre_tiles[2].size());
        int64_t pts = 0;
        for (const Batch &bt : dp->batches) {
            pts += bt.pts;
            max_pts = std::max(max_pts, bt.pts);
        }
        const int64_t records = touch * pts;
        b += 4 * std::max<int64_t>(records, 1);
        b += static_cast<int64_t>(sizeof(SpreadTile)) * (dp->tiles_total + records / kSpreadSplit + 1);
        temp = std::max(temp, 12 * dp->tiles_total);                            // binning counts + cursors
        b += 4 * ((dp->tiles_total + 31) / 32 + kOccWords);                     // tile occupancy bits
    }
    b += staged * max_pts + delta * static_cast<int64_t>(hp.rows - 1) * max_pts + 256;   // staged sources
    b += delta * hp.ws_elems;
    return b + temp;
}

int make_host_plan(const double *uvw, int64_t n_vis, const double *xyz, int64_t n_pix,
                   const Params &prm_in, const int32_t *vis_chunk, const int32_t *sky_chunk,
                   HostPlan *hp, std::string *err)
{
    hp->prm = prm_in;
    Params &p = hp->prm;
    hp->n_vis = n_vis;
    hp->n_pix = n_pix;
    hp->uvw.assign(uvw, uvw + 3 * n_vis);
    hp->xyz.assign(xyz, xyz + 3 * n_pix);
    for (int64_t i = 0; i < 3 * n_vis; ++i)
        if (!std::isfinite(uvw[i])) { *err = "non-finite uvw coordinate"; return HVOX_ERR_ARG; }
    for (int64_t i = 0; i < 3 * n_pix; ++i)
        if (!std::isfinite(xyz[i])) { *err = "non-finite sky coordinate"; return HVOX_ERR_ARG; }

    const double delta = p.dtype == HVOX_F64 ? 16.0 : 8.0;
    double Bw[3] = {0, 0, 0}, Pw[3] = {0, 0, 0};
    for (int d = 0; d < 3; ++d) {
        double lo = INFINITY, hi = -INFINITY;
        for (int64_t i = 0; i < n_vis; ++i) { lo = std::min(lo, uvw[3 * i + d]); hi = std::max(hi, uvw[3 * i + d]); }
        Bw[d] = n_vis > 0 ? hi - lo : 0.0;
        lo = INFINITY; hi = -INFINITY;
        for (int64_t i = 0; i < n_pix; ++i) { lo = std::min(lo, xyz[3 * i + d]); hi = std::max(hi, xyz[3 * i + d]); }
        Pw[d] = n_pix > 0 ? hi - lo : 0.0;
    }
    floor_widths(Bw, Pw, p.sigma);

    // Algorithm 1 for the current kernel widths (sets hp->h, hp->eta).
    auto size_boxes = [&]() -> int {
        // Algorithm 1 with the budget expressed as a Heisenberg volume: the two
        // grid buffers of a sub-problem hold ~ 2 prod(sigma h eta) cells of delta
        // bytes.  The padded sizes (kernel support, smooth FFT lengths, output
        // window) are then checked on a lattice-sized sub-problem and the
        // volume is reduced until they fit the budget and the LDS FFT length.
        const double budget = p.max_fft_bytes;
        double vmax = std::isfinite(budget) ? budget / (2.0 * p.sigma * p.sigma * p.sigma * delta) : INFINITY;
        int rc = HVOX_OK;
        for (int it = 0; it < 200; ++it) {
            rc = alg1(Bw, Pw, vmax, p.alpha, hp->h, hp->eta);
            if (rc != HVOX_OK) { *err = "Algorithm 1 rejected its inputs"; return rc; }
            double X[3], S[3];
            for (int d = 0; d < 3; ++d) { X[d] = 0.5 * hp->eta[d]; S[d] = 0.5 * hp->h[d]; }
            PairGeom g = pair_geometry(X, S, p);
            bool ok = g.fits && (!std::isfinite(budget) || ws_of(g) * delta <= budget);
            if (ok) break;
            double shrink = 0.7;
            if (g.fits && std::isfinite(budget)) shrink = std::min(0.9, std::max(0.3, budget / (ws_of(g) * delta)));
            double cur = 1.0;
            for (int d = 0; d < 3; ++d) cur *= hp->h[d] * hp->eta[d];
            double floor_v = 1.0;
            for (int d = 0; d < 3; ++d) floor_v *= std::min(1.0, Bw[d] * Pw[d]) / p.sigma;
            if (cur * shrink < floor_v) break;      // padding alone exceeds the budget: smallest boxes
            vmax = cur * shrink;
        }
        return rc;
    };
    // Algorithm 2 on both domains (or the caller's partitions) for the current boxes.
    // The two domains are independent: the sky is partitioned on a second
    // host thread while this one partitions the visibilities.
    auto partition_domains = [&]() -> int {
        auto one = [](const double *pts, int64_t n, const int32_t *given, const double *box, ChunkSet *out,
                      std::string *msg, const char *what) -> int {
            std::vector<int32_t> lab(n);
            if (given) std::copy(given, given + n, lab.begin());
            else if (n > 0) {
                int64_t nc = partition(pts, n, box, lab.data());
                if (nc < 0) { *msg = std::string("Algorithm 2 failed on the ") + what; return static_cast<int>(nc); }
            }
            return build_chunkset(pts, n, lab.data(), out, msg);
        };
        std::string err_sky;
        int rc_sky = HVOX_OK;
        std::thread sky([&] { rc_sky = one(xyz, n_pix, sky_chunk, hp->eta, &hp->sky, &err_sky, "sky"); });
        const int rc_vis = one(uvw, n_vis, vis_chunk, hp->h, &hp->vis, err, "visibilities");
        sky.join();
        if (rc_vis) return rc_vis;
        if (rc_sky) { *err = err_sky; return rc_sky; }
        return HVOX_OK;
    };
    // Chunked evaluation sums K > 1 sub-problems into every output; their
    // errors add up (the paper notes the chunked result slightly misses eps
    // and suggests a smaller eps per sub-transform).  Reading: the kernels are
    // sized for eps / min(4, K^), K^ the number of lattice cells Algorithm 1's
    // boxes cut the larger domain into (an upper bound on Algorithm 2's chunk
    // count K), so the partition is computed once, with the final widths.
    // (a caller's partition counts with its own number of chunks)
    auto labels_count = [](const int32_t *lab, int64_t n) {
        int32_t m = -1;
        for (int64_t i = 0; i < n; ++i) m = std::max(m, lab[i]);
        return static_cast<double>(m + 1);
    };
    const double kv_given = vis_chunk ? labels_count(vis_chunk, n_vis) : 0.0;
    const double ks_given = sky_chunk ? labels_count(sky_chunk, n_pix) : 0.0;
    auto lattice_cells = [&]() -> double {
        double kv = 1.0, ks = 1.0;
        for (int d = 0; d < 3; ++d) {
            kv *= std::max(1.0, std::ceil(Bw[d] / hp->h[d]));
            ks *= std::max(1.0, std::ceil(Pw[d] / hp->eta[d]));
        }
        return std::max(vis_chunk ? kv_given : kv, sky_chunk ? ks_given : ks);
    };
    int rc = size_boxes();
    if (rc) return rc;
    if (!p.all_direct && p.eps > 0.0) {
        double kmin = 1.0;
        for (int it = 0; it < 3; ++it) {
            const double k = std::min(4.0, lattice_cells());
            if (k <= kmin) break;
            kmin = k;
            const double eps_sub = p.eps / kmin;
            if (choose_kernels(&p, eps_sub) != HVOX_OK) {
                *err = "no kernel for the per-sub-problem accuracy";
                return HVOX_ERR_EPS;
            }
            p.eps_sub = eps_sub;
            rc = size_boxes();
            if (rc) return rc;
        }
    }
    rc = partition_domains();
    if (rc) return rc;

    // effective target half-widths: a dimension narrower than half a grid
    // cell against every source chunk is floored (its phase is negligible)
    auto s_floor = [&](const ChunkSet &src, double out[3]) {
        for (int d = 0; d < 3; ++d) {
            double xm = 0.0;
            for (int32_t c = 0; c < src.nc; ++c) xm = std::max(xm, src.half[3 * c + d]);
            out[d] = xm > 0.0 ? 1.0 / (4.0 * p.sigma * xm) : 1.0;
        }
    };
    DirInputs syn_in{&hp->sky, &hp->vis, {0, 0, 0}};
    DirInputs ana_in{&hp->vis, &hp->sky, {0, 0, 0}};
    s_floor(hp->sky, syn_in.s_floor);
    s_floor(hp->vis, ana_in.s_floor);

    // workspace: the caller's cap, shared by the rows of a pass (each direction
    // raises its batching cap to its largest NUFFT sub-problem)
    hp->rows = std::max(1, std::min(kRowBatch, p.ntrans_hint));
    hp->ws_elems = static_cast<int64_t>(p.ws_cap / delta / hp->rows);

    std::map<std::pair<int32_t, int32_t>, int64_t> precor_map;
    std::map<int32_t, int64_t> tw_map;
    hp->precor_nu.clear();
    int64_t max_ws_syn = 0, max_ws_ana = 0;
    plan_direction(*hp, syn_in, &hp->syn, &precor_map, &hp->precor_nu, &tw_map, &max_ws_syn);
    plan_direction(*hp, ana_in, &hp->ana, &precor_map, &hp->precor_nu, &tw_map, &max_ws_ana);

    hp->max_pair_ws = std::max(max_ws_syn, max_ws_ana);
    // actual workspace: the largest batch, once per row of a pass (row copies
    // 64 elements aligned)
    int64_t used = 0, max_pts = 0;
    for (const DirPlan *dp : {&hp->syn, &hp->ana})
        for (const Batch &b : dp->batches) {
            used = std::max(used, b.ws_end);
            max_pts = std::max(max_pts, b.pts);
        }
    hp->ws_row = hp->rows > 1 ? (used + 63) / 64 * 64 : used;
    hp->ws_elems = hp->ws_row * hp->rows;
    hp->max_pts = max_pts;

    hp->tw_len.clear();
    hp->tw_off.clear();
    int64_t toff = 0;
    for (auto &kv : tw_map) {
        hp->tw_len.push_back(kv.first);
        hp->tw_off.push_back(toff);
        kv.second = toff;
        toff += kv.first;
    }
    hp->tw_total = toff;
    for (DirPlan *dp : {&hp->syn, &hp->ana})
        for (PairDev &pd : dp->pairs)
            for (int d = 0; d < 3; ++d) pd.tw[d] = tw_map[pd.n2[d]];

    // per-chunk target scales h = 1 / (2 sigma S_eff) for the deconvolution
    auto tgt_scales = [&](const ChunkSet &tgt, const double fl[3], std::vector<double> *out) {
        out->resize(3 * tgt.nc);
        for (int32_t j = 0; j < tgt.nc; ++j)
            for (int d = 0; d < 3; ++d)
                (*out)[3 * j + d] = 1.0 / (2.0 * p.sigma * std::max(tgt.half[3 * j + d], fl[d]));
    };
    tgt_scales(hp->vis, syn_in.s_floor, &hp->syn_tgt_scale);
    tgt_scales(hp->sky, ana_in.s_floor, &hp->ana_tgt_scale);
    return HVOX_OK;
}

}  // namespace hvox
