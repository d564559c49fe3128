// Host model of the FFT pass kernel's addressing (k_fft_pass in
// paper_2306_06007_amd/csrc/kernels.hip): for every FFT geometry that the
// planner produces, it walks the kernel's index arithmetic -- the load phase
// (pass x with its occupancy mask words, passes y and z), every Stockham stage
// of the planner's radix plan, the window output -- and checks that each LDS,
// twiddle, mask and global access stays inside its buffer, that the
// butterflies of a stage fit the workgroup's thread slots, and that each stage
// writes every element of every line exactly once.
//
//   fft_index_model lengths
//       every even 2-3-5-smooth line length up to the longest FFT line, with
//       full and ragged workgroups
//   fft_index_model plan N_VIS N_PIX UVW.bin XYZ.bin DTYPE EPS MAX_FFT_BYTES DIRECT_THRESHOLD
//       every geometry of the host plan of that input (float64 binaries, 3 per row)
//
// Prints "geometries G checks C errors E" and exits non-zero on any error.
// Must follow the kernel: a change to its indexing belongs here too.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <set>
#include <string>
#include <vector>

#include "hvox_internal.hpp"

using namespace hvox;

static long long g_err = 0, g_chk = 0;
#define CHECK(c, ...)                                           \
    do {                                                        \
        ++g_chk;                                                \
        if (!(c)) {                                             \
            if (g_err++ < 20) { printf(__VA_ARGS__); printf("\n"); } \
        }                                                       \
    } while (0)

// the Stockham stages of one workgroup holding nl lines of length n (each
// distinct workgroup shape and radix plan once)
static void check_stages(int NT, int n, int nl, int ls, int lds_elems, int ns, const uint8_t *radix)
{
    static std::set<std::vector<int>> done;
    std::vector<int> key = {NT, n, nl, ls, lds_elems, ns};
    for (int st = 0; st < ns; ++st) key.push_back(radix[st]);
    if (!done.insert(key).second) return;
    int p = 1, prod = 1;
    for (int st = 0; st < ns; ++st) prod *= radix[st];
    CHECK(prod == n, "radix product %d != n %d", prod, n);
    for (int st = 0; st < ns; ++st) {
        const int R = radix[st];
        CHECK(R == 2 || R == 3 || R == 4 || R == 5 || R == 8 || R == 9, "radix %d has no butterfly", R);
        const int MAXB = (fft_elems(NT) / R + NT - 1) / NT;
        const int nbf = n / R, total = nl * nbf;
        CHECK(n % (p * R) == 0, "p R does not divide n (n %d p %d R %d)", n, p, R);
        CHECK(total <= MAXB * NT, "butterflies %d exceed thread slots %d", total, MAXB * NT);
        const int twstep = st == 0 ? 0 : n / (p * R);
        std::vector<int> hit(static_cast<size_t>(nl) * ls, 0);
        for (int b = 0; b < total; ++b) {
            const int j = b / nbf, i = b - j * nbf;
            const int g = st == 0 ? i : i / p, k = st == 0 ? 0 : i - g * p;
            const int lb = j * ls, ob = lb + g * p * R + k, tk = k * twstep;
            for (int q = 0; q < R; ++q) {
                CHECK(i + q * nbf < n && lb + i + q * nbf < lds_elems, "stage read out of line");
                if (st > 0 && q > 0) CHECK(q * tk < n, "twiddle index %d >= n %d", q * tk, n);
            }
            for (int m = 0; m < R; ++m) {
                const int a = ob + m * p;
                CHECK(a >= lb && a < lb + n, "stage write out of line");
                if (a >= lb && a < lb + n) hit[a]++;
            }
        }
        for (int j = 0; j < nl; ++j)
            for (int x = 0; x < n; ++x) CHECK(hit[static_cast<size_t>(j) * ls + x] == 1, "stage %d not a permutation", st);
        p *= R;
    }
}

static int run_lengths()
{
    long long nlen = 0;
    for (int n = 2; n <= kFftMaxLen; n += 2) {
        int m = n;
        for (int f : {2, 3, 5})
            while (m % f == 0) m /= f;
        if (m != 1) continue;
        ++nlen;
        uint8_t rad[kMaxStages];
        const int ns = factor_radices(n, rad);
        CHECK(ns >= 1 && ns <= kMaxStages, "no radix plan for %d", n);
        if (ns < 1) continue;
        const int NT = fft_threads(n), L = fft_lines(n), ls = fft_lds_stride(n);
        CHECK(L >= 1 && L * n <= fft_elems(NT), "workgroup elements (n %d)", n);
        for (int nl : {L, (L + 1) / 2, 1}) check_stages(NT, n, nl, ls, fft_lds_elems(L, n), ns, rad);
    }
    printf("geometries %lld checks %lld errors %lld\n", nlen, g_chk, g_err);
    return g_err != 0;
}

static int run_plan(char **argv)
{
    const int64_t nv = atoll(argv[0]), np_ = atoll(argv[1]);
    std::vector<double> uvw(3 * nv), xyz(3 * np_);
    FILE *f = fopen(argv[2], "rb");
    if (!f || fread(uvw.data(), 8, uvw.size(), f) != uvw.size()) return 2;
    fclose(f);
    f = fopen(argv[3], "rb");
    if (!f || fread(xyz.data(), 8, xyz.size(), f) != xyz.size()) return 2;
    fclose(f);
    Params prm;
    prm.dtype = atoi(argv[4]);
    prm.eps = atof(argv[5]);
    prm.max_fft_bytes = atof(argv[6]);
    prm.direct_threshold = atof(argv[7]);
    prm.ws_cap = 4.0 * 1024 * 1024 * 1024;
    prm.alpha = 1.0;
    prm.all_direct = false;
    if (choose_kernels(&prm, prm.eps)) return 3;
    HostPlan hp;
    std::string err;
    if (make_host_plan(uvw.data(), nv, xyz.data(), np_, prm, nullptr, nullptr, &hp, &err)) {
        printf("plan failed: %s\n", err.c_str());
        return 3;
    }
    std::set<std::vector<int64_t>> seen;
    for (const DirPlan *dp : {&hp.syn, &hp.ana})
        for (const Batch &b : dp->batches)
            for (int pass = 0; pass < 3; ++pass) {
                const int NT = fft_threads(b.max_pass_len[pass]);
                for (int64_t pi = 0; pi < b.npairs; ++pi) {
                    const PairDev &P = dp->pairs[b.pair0 + pi];
                    // the addressing depends only on these
                    std::vector<int64_t> key = {pass, NT, b.lds_elems[pass], b.max_pass_len[pass], P.n1[0], P.n1[1],
                                                P.n1[2], P.n2[0], P.n2[1], P.n2[2], P.wstart[0], P.wstart[1],
                                                P.wstart[2], P.wcount[0], P.wcount[1], P.wcount[2],
                                                P.lines_per_tile[pass], P.ntile[0], P.ntile[1], P.tile0 & 31};
                    if (!seen.insert(key).second) continue;
                    const int n = P.n2[pass], nin = P.n1[pass], wst = P.wstart[pass], wcnt = P.wcount[pass];
                    CHECK(n <= b.max_pass_len[pass], "line longer than the batch's twiddle table");
                    const int64_t g1 = (int64_t)P.n1[0] * P.n1[1] * P.n1[2];
                    const int64_t xo = (int64_t)P.wcount[0] * P.n1[1] * P.n1[2];
                    const int64_t yo = (int64_t)P.wcount[0] * P.wcount[1] * P.n1[2];
                    const int64_t zo = (int64_t)P.wcount[0] * P.wcount[1] * P.wcount[2];
                    int64_t lines, src_size, dst_size;
                    if (pass == 0) { lines = (int64_t)P.n1[2] * P.n1[1]; src_size = g1; dst_size = xo; }
                    else if (pass == 1) { lines = (int64_t)P.n1[2] * P.wcount[0]; src_size = xo; dst_size = yo; }
                    else { lines = (int64_t)P.wcount[0] * P.wcount[1]; src_size = yo; dst_size = zo; }
                    const int L = P.lines_per_tile[pass], ls = fft_lds_stride(n), lds_elems = b.lds_elems[pass];
                    CHECK(L >= 1 && L <= kFftMaxLines && L * n <= fft_elems(NT), "lines per workgroup");
                    const int64_t tiles = (lines + L - 1) / L;
                    std::vector<int64_t> tl = {0};
                    if (tiles > 1) tl.push_back(tiles - 1);   // a full workgroup and the ragged last one
                    for (int64_t t : tl) {
                        const int64_t line0 = t * L;
                        const int nl = (int)std::min<int64_t>(L, lines - line0);
                        CHECK(nl * ls <= lds_elems, "LDS lines");
                        const int half_in = nin / 2, half_n = n / 2;
                        for (int e = 0; e < nl * n; ++e) {   // load phase
                            int j, ff;
                            if (pass < 2) { j = e / n; ff = e - j * n; }
                            else { ff = e / nl; j = e - ff * nl; }
                            const int l = ff < half_n ? ff : ff - n;
                            CHECK(j * ls + ff < lds_elems, "LDS slot");
                            if (l < -half_in || l >= half_in) continue;
                            const int64_t idx = pass < 2 ? (line0 + j) * nin + l + half_in
                                                         : line0 + (int64_t)(l + half_in) * lines + j;
                            CHECK(idx >= 0 && idx < src_size, "load out of the input grid");
                            if (pass == 0) {
                                const int64_t li = line0 + j, lz = li / P.n1[1], ly = li - lz * P.n1[1];
                                const int64_t rowbit = P.tile0 + ((lz / kTileZ) * P.ntile[1] + ly / kTileY) * P.ntile[0];
                                const int bb = (int)(rowbit & 31) + ((l + half_in) >> 5);
                                CHECK((bb >> 5) < kOccWords, "occupancy mask word");
                            }
                        }
                        check_stages(NT, n, nl, ls, lds_elems, P.nrad[pass], P.radix[pass]);
                        for (int e = 0; e < nl * wcnt; ++e) {   // window output
                            const int q = e - (e / wcnt) * wcnt;
                            int m = wst + q;
                            if (m < 0) m += n;
                            CHECK(m >= 0 && m < n, "window index");
                            CHECK(line0 * wcnt + e < dst_size, "store out of the output grid");
                        }
                    }
                    if (g_err > 20) break;
                }
            }
    printf("geometries %zu checks %lld errors %lld\n", seen.size(), g_chk, g_err);
    return g_err != 0;
}

int main(int argc, char **argv)
{
    if (argc == 2 && !strcmp(argv[1], "lengths")) return run_lengths();
    if (argc == 10 && !strcmp(argv[1], "plan")) return run_plan(argv + 2);
    fprintf(stderr, "usage: fft_index_model lengths | plan N_VIS N_PIX UVW XYZ DTYPE EPS MAX_FFT_BYTES THRESHOLD\n");
    return 2;
}
