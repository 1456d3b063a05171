// Exercises the host half of the library (pair selection, delay tables, beamforming plans)
// for a build with AddressSanitizer and UndefinedBehaviorSanitizer: the named workload shapes,
// the eight window-class geometries, seeded random geometries, capacity queries and error
// paths.  Independently of the library's own checks it verifies that every pixel's Eq. 5 (KK)
// and Eq. 4 (DAS) delay falls inside the record window the plan records for its pair and
// tile, and inside the plan's window class: the property the gather kernels rely on to keep
// their on-chip window reads in bounds.  Exit status 0 = every check passed.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/kk.h"

namespace {

int failures = 0;

#define CHECK(c)                                                               \
    do {                                                                       \
        if (!(c)) {                                                            \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                                        \
        }                                                                      \
    } while (0)

// header words of a beamforming plan (the library's plan layout)
enum { W_N = 2, W_M, W_T, W_P, W_S, W_X, W_Z, W_NXT, W_NZT, W_XPAD, W_ZPAD, W_CAP, W_MAXW, W_PB,
       W_OFF_SET, W_OFF_REC, W_OFF_A, W_OFF_B, W_OFF_LO, W_OFF_C, W_OFF_TX, W_TOTAL, W_SPLIT };

struct Case {
    int L, T, N;
    double pitch, c, fs, fc, theta_max_deg;
    int scheme, M;
    std::vector<int32_t> jl;
    int X, Z;
    double z0, t0;
};

uint64_t lcg_state = 88172645463325252ull;
double urand() {  // xorshift64, uniform in [0, 1)
    lcg_state ^= lcg_state << 13;
    lcg_state ^= lcg_state >> 7;
    lcg_state ^= lcg_state << 17;
    return (double)(lcg_state >> 11) * (1.0 / 9007199254740992.0);
}
int irand(int lo, int hi) { return lo + (int)(urand() * (hi - lo + 1)) % (hi - lo + 1); }

// window of plan word lo[tile][pair] must hold floor(q / 65536) .. floor(q / 65536) + 1 for
// every pixel's composite delay q (the window's 16-byte entries hold R[n] and R[n+1]-R[n])
void check_plan_windows(const std::vector<int32_t>& plan, bool das, int L) {
    const int32_t* w = plan.data();
    const int P = w[W_P], nxt = w[W_NXT], nzt = w[W_NZT], xpad = w[W_XPAD], zpad = w[W_ZPAD];
    const int cap = w[W_CAP], maxw = w[W_MAXW];
    CHECK(maxw >= 1 && maxw <= cap);
    CHECK(w[W_TOTAL] == (int32_t)plan.size());
    CHECK(w[W_SPLIT] >= 1 && w[W_SPLIT] <= 8);
    const int32_t* A = w + w[W_OFF_A];
    const int32_t* B = w + w[W_OFF_B];
    const int32_t* lo = w + w[W_OFF_LO];
    const int32_t* tx = w + w[W_OFF_TX];
    const int32_t* C = das ? w + w[W_OFF_C] : nullptr;
    for (int zt = 0; zt < nzt; ++zt)
        for (int xt = 0; xt < nxt; ++xt) {
            const int64_t tile = (int64_t)zt * nxt + xt;
            for (int p = 0; p < P; ++p) {
                const int row = das ? tx[p] : p;  // DAS: folded transmit delays per transmit
                const int l = das ? p / w[W_N] : 0;
                const int64_t first = lo[tile * P + p];
                for (int z = zt * 16; z < zt * 16 + 16; ++z)
                    for (int x = xt * 64; x < xt * 64 + 64; ++x) {
                        int64_t q = (int64_t)A[(int64_t)row * xpad + x] + B[(int64_t)row * zpad + z];
                        if (das) q += C[((int64_t)l * zpad + z) * xpad + x];
                        const int64_t idx = q >> 16;
                        if (idx < first || idx - first >= maxw) {
                            ++failures;
                            if (failures < 5)
                                std::fprintf(stderr, "window miss: tile %lld pair %d pixel (%d, %d) idx %lld lo %lld\n",
                                             (long long)tile, p, x, z, (long long)idx, (long long)first);
                        }
                    }
            }
        }
    (void)L;
}

void run_case(const Case& k, bool with_das) {
    const double th = k.theta_max_deg * 3.14159265358979323846 / 180.0;
    std::vector<double> tx(k.N);
    int32_t Md = 0, P = 0, S = 0;
    double comp = 0;
    // size query with zero capacities
    int st = kk_select_pairs(k.scheme, k.L, k.N, th, k.M, k.jl.data(), (int)k.jl.size(), tx.data(), nullptr,
                             nullptr, nullptr, 0, &Md, nullptr, 0, &P, &S, &comp);
    CHECK(st == KK_E_CAPACITY);
    std::vector<double> rx(Md);
    std::vector<int32_t> num(Md), den(Md), pairs(3 * (size_t)P);
    st = kk_select_pairs(k.scheme, k.L, k.N, th, k.M, k.jl.data(), (int)k.jl.size(), tx.data(), rx.data(),
                         num.data(), den.data(), Md, &Md, pairs.data(), P, &P, &S, &comp);
    CHECK(st == KK_OK);
    if (st != KK_OK) return;
    const double lam = k.c / k.fc;
    kk_geom g{k.L, k.T, k.pitch, k.c, k.fs, k.t0};
    kk_grid gr{k.X, k.Z, -((k.X - 1) * (lam / 2)) / 2.0, lam / 2, k.z0, lam / 2};
    std::vector<int32_t> l1((size_t)k.N * k.X), l2((size_t)k.N * k.Z), l3((size_t)Md * k.X), l4((size_t)Md * k.Z),
        sh((size_t)Md * k.L);
    int32_t t0q = 0, tpad = 0;
    st = kk_build_luts(&g, &gr, tx.data(), k.N, rx.data(), Md, l1.data(), l2.data(), l3.data(), l4.data(), &t0q,
                       sh.data(), &tpad);
    CHECK(st == KK_OK);
    if (st != KK_OK) return;
    CHECK(tpad >= k.T && (tpad & (tpad - 1)) == 0);
    size_t need = 0;
    st = kk_beamform_plan(pairs.data(), P, S, k.N, Md, k.T, l1.data(), l2.data(), l3.data(), l4.data(), t0q, &gr,
                          nullptr, 0, &need);
    CHECK(st == KK_E_CAPACITY || st == KK_E_UNSUPPORTED);
    if (st == KK_E_CAPACITY) {
        std::vector<int32_t> plan(need / 4);
        // one word short: capacity error, nothing written past the buffer
        st = kk_beamform_plan(pairs.data(), P, S, k.N, Md, k.T, l1.data(), l2.data(), l3.data(), l4.data(), t0q,
                              &gr, plan.data(), need - 4, &need);
        CHECK(st == KK_E_CAPACITY);
        st = kk_beamform_plan(pairs.data(), P, S, k.N, Md, k.T, l1.data(), l2.data(), l3.data(), l4.data(), t0q,
                              &gr, plan.data(), need, &need);
        CHECK(st == KK_OK);
        if (st == KK_OK) check_plan_windows(plan, false, k.L);
    }
    if (!with_das) return;
    std::vector<int32_t> das_rx((size_t)k.X * k.L * k.Z);
    st = kk_build_das_rx(&g, &gr, das_rx.data());
    CHECK(st == KK_OK);
    if (st != KK_OK) return;
    st = das_plan(k.N, &g, l1.data(), l2.data(), das_rx.data(), t0q, &gr, nullptr, 0, &need);
    CHECK(st == KK_E_CAPACITY || st == KK_E_UNSUPPORTED);
    if (st == KK_E_CAPACITY) {
        std::vector<int32_t> plan(need / 4);
        st = das_plan(k.N, &g, l1.data(), l2.data(), das_rx.data(), t0q, &gr, plan.data(), need, &need);
        CHECK(st == KK_OK);
        if (st == KK_OK) check_plan_windows(plan, true, k.L);
    }
}

void error_paths() {
    double tx[4], rx[8];
    int32_t num[8], den[8], pairs[3 * 64], Md, P, S;
    double comp;
    const int32_t j0 = 0, jbad = 9;
    CHECK(kk_select_pairs(0, 16, 4, 0.2, 3, &j0, 1, nullptr, rx, num, den, 8, &Md, pairs, 64, &P, &S, &comp) ==
          KK_E_NULL);
    CHECK(kk_select_pairs(0, 16, 1, 0.2, 3, &j0, 1, tx, rx, num, den, 8, &Md, pairs, 64, &P, &S, &comp) == KK_E_ARG);
    CHECK(kk_select_pairs(0, 16, 4, 0.2, 3, &jbad, 1, tx, rx, num, den, 8, &Md, pairs, 64, &P, &S, &comp) ==
          KK_E_ARG);
    CHECK(kk_select_pairs(9, 16, 4, 0.2, 3, &j0, 1, tx, rx, num, den, 8, &Md, pairs, 64, &P, &S, &comp) == KK_E_ARG);
    CHECK(kk_select_pairs(0, 16, 4, 1.6, 3, &j0, 1, tx, rx, num, den, 8, &Md, pairs, 64, &P, &S, &comp) == KK_E_ARG);
    CHECK(kk_select_pairs(1, 16, 4, 0.2, 3, nullptr, 0, tx, rx, num, den, 8, &Md, pairs, 64, &P, &S, &comp) ==
          KK_OK);
    kk_geom g{16, 1024, 0.3e-3, 1540.0, 20e6, 0.0};
    kk_grid gr{64, 64, -0.005, 1.54e-4, 0.01, 1.54e-4};
    int32_t l[64 * 64], t0q, tp;
    kk_geom bad = g;
    bad.c_mps = -1.0;
    CHECK(kk_build_luts(&bad, &gr, tx, 1, rx, 1, l, l, l, l, &t0q, nullptr, &tp) == KK_E_ARG);
    CHECK(kk_build_luts(nullptr, &gr, tx, 1, rx, 1, l, l, l, l, &t0q, nullptr, &tp) == KK_E_NULL);
    bad = g;
    bad.fs_hz = 2e12;
    tx[0] = rx[0] = 0.1;
    CHECK(kk_build_luts(&bad, &gr, tx, 1, rx, 1, l, l, l, l, &t0q, nullptr, &tp) == KK_E_RANGE);
    size_t need = 0;
    const int32_t bad_pair[3] = {0, 5, 0};  // receive index beyond M
    CHECK(kk_beamform_plan(bad_pair, 1, 1, 1, 1, 1024, l, l, l, l, 0, &gr, nullptr, 0, &need) == KK_E_ARG);
    CHECK(kk_beamform_plan(nullptr, 1, 1, 1, 1, 1024, l, l, l, l, 0, &gr, nullptr, 0, &need) == KK_E_NULL);
    for (int s = -8; s <= 0; ++s) CHECK(kk_status_string(s) != nullptr && std::strlen(kk_status_string(s)) > 0);
    CHECK(kk_status_string(42) != nullptr);
}

}  // namespace

int main() {
    const double c = 1540.0, fs = 20e6;
    std::vector<Case> cases;
    // named shapes: tiny (16 el, 1024 samples, 5 tx, 16-angle bank, 64 x 64), vernier (128 el,
    // 2048 samples, 31 tx, Eq. 6 j = 0, 15, 256 x 512), a reduced large shape
    cases.push_back({16, 1024, 5, 0.3e-3, c, fs, 5e6, 10.0, 3, 16, {0}, 64, 64, 0.01, 0.0});
    cases.push_back({128, 2048, 31, 0.3e-3, c, fs, 5e6, 15.0, 0, 7, {0, 15}, 256, 512, 0.0, 0.0});
    cases.push_back({192, 4096, 75, 0.3e-3, c, fs, 5e6, 18.0, 0, 9, {0, 37}, 96, 160, 0.0, 0.0});
    // one geometry per window class (centre frequency sets the pixel pitch lambda / 2)
    const double fcs[8] = {20e6, 10e6, 5e6, 3.5e6, 3.5e6, 2.5e6, 2e6, 1.6e6};
    const double fans[8] = {10.0, 20.0, 20.0, 20.0, 35.0, 25.0, 20.0, 20.0};
    for (int k = 0; k < 8; ++k)
        cases.push_back({16, 1024, 5, 0.3e-3, c, fs, fcs[k], fans[k], k == 0 || k == 3 ? 3 : 0, k == 0 || k == 3 ? 16 : 7,
                         k == 0 || k == 3 ? std::vector<int32_t>{0} : std::vector<int32_t>{0, 2}, 64, 64, 0.01, 0.0});
    // seeded random small geometries: ragged grids, early and late record starts, all schemes
    for (int r = 0; r < 40; ++r) {
        Case k;
        k.L = irand(2, 40);
        k.N = irand(2, 15);
        k.T = irand(64, 1500);
        k.pitch = 0.2e-3 + 0.2e-3 * urand();
        k.c = c;
        k.fs = fs;
        k.fc = 1.8e6 + 8e6 * urand();
        k.theta_max_deg = 3.0 + 25.0 * urand();
        k.scheme = irand(0, 3);
        k.M = k.scheme == 3 ? irand(2, 20) : 2 * irand(0, 5) + 1;
        k.jl.clear();
        const int J = irand(1, 3);
        for (int j = 0; j < J; ++j) k.jl.push_back(irand(0, k.N / 2));
        k.X = irand(1, 150);
        k.Z = irand(1, 90);
        k.z0 = 1e-3 + 15e-3 * urand();
        k.t0 = -2e-6 + 6e-6 * urand();
        cases.push_back(k);
    }
    int n = 0;
    for (const Case& k : cases) {
        run_case(k, k.L <= 64 && (int64_t)k.X * k.Z * k.L <= 2000000);
        ++n;
    }
    error_paths();
    std::printf("host driver: %d geometries, %d failures\n", n, failures);
    return failures == 0 ? 0 : 1;
}
