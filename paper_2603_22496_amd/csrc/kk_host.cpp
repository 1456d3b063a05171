// Host half of the KK beamforming library: receive-angle selection (Sec. II-C/D, Eq. 6/7),
// FP64 delay tables (Sec. II-F), and the per-geometry beamforming plans.
//
// Built with -O2 -ffp-contract=off and without fast-math: every FP64 expression below is
// evaluated exactly in the order written (one IEEE operation at a time), so the integer
// tables are reproducible bit for bit.  rint = round half to even (default rounding mode).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>

#include "../../include/kk.h"
#include "kk_plan.h"

namespace {

constexpr double kQ16 = 65536.0;
constexpr double kQ22 = 4194304.0;
constexpr double kHalfPi = 1.5707963267948966;  // pi / 2 rounded to FP64

struct Rational {
    int64_t num, den;  // den > 0, lowest terms
};

int64_t gcd64(int64_t a, int64_t b) {
    a = a < 0 ? -a : a;
    b = b < 0 ? -b : b;
    while (b) {
        int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

Rational make_rational(int64_t n, int64_t d) {
    if (d < 0) {
        n = -n;
        d = -d;
    }
    if (n == 0) return {0, 1};
    int64_t g = gcd64(n, d);
    return {n / g, d / g};
}

bool rational_less(const Rational& a, const Rational& b) { return a.num * b.den < b.num * a.den; }
bool rational_equal(const Rational& a, const Rational& b) { return a.num == b.num && a.den == b.den; }

int sgn(int o) { return (o > 0) - (o < 0); }

// Round half to even and range check into int32.
bool rint32(double v, int32_t* out) {
    if (!(v == v)) return false;
    double r = std::nearbyint(v);
    if (r < -2147483648.0 || r > 2147483647.0) return false;
    *out = (int32_t)r;
    return true;
}

double element_x(int32_t l, int32_t L, double pitch) { return ((double)(2 * l - (L - 1)) * pitch) / 2.0; }

bool geom_ok(const kk_geom* g) {
    return g->L >= 1 && g->T >= 1 && g->pitch_m > 0.0 && g->c_mps > 0.0 && g->fs_hz > 0.0 &&
           std::isfinite(g->t0_s) && std::isfinite(g->pitch_m) && std::isfinite(g->c_mps) &&
           std::isfinite(g->fs_hz);
}

bool grid_ok(const kk_grid* gr) {
    return gr->X >= 1 && gr->Z >= 1 && gr->dx_m > 0.0 && gr->dz_m > 0.0 && std::isfinite(gr->x0_m) &&
           std::isfinite(gr->z0_m) && std::isfinite(gr->dx_m) && std::isfinite(gr->dz_m);
}

int32_t next_pow2(int64_t n) {
    int64_t p = 1;
    while (p < n) p *= 2;
    return p > 0x40000000 ? -1 : (int32_t)p;
}

}  // namespace

extern "C" {

const char* kk_status_string(int32_t s) {
    switch (s) {
        case KK_OK: return "KK_OK";
        case KK_E_NULL: return "KK_E_NULL: required pointer is NULL";
        case KK_E_ARG: return "KK_E_ARG: argument out of range";
        case KK_E_CAPACITY: return "KK_E_CAPACITY: output too small";
        case KK_E_WORKSPACE: return "KK_E_WORKSPACE: workspace or plan too small or invalid";
        case KK_E_RANGE: return "KK_E_RANGE: delay outside int32 fixed point";
        case KK_E_HIP: return "KK_E_HIP: HIP runtime error";
        case KK_E_UNSUPPORTED: return "KK_E_UNSUPPORTED: not implemented for these arguments";
        default: return "unknown kk_status";
    }
}

int32_t kk_select_pairs(int32_t scheme, int32_t L, int32_t N, double theta_max, int32_t M,
                        const int32_t* j_list, int32_t J, double* tx_theta, double* rx_theta,
                        int32_t* rx_num, int32_t* rx_den, int32_t cap_rx, int32_t* M_out,
                        int32_t* pairs, int32_t cap_p, int32_t* P_out, int32_t* S_out,
                        double* compression) {
    if (!tx_theta || !M_out || !P_out || !S_out || !compression) return KK_E_NULL;
    if (N < 2 || L < 1 || N > 100000 || L > 1000000) return KK_E_ARG;
    if (!(theta_max > 0.0 && theta_max < kHalfPi)) return KK_E_ARG;
    if (scheme != KK_SCHEME_SAME && (M < 1 || M > 100000)) return KK_E_ARG;
    const double dth = (2.0 * theta_max) / (double)(N - 1);

    struct Entry {
        Rational r;
        double th;
    };
    std::vector<std::vector<Entry>> sets;
    switch (scheme) {
        case KK_SCHEME_SHIFTED: {
            if (!j_list) return KK_E_NULL;
            if (J < 1 || J > 4096) return KK_E_ARG;
            const int h = M / 2;
            for (int32_t s = 0; s < J; ++s) {
                const int32_t j = j_list[s];
                if (j < 0 || j > N / 2) return KK_E_ARG;
                std::vector<Entry> st;
                for (int o = -h; o <= h; ++o) {
                    const int64_t n = (int64_t)sgn(o) * (2 * (int64_t)std::abs(o) + (int64_t)j * M);
                    st.push_back({make_rational(n, M), ((double)n * dth) / (double)M});
                }
                sets.push_back(st);
            }
            break;
        }
        case KK_SCHEME_CONFOCAL: {
            const int h = M / 2, hn = N / 2;
            std::vector<Entry> st;
            for (int o = -h; o <= h; ++o) {
                const int a = std::abs(o);
                const int64_t n = (int64_t)sgn(o) * (2 * (int64_t)a + (int64_t)(a % hn) * M);
                st.push_back({make_rational(n, M), ((double)n * dth) / (double)M});
            }
            sets.push_back(st);
            break;
        }
        case KK_SCHEME_SAME: {
            std::vector<Entry> st;
            for (int32_t i = 0; i < N; ++i)
                st.push_back({make_rational(2 * (int64_t)i - (N - 1), 2),
                              ((double)(2 * i - (N - 1)) * theta_max) / (double)(N - 1)});
            sets.push_back(st);
            break;
        }
        case KK_SCHEME_FULL_UNIFORM: {
            if (M < 2) return KK_E_ARG;
            const double th_hi = theta_max + dth;
            std::vector<Entry> st;
            for (int32_t k = 0; k < M; ++k)
                st.push_back({make_rational((2 * (int64_t)k - (M - 1)) * (int64_t)(N + 1), 2 * (int64_t)(M - 1)),
                              ((double)(2 * k - (M - 1)) * th_hi) / (double)(M - 1)});
            sets.push_back(st);
            break;
        }
        default:
            return KK_E_ARG;
    }
    for (auto& st : sets)
        for (auto& e : st)
            if (!(std::fabs(e.th) < kHalfPi)) return KK_E_ARG;

    // distinct receive angles: first occurrence of each rational, sorted by value
    std::vector<Entry> distinct;
    for (auto& st : sets)
        for (auto& e : st) {
            bool seen = false;
            for (auto& d : distinct)
                if (rational_equal(d.r, e.r)) {
                    seen = true;
                    break;
                }
            if (!seen) distinct.push_back(e);
        }
    std::stable_sort(distinct.begin(), distinct.end(),
                     [](const Entry& a, const Entry& b) { return rational_less(a.r, b.r); });
    const int64_t Md = (int64_t)distinct.size();
    int64_t P = 0;
    for (auto& st : sets) P += (int64_t)st.size() * N;
    *M_out = (int32_t)Md;
    *P_out = P > 0x7fffffff ? 0x7fffffff : (int32_t)P;
    *S_out = (int32_t)sets.size();
    *compression = (double)L / ((double)sets.size() * (double)sets[0].size());
    if (cap_rx < Md || cap_p < P) return KK_E_CAPACITY;
    if (!rx_theta || !rx_num || !rx_den || !pairs) return KK_E_NULL;
    if (Md > 0x7fffffff / 2) return KK_E_ARG;

    for (int32_t i = 0; i < N; ++i) tx_theta[i] = ((double)(2 * i - (N - 1)) * theta_max) / (double)(N - 1);
    for (int64_t o = 0; o < Md; ++o) {
        rx_theta[o] = distinct[o].th;
        rx_num[o] = (int32_t)distinct[o].r.num;
        rx_den[o] = (int32_t)distinct[o].r.den;
    }
    int64_t w = 0;
    for (size_t s = 0; s < sets.size(); ++s) {
        std::vector<int32_t> idx;
        for (auto& e : sets[s])
            for (int64_t o = 0; o < Md; ++o)
                if (rational_equal(distinct[o].r, e.r)) {
                    idx.push_back((int32_t)o);
                    break;
                }
        std::sort(idx.begin(), idx.end());
        for (int32_t o : idx)
            for (int32_t i = 0; i < N; ++i) {
                pairs[3 * w + 0] = i;
                pairs[3 * w + 1] = o;
                pairs[3 * w + 2] = (int32_t)s;
                ++w;
            }
    }
    return KK_OK;
}

int32_t kk_build_luts(const kk_geom* g, const kk_grid* gr, const double* tx_theta, int32_t N,
                      const double* rx_theta, int32_t M, int32_t* lut1, int32_t* lut2, int32_t* lut3,
                      int32_t* lut4, int32_t* t0_q, int32_t* shift_q, int32_t* tpad) {
    if (!g || !gr || !tx_theta || !rx_theta) return KK_E_NULL;
    if (!geom_ok(g) || !grid_ok(gr) || N < 1 || M < 1) return KK_E_ARG;
    const int32_t L = g->L, X = gr->X, Z = gr->Z;
    const double c = g->c_mps, fs = g->fs_hz;
    std::vector<double> xs(X), zs(Z), u(L);
    for (int32_t k = 0; k < X; ++k) xs[k] = gr->x0_m + (double)k * gr->dx_m;
    for (int32_t k = 0; k < Z; ++k) zs[k] = gr->z0_m + (double)k * gr->dz_m;
    for (int32_t l = 0; l < L; ++l) u[l] = element_x(l, L, g->pitch_m);

    std::vector<int32_t> l1((size_t)N * X), l2((size_t)N * Z), l3((size_t)M * X), l4((size_t)M * Z),
        sh((size_t)M * L);
    for (int32_t i = 0; i < N; ++i) {
        const double s = std::sin(tx_theta[i]), co = std::cos(tx_theta[i]);
        for (int32_t k = 0; k < X; ++k)
            if (!rint32((((xs[k] * s) / c) * fs) * kQ16, &l1[(size_t)i * X + k])) return KK_E_RANGE;
        for (int32_t k = 0; k < Z; ++k)
            if (!rint32((((zs[k] * co) / c) * fs) * kQ16, &l2[(size_t)i * Z + k])) return KK_E_RANGE;
    }
    for (int32_t o = 0; o < M; ++o) {
        const double th = rx_theta[o];
        const double s = std::sin(th), co = std::cos(th);
        const double xr = th >= 0.0 ? u[0] : u[L - 1];
        for (int32_t k = 0; k < X; ++k)
            if (!rint32((((-(xs[k] - xr) * s) / c) * fs) * kQ16, &l3[(size_t)o * X + k])) return KK_E_RANGE;
        for (int32_t k = 0; k < Z; ++k)
            if (!rint32((((zs[k] * co) / c) * fs) * kQ16, &l4[(size_t)o * Z + k])) return KK_E_RANGE;
        const double ref = th > 0.0 ? u[0] : (th < 0.0 ? u[L - 1] : 0.0);
        for (int32_t l = 0; l < L; ++l) {
            const double d = u[l] - ref;
            if (!rint32((((d * s) / c) * fs) * kQ22, &sh[(size_t)o * L + l])) return KK_E_RANGE;
        }
    }
    int32_t t0 = 0;
    if (!rint32(((-g->t0_s) * fs) * kQ16, &t0)) return KK_E_RANGE;

    // composite delays lut1 + lut2 + lut3 + lut4 + t0 must fit int32 for every combination
    auto ext = [](const std::vector<int32_t>& v, int64_t* lo, int64_t* hi) {
        *lo = *std::min_element(v.begin(), v.end());
        *hi = *std::max_element(v.begin(), v.end());
    };
    int64_t a0, a1, b0, b1, c0, c1, d0, d1;
    ext(l1, &a0, &a1);
    ext(l2, &b0, &b1);
    ext(l3, &c0, &c1);
    ext(l4, &d0, &d1);
    if (a0 + b0 + c0 + d0 + t0 < INT32_MIN || a1 + b1 + c1 + d1 + t0 > INT32_MAX) return KK_E_RANGE;

    int64_t smax = 0;
    for (int32_t v : sh) smax = std::max<int64_t>(smax, v);
    const int64_t s_samples = (smax + (1 << 22) - 1) >> 22;
    const int32_t tp = next_pow2((int64_t)g->T + s_samples);
    if (tp < 0) return KK_E_RANGE;

    if (lut1) std::memcpy(lut1, l1.data(), l1.size() * 4);
    if (lut2) std::memcpy(lut2, l2.data(), l2.size() * 4);
    if (lut3) std::memcpy(lut3, l3.data(), l3.size() * 4);
    if (lut4) std::memcpy(lut4, l4.data(), l4.size() * 4);
    if (shift_q) std::memcpy(shift_q, sh.data(), sh.size() * 4);
    if (t0_q) *t0_q = t0;
    if (tpad) *tpad = tp;
    return KK_OK;
}

int32_t kk_build_das_rx(const kk_geom* g, const kk_grid* gr, int32_t* das_rx) {
    if (!g || !gr || !das_rx) return KK_E_NULL;
    if (!geom_ok(g) || !grid_ok(gr)) return KK_E_ARG;
    const int32_t L = g->L, X = gr->X, Z = gr->Z;
    const double c = g->c_mps, fs = g->fs_hz;
    std::vector<double> zs(Z), u(L);
    for (int32_t k = 0; k < Z; ++k) zs[k] = gr->z0_m + (double)k * gr->dz_m;
    for (int32_t l = 0; l < L; ++l) u[l] = element_x(l, L, g->pitch_m);
    int32_t status = KK_OK;
#pragma omp parallel for schedule(static)
    for (int32_t k = 0; k < X; ++k) {
        const double x = gr->x0_m + (double)k * gr->dx_m;
        for (int32_t l = 0; l < L; ++l) {
            const double d = x - u[l];
            const double dd = d * d;
            int32_t* row = das_rx + ((size_t)k * L + l) * Z;
            for (int32_t m = 0; m < Z; ++m) {
                const double r = std::sqrt(dd + zs[m] * zs[m]);
                if (!rint32(((r / c) * fs) * kQ16, &row[m])) {
#pragma omp atomic write
                    status = KK_E_RANGE;
                }
            }
        }
    }
    return status;
}

}  // extern "C"

// ------------------------------------------------------------------------------ plans

namespace {

int32_t pick_cap(int64_t max_w) {
    for (int32_t i = 0; i < kk::kNumCaps; ++i)
        if (max_w <= kk::kCaps[i]) return kk::kCaps[i];
    return -1;
}

int64_t floor_div65536(int64_t q) { return q >> 16; }  // arithmetic shift = floor for int64

// Pair shares per (set, tile): enough workgroups to cover the CUs while every share keeps at
// least two batches of pairs.
int32_t choose_split(int64_t units, int64_t min_set_pairs, int32_t pb) {
    int32_t k = 1;
    while (k < kk::kMaxSplit && units * k < kk::kTargetWorkgroups && min_set_pairs >= (int64_t)(k + 1) * 2 * pb) ++k;
    return k;
}

}  // namespace

extern "C" {

int32_t kk_beamform_plan(const int32_t* pairs, int32_t P, int32_t S, int32_t N, int32_t M, int32_t T,
                         const int32_t* lut1, const int32_t* lut2, const int32_t* lut3, const int32_t* lut4,
                         int32_t t0_q, const kk_grid* gr, void* plan, size_t plan_bytes,
                         size_t* plan_bytes_out) {
    using namespace kk;
    if (!pairs || !lut1 || !lut2 || !lut3 || !lut4 || !gr || !plan_bytes_out) return KK_E_NULL;
    if (P < 1 || S < 1 || N < 1 || M < 1 || T < 1 || !grid_ok(gr)) return KK_E_ARG;
    const int32_t X = gr->X, Z = gr->Z;
    const int32_t nxt = (X + kTileX - 1) / kTileX, nzt = (Z + kTileZ - 1) / kTileZ;
    const int64_t xpad = (int64_t)nxt * kTileX, zpad = (int64_t)nzt * kTileZ, ntiles = (int64_t)nxt * nzt;

    // group pairs by set (stable)
    std::vector<int32_t> order;
    std::vector<int32_t> set_start(S + 1, 0);
    for (int32_t p = 0; p < P; ++p) {
        const int32_t i = pairs[3 * p], o = pairs[3 * p + 1], s = pairs[3 * p + 2];
        if (i < 0 || i >= N || o < 0 || o >= M || s < 0 || s >= S) return KK_E_ARG;
        set_start[s + 1]++;
    }
    for (int32_t s = 0; s < S; ++s) {
        if (set_start[s + 1] == 0) return KK_E_ARG;
        set_start[s + 1] += set_start[s];
    }
    for (int32_t s = 0; s < S; ++s)
        for (int32_t p = 0; p < P; ++p)
            if (pairs[3 * p + 2] == s) order.push_back(p);

    const int64_t words = PW_HEADER_WORDS + (S + 1) + 2 * (int64_t)P + (int64_t)P * xpad + (int64_t)P * zpad +
                          ntiles * P;
    *plan_bytes_out = (size_t)words * 4;
    if (words > 0x7fffffff) return KK_E_ARG;

    // folded delays; composite A + B must fit int32 (checked on the extremes)
    std::vector<int32_t> A((size_t)P * xpad), B((size_t)P * zpad);
    for (int32_t q = 0; q < P; ++q) {
        const int32_t p = order[q], i = pairs[3 * p], o = pairs[3 * p + 1];
        for (int64_t k = 0; k < xpad; ++k) {
            const int64_t kk = k < X ? k : X - 1;
            const int64_t v = (int64_t)lut1[(size_t)i * X + kk] + lut3[(size_t)o * X + kk] + t0_q;
            if (v < INT32_MIN || v > INT32_MAX) return KK_E_RANGE;
            A[(size_t)q * xpad + k] = (int32_t)v;
        }
        for (int64_t k = 0; k < zpad; ++k) {
            const int64_t kk = k < Z ? k : Z - 1;
            const int64_t v = (int64_t)lut2[(size_t)i * Z + kk] + lut4[(size_t)o * Z + kk];
            if (v < INT32_MIN || v > INT32_MAX) return KK_E_RANGE;
            B[(size_t)q * zpad + k] = (int32_t)v;
        }
    }
    // exact per-tile extremes: the composite delay is separable, so
    // min over the tile = min_x A + min_z B (same for max)
    std::vector<int64_t> amin((size_t)P * nxt), amax((size_t)P * nxt), bmin((size_t)P * nzt), bmax((size_t)P * nzt);
    for (int32_t q = 0; q < P; ++q) {
        for (int32_t t = 0; t < nxt; ++t) {
            const int32_t* a = &A[(size_t)q * xpad + (size_t)t * kTileX];
            amin[(size_t)q * nxt + t] = *std::min_element(a, a + kTileX);
            amax[(size_t)q * nxt + t] = *std::max_element(a, a + kTileX);
        }
        for (int32_t t = 0; t < nzt; ++t) {
            const int32_t* b = &B[(size_t)q * zpad + (size_t)t * kTileZ];
            bmin[(size_t)q * nzt + t] = *std::min_element(b, b + kTileZ);
            bmax[(size_t)q * nzt + t] = *std::max_element(b, b + kTileZ);
        }
    }
    std::vector<int32_t> lo((size_t)ntiles * P);
    int64_t max_w = 0;
    for (int32_t zt = 0; zt < nzt; ++zt)
        for (int32_t xt = 0; xt < nxt; ++xt) {
            const int64_t tile = (int64_t)zt * nxt + xt;
            for (int32_t q = 0; q < P; ++q) {
                const int64_t qlo = amin[(size_t)q * nxt + xt] + bmin[(size_t)q * nzt + zt];
                const int64_t qhi = amax[(size_t)q * nxt + xt] + bmax[(size_t)q * nzt + zt];
                if (qlo < INT32_MIN || qhi > INT32_MAX) return KK_E_RANGE;
                const int64_t first = floor_div65536(qlo), last = floor_div65536(qhi);
                max_w = std::max(max_w, last - first + 1);
                lo[(size_t)tile * P + q] = (int32_t)first;
            }
        }
    const int32_t cap = pick_cap(max_w);
    if (cap < 0) return KK_E_UNSUPPORTED;
    if (!plan || plan_bytes < (size_t)words * 4) return KK_E_CAPACITY;

    int32_t* w = (int32_t*)plan;
    std::memset(w, 0, (size_t)PW_HEADER_WORDS * 4);
    int64_t off = PW_HEADER_WORDS;
    w[PW_MAGIC] = kPlanMagic;
    w[PW_KIND] = kPlanKindKK;
    w[PW_N] = N;
    w[PW_M] = M;
    w[PW_T] = T;
    w[PW_P] = P;
    w[PW_S] = S;
    w[PW_X] = X;
    w[PW_Z] = Z;
    w[PW_NXT] = nxt;
    w[PW_NZT] = nzt;
    w[PW_XPAD] = (int32_t)xpad;
    w[PW_ZPAD] = (int32_t)zpad;
    w[PW_CAP] = cap;
    w[PW_MAXW] = (int32_t)max_w;
    w[PW_PB] = pairs_per_batch(cap);
    w[PW_OFF_SET] = (int32_t)off;
    for (int32_t s = 0; s <= S; ++s) w[off++] = set_start[s];
    w[PW_OFF_REC] = (int32_t)off;
    for (int32_t q = 0; q < P; ++q) w[off++] = pairs[3 * order[q]] * M + pairs[3 * order[q] + 1];
    w[PW_OFF_TX] = (int32_t)off;
    for (int32_t q = 0; q < P; ++q) w[off++] = q;
    w[PW_OFF_A] = (int32_t)off;
    std::memcpy(w + off, A.data(), A.size() * 4);
    off += (int64_t)A.size();
    w[PW_OFF_B] = (int32_t)off;
    std::memcpy(w + off, B.data(), B.size() * 4);
    off += (int64_t)B.size();
    w[PW_OFF_LO] = (int32_t)off;
    std::memcpy(w + off, lo.data(), lo.size() * 4);
    off += (int64_t)lo.size();
    w[PW_OFF_C] = 0;
    w[PW_TOTAL] = (int32_t)off;
    int64_t min_set = P;
    for (int32_t s = 0; s < S; ++s) min_set = std::min<int64_t>(min_set, set_start[s + 1] - set_start[s]);
    w[PW_SPLIT] = choose_split(ntiles * S, min_set, pairs_per_batch(cap));
    return off == words ? KK_OK : KK_E_ARG;
}

int32_t das_plan(int32_t N, const kk_geom* g, const int32_t* lut1, const int32_t* lut2, const int32_t* das_rx,
                 int32_t t0_q, const kk_grid* gr, void* plan, size_t plan_bytes, size_t* plan_bytes_out) {
    using namespace kk;
    if (!g || !lut1 || !lut2 || !das_rx || !gr || !plan_bytes_out) return KK_E_NULL;
    if (N < 1 || !geom_ok(g) || !grid_ok(gr)) return KK_E_ARG;
    const int32_t L = g->L, T = g->T, X = gr->X, Z = gr->Z;
    const int32_t nxt = (X + kTileX - 1) / kTileX, nzt = (Z + kTileZ - 1) / kTileZ;
    const int64_t xpad = (int64_t)nxt * kTileX, zpad = (int64_t)nzt * kTileZ, ntiles = (int64_t)nxt * nzt;
    const int64_t P = (int64_t)N * L;
    const int64_t words = PW_HEADER_WORDS + 2 + 2 * P + (int64_t)N * xpad + (int64_t)N * zpad + ntiles * P +
                          (int64_t)L * zpad * xpad;
    *plan_bytes_out = (size_t)words * 4;
    if (words > 0x7fffffff) return KK_E_ARG;

    std::vector<int32_t> A((size_t)N * xpad), B((size_t)N * zpad), C((size_t)L * zpad * xpad);
    for (int32_t i = 0; i < N; ++i) {
        for (int64_t k = 0; k < xpad; ++k) {
            const int64_t v = (int64_t)lut1[(size_t)i * X + (k < X ? k : X - 1)] + t0_q;
            if (v < INT32_MIN || v > INT32_MAX) return KK_E_RANGE;
            A[(size_t)i * xpad + k] = (int32_t)v;
        }
        for (int64_t k = 0; k < zpad; ++k) B[(size_t)i * zpad + k] = lut2[(size_t)i * Z + (k < Z ? k : Z - 1)];
    }
    for (int32_t l = 0; l < L; ++l)
        for (int64_t m = 0; m < zpad; ++m)
            for (int64_t k = 0; k < xpad; ++k)
                C[((size_t)l * zpad + m) * xpad + k] =
                    das_rx[((size_t)(k < X ? k : X - 1) * L + l) * Z + (m < Z ? m : Z - 1)];

    // exact per (transmit, element, tile) extremes of A + B + C over the tile
    std::vector<int32_t> lo((size_t)ntiles * P);
    int64_t max_w = 0;
    int32_t status = KK_OK;
#pragma omp parallel for schedule(dynamic) reduction(max : max_w)
    for (int64_t tile = 0; tile < ntiles; ++tile) {
        const int64_t zt = tile / nxt, xt = tile % nxt;
        std::vector<int64_t> ab_lo(kTileZ * kTileX), ab_hi(kTileZ * kTileX);
        for (int32_t l = 0; l < L; ++l) {
            for (int32_t i = 0; i < N; ++i) {
                int64_t qlo = INT64_MAX, qhi = INT64_MIN;
                for (int32_t m = 0; m < kTileZ; ++m) {
                    const int64_t b = B[(size_t)i * zpad + zt * kTileZ + m];
                    const int32_t* crow = &C[((size_t)l * zpad + zt * kTileZ + m) * xpad + xt * kTileX];
                    const int32_t* arow = &A[(size_t)i * xpad + xt * kTileX];
                    for (int32_t k = 0; k < kTileX; ++k) {
                        const int64_t q = (int64_t)arow[k] + b + crow[k];
                        qlo = q < qlo ? q : qlo;
                        qhi = q > qhi ? q : qhi;
                    }
                }
                if (qlo < INT32_MIN || qhi > INT32_MAX) {
#pragma omp atomic write
                    status = KK_E_RANGE;
                }
                const int64_t first = floor_div65536(qlo), last = floor_div65536(qhi);
                max_w = std::max(max_w, last - first + 1);
                lo[(size_t)tile * P + (size_t)l * N + i] = (int32_t)first;
            }
        }
    }
    if (status != KK_OK) return status;
    const int32_t cap = pick_cap(max_w);
    if (cap < 0) return KK_E_UNSUPPORTED;
    if (!plan || plan_bytes < (size_t)words * 4) return KK_E_CAPACITY;

    int32_t* w = (int32_t*)plan;
    std::memset(w, 0, (size_t)PW_HEADER_WORDS * 4);
    int64_t off = PW_HEADER_WORDS;
    w[PW_MAGIC] = kPlanMagic;
    w[PW_KIND] = kPlanKindDAS;
    w[PW_N] = N;
    w[PW_M] = L;
    w[PW_T] = T;
    w[PW_P] = (int32_t)P;
    w[PW_S] = 1;
    w[PW_X] = X;
    w[PW_Z] = Z;
    w[PW_NXT] = nxt;
    w[PW_NZT] = nzt;
    w[PW_XPAD] = (int32_t)xpad;
    w[PW_ZPAD] = (int32_t)zpad;
    w[PW_CAP] = cap;
    w[PW_MAXW] = (int32_t)max_w;
    w[PW_PB] = pairs_per_batch(cap);
    w[PW_OFF_SET] = (int32_t)off;
    w[off++] = 0;
    w[off++] = (int32_t)P;
    // pair p = l * N + i (element-major): record index i * L + l, transmit row i
    w[PW_OFF_REC] = (int32_t)off;
    for (int64_t p = 0; p < P; ++p) w[off++] = (int32_t)((p % N) * L + p / N);
    w[PW_OFF_TX] = (int32_t)off;
    for (int64_t p = 0; p < P; ++p) w[off++] = (int32_t)(p % N);
    w[PW_OFF_A] = (int32_t)off;
    std::memcpy(w + off, A.data(), A.size() * 4);
    off += (int64_t)A.size();
    w[PW_OFF_B] = (int32_t)off;
    std::memcpy(w + off, B.data(), B.size() * 4);
    off += (int64_t)B.size();
    w[PW_OFF_LO] = (int32_t)off;
    std::memcpy(w + off, lo.data(), lo.size() * 4);
    off += (int64_t)lo.size();
    w[PW_OFF_C] = (int32_t)off;
    std::memcpy(w + off, C.data(), C.size() * 4);
    off += (int64_t)C.size();
    w[PW_TOTAL] = (int32_t)off;
    w[PW_SPLIT] = choose_split(ntiles, P, pairs_per_batch(cap));
    return off == words ? KK_OK : KK_E_ARG;
}

}  // extern "C"
