/*
 * Synthetic linear-array channel data for coherent plane-wave compounding.
 *
 * Forward model only (it is the acquisition, not the beamforming method):
 *   rf[i][l][n] = sum_s a_s * p(t0 + n/fs - tau_in(r_s, theta_i) - |r_s - (u_l, 0)| / c)
 * with a far-field transmit delay tau_in = (x sin(theta) + z cos(theta)) / c (the plane
 * wavefront crosses the array centre at t = 0) and a spherical receive path.  The pulse is
 * p(t) = cos(2 pi fc t) exp(-t^2 / (2 sigma^2)), truncated at |t| <= trunc * sigma.
 *
 * Each trace is accumulated sequentially over scatterers in input order, so the result is
 * deterministic whatever the thread count.  The per-scatterer pulse samples use exact
 * rotation / Gaussian-ratio recurrences seeded by one libm call each, which keeps a
 * 1e5-scatterer phantom to seconds.
 */
#include <math.h>
#include <stdint.h>

void kk_rfsim(int32_t N, int32_t L, int32_t T,
              const double* tx_theta, const double* elem_x,
              double c, double fs, double t0, double fc, double sigma, double trunc,
              int32_t S, const double* sx, const double* sz, const double* sa,
              double* out)
{
    const double h = 1.0 / fs;
    const double two_pi = 6.283185307179586476925286766559;
    const double rot_c = cos(two_pi * fc * h);
    const double rot_s = sin(two_pi * fc * h);
    const double inv2s2 = 1.0 / (2.0 * sigma * sigma);
    const double gstep = exp(-h * h / (sigma * sigma)); /* ratio of successive Gaussian ratios */
    const double half_width = trunc * sigma;

#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t tr = 0; tr < (int64_t)N * L; ++tr) {
        const int i = (int)(tr / L);
        const int l = (int)(tr % L);
        const double st = sin(tx_theta[i]);
        const double ct = cos(tx_theta[i]);
        const double u = elem_x[l];
        double* o = out + tr * (int64_t)T;
        for (int n = 0; n < T; ++n) o[n] = 0.0;
        for (int s = 0; s < S; ++s) {
            const double dx = sx[s] - u;
            const double t_arr = (sx[s] * st + sz[s] * ct) / c + sqrt(dx * dx + sz[s] * sz[s]) / c;
            /* sample window where |t0 + n h - t_arr| <= half_width */
            const double nlo = ceil((t_arr - half_width - t0) * fs);
            const double nhi = floor((t_arr + half_width - t0) * fs);
            if (nhi < 0.0 || nlo > (double)(T - 1)) continue;
            int n0 = nlo < 0.0 ? 0 : (int)nlo;
            int n1 = nhi > (double)(T - 1) ? T - 1 : (int)nhi;
            double t = t0 + (double)n0 * h - t_arr;
            /* phasor exp(i 2 pi fc t) and Gaussian g(t), advanced by h per sample */
            double pc = cos(two_pi * fc * t), ps = sin(two_pi * fc * t);
            double g = exp(-t * t * inv2s2);
            double ratio = exp(-(2.0 * t * h + h * h) * inv2s2); /* g(t+h)/g(t) */
            const double a = sa[s];
            for (int n = n0; n <= n1; ++n) {
                o[n] += a * pc * g;
                const double npc = pc * rot_c - ps * rot_s;
                ps = ps * rot_c + pc * rot_s;
                pc = npc;
                g *= ratio;
                ratio *= gstep;
            }
        }
    }
}
