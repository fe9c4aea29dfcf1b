// Device helpers shared by the engines: slice weights (expand step),
// expm planning, Taylor coefficients, wave utilities.
#pragma once

#include "pm_internal.h"

namespace pm {

// Taylor coefficients of cos and sin split by powers of Y = G^2:
//   exp(-i G) = sum_k (-1)^k Y^k / (2k)!  -  i G sum_k (-1)^k Y^k / (2k+1)!
__device__ __forceinline__ double cos_coef(int k) {
    constexpr double t[11] = {
        1.0, -1.0 / 2, 1.0 / 24, -1.0 / 720, 1.0 / 40320, -1.0 / 3628800, 1.0 / 479001600,
        -1.0 / 87178291200.0, 1.0 / 20922789888000.0, -1.0 / 6402373705728000.0,
        1.0 / 2432902008176640000.0};
    return t[k];
}
__device__ __forceinline__ double sin_coef(int k) {
    constexpr double t[11] = {
        1.0, -1.0 / 6, 1.0 / 120, -1.0 / 5040, 1.0 / 362880, -1.0 / 39916800,
        1.0 / 6227020800.0, -1.0 / 1307674368000.0, 1.0 / 355687428096000.0,
        -1.0 / 121645100408832000.0, 1.0 / 51090942171709440000.0};
    return t[k];
}

// Wave-uniform copy of a value that every lane already holds.
__device__ __forceinline__ double wave_uniform(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffLL));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ int wave_uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Weight of basis matrix m in slice j (the expand step; eq. magnus_coeffs
// for order 4 with the commutator sign of the standard product order).
__device__ __forceinline__ double slice_weight(const PropParams& p, int64_t j, int m) {
    const double h = p.h;
    if (m == 0) return h;
    const double* c = p.samples;
    const int64_t S = p.n_samples;
    if (p.order == 2) return h * c[(int64_t)(m - 1) * S + j];
    const int K = p.K;
    const double h2 = h * h * (1.0 / 12.0);
    if (m <= K) {
        const double* ck = c + (int64_t)(m - 1) * S + 2 * j;
        return (h * (1.0 / 6.0)) * (ck[0] + 4.0 * ck[1] + ck[2]);
    }
    if (m <= 2 * K) {
        const double* ck = c + (int64_t)(m - 1 - K) * S + 2 * j;
        return h2 * (ck[2] - ck[0]);
    }
    const double* ca = c + (int64_t)p.pair_a[m] * S + 2 * j;
    const double* cb = c + (int64_t)p.pair_b[m] * S + 2 * j;
    return h2 * (ca[0] * cb[2] - ca[2] * cb[0]);
}

// Products used by the cos/sin Taylor evaluation of degree m:
// Y, Y^2 .. Y^{m/2}, and G * S'(Y) when S' has a Y term.
__device__ __forceinline__ int taylor_products(int m) {
    if (m <= 1) return 0;
    if (m == 2) return 1;
    return m / 2 + 1;
}

// Choose (m, s): minimise taylor_products(m) + s with nu / 2^s <= theta_m,
// m <= max_degree; ties go to the smaller s.  Degrees 1, 2 and odd m >= 3
// are the only candidates (an even m >= 4 costs as much as m + 1).
__device__ __forceinline__ void plan_expm(const PropParams& p, double nu, int& m_out, int& s_out) {
    const int md = p.max_degree;
    if (p.force_s >= 0) {
        const double x = ldexp(nu, -p.force_s);
        int m = md;
        for (int c = 1; c <= md; c = (c < 3 ? c + 1 : c + 2)) {
            if (p.theta[c] >= x) { m = c; break; }
        }
        m_out = m;
        s_out = p.force_s;
        return;
    }
    int best_m = md, best_s = 0, best_cost = 1 << 30;
    for (int s = 0; s < 64; ++s) {
        if (s >= best_cost) break;
        const double x = ldexp(nu, -s);
        for (int c = 1; c <= md; c = (c < 3 ? c + 1 : c + 2)) {
            if (p.theta[c] >= x) {
                const int cost = taylor_products(c) + s;
                if (cost < best_cost) { best_cost = cost; best_m = c; best_s = s; }
                break;
            }
        }
    }
    if (best_cost == (1 << 30)) {  // nu not finite: keep going, result is NaN anyway
        best_m = md;
        best_s = 0;
    }
    m_out = best_m;
    s_out = best_s;
}

}  // namespace pm
