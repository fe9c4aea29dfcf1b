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

// First slice of chain c: the first p.n_long chains hold p.chunk_long slices
// each, the rest p.chunk (for c = n_chains, at least N).
__device__ __forceinline__ int64_t chain_first(const PropParams& p, int64_t c) {
    return c <= p.n_long ? c * p.chunk_long : p.n_long * p.chunk_long + (c - p.n_long) * p.chunk;
}

// The block copies n doubles (n even, both ends 16-byte aligned) from global
// memory into LDS in 16-byte pieces, eight loads in flight per thread before
// their stores.  The caller synchronises the block afterwards.
__device__ __forceinline__ void block_copy_to_lds(double* dst, const double* src, int n) {
    const int n2 = n / 2, step = (int)blockDim.x;
    const double2* s2 = reinterpret_cast<const double2*>(src);
    double2* d2 = reinterpret_cast<double2*>(dst);
    int i = (int)threadIdx.x;
    for (; i + 7 * step < n2; i += 8 * step) {
        double2 v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = s2[i + q * step];
#pragma unroll
        for (int q = 0; q < 8; ++q) d2[i + q * step] = v[q];
    }
    for (; i < n2; i += step) d2[i] = s2[i];
}

// Wave-uniform copy of a value that every lane already holds.
__device__ __forceinline__ double wave_uniform(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffLL));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ int wave_uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Value of x in lane l (l wave-uniform).
__device__ __forceinline__ double readlane_d(double x, int l) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Weight of basis matrix m in exponent j (the expand step; eq. magnus_coeffs
// for order 4 with the commutator sign of the standard product order; for
// the commutator-free scheme exponent j is factor j & 1 of slice j >> 1,
// (h/12)(3 s0 + 4 s1 - s2) for the first and its mirror for the second).
__device__ __forceinline__ double slice_weight(const PropParams& p, int64_t j, int m) {
    const double h = p.h;
    const double* c = p.samples;
    const int64_t S = p.n_samples;
    if (p.order == kOrderCF4) {
        if (m == 0) return 0.5 * h;
        const double* ck = c + (int64_t)(m - 1) * S + (j & ~(int64_t)1);
        const double a = (j & 1) ? ck[2] : ck[0], b = (j & 1) ? ck[0] : ck[2];
        return (h * (1.0 / 12.0)) * (3.0 * a + 4.0 * ck[1] - b);
    }
    if (m == 0) return h;
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

// Smallest s >= 0 with nu / 2^s <= th (th > 0).  With nu = a 2^e1 and
// th = b 2^e2 (a, b in [1/2, 1)), log2(nu / th) lies in (e1 - e2 - 1,
// e1 - e2 + 1), so the answer is e1 - e2 or one more; the comparisons of
// exact power-of-two scalings decide (no division).
__device__ __forceinline__ int min_squarings(double nu, double th) {
    if (!(nu > th)) return 0;
    int e1, e2;
    (void)frexp(nu, &e1);
    (void)frexp(th, &e2);
    int s = e1 - e2;
    if (ldexp(nu, -s) > th) s += 1;
    else if (s > 0 && ldexp(nu, -(s - 1)) <= th) s -= 1;
    return s;
}

// Choose (m, s): minimise taylor_products(m) + s with nu / 2^s <= theta_m,
// m <= max_degree; ties go to the smaller s.  Degrees 1, 2 and odd m >= 3
// are the only candidates (an even m >= 4 costs as much as m + 1).  With
// force_s >= 0 the smallest feasible degree is taken (max_degree if none).
// Unrolled over the candidates so the thresholds stay in scalar registers.
__device__ __forceinline__ void plan_expm(const PropParams& p, double nu, int& m_out, int& s_out) {
    constexpr int kCand[12] = {1, 2, 3, 5, 7, 9, 11, 13, 15, 17, 19, 21};
    const int md = p.max_degree;
    int bm = md, bs = 0, bc = 1 << 30;
    if (p.force_s >= 0) {
        const double x = ldexp(nu, -p.force_s);
#pragma unroll
        for (int i = 11; i >= 0; --i) {
            const int c = kCand[i];
            if (c <= md && p.theta[c] >= x) bm = c;
        }
        m_out = bm;
        s_out = p.force_s;
        return;
    }
#pragma unroll
    for (int i = 0; i < 12; ++i) {
        const int c = kCand[i];
        if (c <= md) {
            const int s = min_squarings(nu, p.theta[c]);
            const int cost = taylor_products(c) + s;
            if (cost < bc || (cost == bc && s < bs)) {
                bc = cost;
                bm = c;
                bs = s;
            }
        }
    }
    m_out = bm;
    s_out = bs;
}

// The same plan with the 12 candidate degrees spread over lanes 0..11 (one
// candidate each, threshold preloaded in `lane_theta`, +inf elsewhere):
// every lane packs (cost, s, candidate) into an integer key, and the row
// minimum of the keys is the plan (ties to the smaller s, as above).
constexpr int kNumCand = 12;
__device__ __forceinline__ int cand_degree(int i) { return i < 3 ? i + 1 : 2 * i - 1; }

__device__ __forceinline__ double lane_theta_of(const PropParams& p, int lane) {
    if (lane >= kNumCand || cand_degree(lane) > p.max_degree) return __builtin_inf();
    return p.theta[cand_degree(lane)];
}

__device__ __forceinline__ int row16_min_i(int x) {
    x = min(x, __builtin_amdgcn_update_dpp(0, x, 0x128, 0xF, 0xF, false));
    x = min(x, __builtin_amdgcn_update_dpp(0, x, 0x124, 0xF, 0xF, false));
    x = min(x, __builtin_amdgcn_update_dpp(0, x, 0x122, 0xF, 0xF, false));
    x = min(x, __builtin_amdgcn_update_dpp(0, x, 0x121, 0xF, 0xF, false));
    return x;
}

__device__ __forceinline__ void plan_expm_lanes(const PropParams& p, double nu, int lane,
                                                double lane_theta, int& m_out, int& s_out) {
    const bool cand = lane_theta < __builtin_inf();
    int key;
    if (p.force_s >= 0) {
        key = (cand && ldexp(nu, -p.force_s) <= lane_theta) ? lane : 1 << 20;
        key = __builtin_amdgcn_readfirstlane(row16_min_i(key));
        m_out = key < kNumCand ? cand_degree(key) : p.max_degree;
        s_out = p.force_s;
        return;
    }
    const int s = min(min_squarings(nu, cand ? lane_theta : 1.0), 63);
    const int deg = cand_degree(lane);
    key = cand ? ((taylor_products(deg) + s) << 12) | (s << 5) | lane : 0x7fffffff;
    key = __builtin_amdgcn_readfirstlane(row16_min_i(key));
    m_out = cand_degree(key & 31);
    s_out = (key >> 5) & 63;
}

// Chebyshev planner: lane l tests degree l + 1 against its interval
// half-width (preloaded in lane_ctheta, +inf past the last degree) and
// minimises the products of the even/odd split evaluation plus the
// squarings (the Taylor count taylor_products(m) + s), ties to the smaller s,
// then to the smaller degree.  With force_s >= 0 the smallest feasible
// degree (the largest if none is).
__device__ __forceinline__ double lane_ctheta_of(const PropParams& p, int lane) {
    return lane < kMaxCheb ? p.ctheta[lane + 1] : __builtin_inf();
}

__device__ __forceinline__ void plan_cheb_lanes(const PropParams& p, double nu, int lane, double lane_ctheta,
                                                int& m_out, int& s_out) {
    // the candidates occupy lanes 0..24: minimum over the first two rows
    auto min2rows = [](int k) {
        const int r = row16_min_i(k);
        return min(__builtin_amdgcn_readlane(r, 0), __builtin_amdgcn_readlane(r, 16));
    };
    const bool cand = lane_ctheta < __builtin_inf();
    if (p.force_s >= 0) {
        const int key = min2rows((cand && ldexp(nu, -p.force_s) <= lane_ctheta) ? lane : 1 << 20);
        m_out = key < kMaxCheb ? key + 1 : kMaxCheb;
        s_out = p.force_s;
        return;
    }
    const int s = min(min_squarings(nu, cand ? lane_ctheta : 1.0), 63);
    const int key = min2rows(cand ? ((taylor_products(lane + 1) + s) << 12) | (s << 6) | lane : 0x7fffffff);
    m_out = (key & 63) + 1;
    s_out = (key >> 6) & 63;
}

// Branch-free form of slice_weight for a lane-dependent basis index m: the
// lane gathers up to five samples of the slice and combines them with the
// formula of its basis matrix.  Lanes m >= M get weight 0.
struct WeightRecipe {
    int kind;        // 0: H0, 1: order-2 control, 2: Simpson, 3: commutator with H0, 4: pair, 5: none,
                     // 6: commutator-free control, 7: sixth-order moment of a control
    int64_t xa, xb;  // sample offsets of controls a, b (before adding the slice position);
                     // sixth order: xb is the moment (0, 1, 2)
};

struct SliceSamples {
    double x0, x1, x2, y0, y2;
};

__device__ __forceinline__ WeightRecipe weight_recipe(const PropParams& p, int m) {
    WeightRecipe r;
    const int K = p.K;
    const int64_t S = p.n_samples;
    r.xa = 0;
    r.xb = 0;
    if (m >= p.M) {
        r.kind = 5;
    } else if (m == 0) {
        r.kind = 0;
    } else if (p.order == 2) {
        r.kind = 1;
        r.xa = (int64_t)(m - 1) * S;
    } else if (p.order == kOrderCF4) {
        r.kind = 6;
        r.xa = (int64_t)(m - 1) * S;
    } else if (m <= K) {
        r.kind = 2;
        r.xa = (int64_t)(m - 1) * S;
    } else if (m <= 2 * K) {
        r.kind = 3;
        r.xa = (int64_t)(m - 1 - K) * S;
    } else {
        r.kind = 4;
        r.xa = (int64_t)p.pair_a[m] * S;
        r.xb = (int64_t)p.pair_b[m] * S;
    }
    return r;
}

// Issue the sample loads of slice j (no use of the values here).
__device__ __forceinline__ SliceSamples gather_samples(const PropParams& p, const WeightRecipe& r, int64_t j) {
    SliceSamples v{0.0, 0.0, 0.0, 0.0, 0.0};
    if (p.K == 0) return v;
    const double* c = p.samples;
    if (p.order == 2) {
        v.x0 = c[r.xa + j];
    } else if (p.order == kOrderCF4) {
        // the second factor reads the slice's samples mirrored
        const double* a = c + r.xa + (j & ~(int64_t)1);
        const bool second = (j & 1) != 0;
        v.x0 = a[second ? 2 : 0];
        v.x1 = a[1];
        v.x2 = a[second ? 0 : 2];
    } else {
        const double* a = c + r.xa + 2 * j;
        const double* b = c + r.xb + 2 * j;
        v.x0 = a[0];
        v.x1 = a[1];
        v.x2 = a[2];
        v.y0 = b[0];
        v.y2 = b[2];
    }
    return v;
}

__device__ __forceinline__ double combine_weight(const PropParams& p, const WeightRecipe& r,
                                                 const SliceSamples& v) {
    const double h = p.h;
    const double h2 = h * h * (1.0 / 12.0);
    const double w1 = h * v.x0;
    const double w2 = (h * (1.0 / 6.0)) * (v.x0 + 4.0 * v.x1 + v.x2);
    const double w3 = h2 * (v.x2 - v.x0);
    const double w4 = h2 * (v.x0 * v.y2 - v.x2 * v.y0);
    const double w6 = (h * (1.0 / 12.0)) * (3.0 * v.x0 + 4.0 * v.x1 - v.x2);
    double w = 0.0;
    w = r.kind == 0 ? (p.order == kOrderCF4 ? 0.5 * h : h) : w;
    w = r.kind == 6 ? w6 : w;
    w = r.kind == 1 ? w1 : w;
    w = r.kind == 2 ? w2 : w;
    w = r.kind == 3 ? w3 : w;
    w = r.kind == 4 ? w4 : w;
    return w;
}

// Sixth-order Magnus (PM_ORDER_MAGNUS6): slice j has the samples 3j, 3j+1,
// 3j+2 of each control, taken at the Gauss-Legendre nodes of the slice, and
// three moments of H over it are formed on the basis {H0, H_k}:
//   P1 = h A2,  P2 = (sqrt(15) h / 3)(A3 - A1),  P3 = (10 h / 3)(A3 - 2 A2 + A1),
// with A_i = H at node i (H0 enters P1 only).  Lane 16 q + m (q < 3, m < M)
// gathers the samples of control m - 1 and combines the weight of basis
// matrix m in moment q + 1; other lanes get weight 0.
constexpr double kSqrt15 = 3.872983346207417;

__device__ __forceinline__ WeightRecipe m6_recipe(const PropParams& p, int lane) {
    WeightRecipe r;
    const int q = lane >> 4, m = lane & 15;
    r.xb = q;
    r.kind = (q > 2 || m >= p.M) ? 5 : (m == 0 ? 0 : 7);
    // control m - 1's row for the lanes that weight a control (m <= K);
    // every other lane still loads (its weight is zero), from row 0, so no
    // lane reads past the K rows of samples
    r.xa = r.kind == 7 ? (int64_t)(m - 1) * p.n_samples : 0;
    return r;
}

__device__ __forceinline__ SliceSamples m6_gather(const PropParams& p, const WeightRecipe& r, int64_t j) {
    SliceSamples v{0.0, 0.0, 0.0, 0.0, 0.0};
    if (p.K == 0) return v;
    const double* a = p.samples + r.xa + 3 * j;
    v.x0 = a[0];
    v.x1 = a[1];
    v.x2 = a[2];
    return v;
}

__device__ __forceinline__ double m6_weight(const PropParams& p, const WeightRecipe& r, const SliceSamples& v) {
    const double h = p.h;
    const double c1 = h * v.x1;
    const double c2 = (h * (kSqrt15 / 3.0)) * (v.x2 - v.x0);
    const double c3 = (h * (10.0 / 3.0)) * ((v.x2 - 2.0 * v.x1) + v.x0);
    double w = r.xb == 0 ? c1 : (r.xb == 1 ? c2 : c3);
    w = r.kind == 0 ? (r.xb == 0 ? h : 0.0) : w;
    return r.kind == 5 ? 0.0 : w;
}

// DPP row rotation (within each row of 16 lanes) of a double.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 16 lanes of each row (every lane of the row gets the sum).
__device__ __forceinline__ double row16_sum(double x) {
    x += dpp_d<0x128>(x);   // row_ror:8
    x += dpp_d<0x124>(x);   // row_ror:4
    x += dpp_d<0x122>(x);   // row_ror:2
    x += dpp_d<0x121>(x);   // row_ror:1
    return x;
}

__device__ __forceinline__ double row16_max(double x) {
    x = fmax(x, dpp_d<0x128>(x));
    x = fmax(x, dpp_d<0x124>(x));
    x = fmax(x, dpp_d<0x122>(x));
    x = fmax(x, dpp_d<0x121>(x));
    return x;
}

// Maximum over the four rows of a wave (lanes 0, 16, 32, 48 hold the row
// values after a row16 reduction); wave-uniform result.
__device__ __forceinline__ double rows_max(double x) {
    return fmax(fmax(readlane_d(x, 0), readlane_d(x, 16)), fmax(readlane_d(x, 32), readlane_d(x, 48)));
}

// Single-precision variants for row sums of entry bounds: the sum of 16
// non-negative terms in FP32 is within 16 * 2^-24 of exact, the hardware
// square root (no correctly rounded expansion: one instruction) within
// 2^-22; rows_max_f inflates the result by 2^-16 so it stays an upper bound,
// and returns it in FP64.
__device__ __forceinline__ float abs_bound_f(double re, double im) {
    return __builtin_amdgcn_sqrtf((float)(re * re + im * im));
}

__device__ __forceinline__ float row16_sum_f(float x) {
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x128, 0xF, 0xF, false));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x124, 0xF, 0xF, false));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x122, 0xF, 0xF, false));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x121, 0xF, 0xF, false));
    return x;
}

__device__ __forceinline__ double rows_max_f(float x) {
    const float a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 0));
    const float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 16));
    const float c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 32));
    const float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 48));
    return (double)fmaxf(fmaxf(a, b), fmaxf(c, d)) * (1.0 + 0x1p-16) + 0x1p-60;
}

// Upper bound of |re + i im| from the hardware single-precision square root,
// inflated past its rounding (relative error < 2^-22) so the bound never
// falls short.
__device__ __forceinline__ double abs_bound(double re, double im) {
    const float q = (float)(re * re + im * im);
    return (double)__builtin_amdgcn_sqrtf(q) * (1.0 + 0x1p-20) + 0x1p-60;
}

}  // namespace pm
