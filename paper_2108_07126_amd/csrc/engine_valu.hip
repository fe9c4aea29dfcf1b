// VALU engine for dimensions 2 and 4: one slice per lane, all matrices in
// registers.  Lane l of a wave runs `chunk/64` consecutive slices and keeps
// its own chain product; the 64 lane products are then multiplied by a
// pairwise tree across lanes (register shuffles), and the wave's product
// enters the same ticketed FP64 tree as the MFMA engine's teams.
//
// Per slice: expand G = sum_m w_m B_m (FP64; the basis is wave-uniform and
// read through the scalar cache), shift by the mean eigenvalue mu = tr G / D
// (exp(-i G) = e^{-i mu} exp(-i (G - mu I)), the phase by sincos), bound the
// 1-norm of the shifted matrix, plan once per wave (maximum over its lanes),
// and evaluate the truncated Taylor series of exp(-i X), X = (G - mu I)/2^s,
// in the D-dimensional algebra spanned by I, X, .., X^{D-1} (Cayley-Hamilton:
// the series becomes D scalar recurrences; D = 4 needs the matrix powers X^2
// and X^3 only), then square s times in FP64.
#include <type_traits>

#include "engine_common.h"

namespace pm {
namespace {

template <int D>
constexpr int hidx(int i, int j) {  // i <= j, packed upper triangle, row-major
    return i * D - (i * (i - 1)) / 2 + (j - i);
}

template <int D, typename T>
struct Herm {
    static constexpr int NE = D * (D + 1) / 2;
    T re[NE], im[NE];
    __device__ __forceinline__ T gre(int i, int j) const { return i <= j ? re[hidx<D>(i, j)] : re[hidx<D>(j, i)]; }
    __device__ __forceinline__ T gim(int i, int j) const { return i <= j ? im[hidx<D>(i, j)] : -im[hidx<D>(j, i)]; }
};

template <int D, typename T>
struct Mat {
    T re[D * D], im[D * D];
};

template <int D, typename T>
__device__ __forceinline__ void mat_ident(Mat<D, T>& a) {
#pragma unroll
    for (int i = 0; i < D * D; ++i) {
        a.re[i] = (i % (D + 1) == 0) ? T(1) : T(0);
        a.im[i] = T(0);
    }
}

// Upper triangle of A B for commuting Hermitian A, B (the product is Hermitian).
template <int D, typename T>
__device__ __forceinline__ Herm<D, T> herm_mul(const Herm<D, T>& a, const Herm<D, T>& b) {
    Herm<D, T> c;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = i; j < D; ++j) {
            T sr = 0, si = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const T ar = a.gre(i, k), ai = a.gim(i, k), br = b.gre(k, j), bi = b.gim(k, j);
                sr = fma(ar, br, sr);
                sr = fma(-ai, bi, sr);
                si = fma(ar, bi, si);
                si = fma(ai, br, si);
            }
            c.re[hidx<D>(i, j)] = sr;
            c.im[hidx<D>(i, j)] = si;
        }
    return c;
}

template <int D, typename T>
__device__ __forceinline__ Mat<D, T> mat_mul(const Mat<D, T>& a, const Mat<D, T>& b) {
    Mat<D, T> c;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            T sr = 0, si = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const T ar = a.re[i * D + k], ai = a.im[i * D + k];
                const T br = b.re[k * D + j], bi = b.im[k * D + j];
                sr = fma(ar, br, sr);
                sr = fma(-ai, bi, sr);
                si = fma(ar, bi, si);
                si = fma(ai, br, si);
            }
            c.re[i * D + j] = sr;
            c.im[i * D + j] = si;
        }
    return c;
}

template <int D, typename T, typename U>
__device__ __forceinline__ Mat<D, T> mat_convert(const Mat<D, U>& a) {
    Mat<D, T> c;
#pragma unroll
    for (int e = 0; e < D * D; ++e) {
        c.re[e] = (T)a.re[e];
        c.im[e] = (T)a.im[e];
    }
    return c;
}

template <int D>
__device__ __forceinline__ Mat<D, double> mat_shfl_down(const Mat<D, double>& a, int delta) {
    Mat<D, double> c;
#pragma unroll
    for (int e = 0; e < D * D; ++e) {
        c.re[e] = __shfl_down(a.re[e], delta);
        c.im[e] = __shfl_down(a.im[e], delta);
    }
    return c;
}

// Characteristic-polynomial coefficients r_0..r_{D-1} of a Hermitian X
// (X^D = sum_i r_i X^i, Cayley-Hamilton) from the power traces
// p_k = tr X^k by Newton's identities.
template <int D>
__device__ __forceinline__ void ch_coeffs(const double (&pw)[D + 1], double (&r)[D]) {
    double e[D + 1];
    e[0] = 1.0;
#pragma unroll
    for (int k = 1; k <= D; ++k) {
        double acc = 0.0;
#pragma unroll
        for (int i = 1; i <= k; ++i) acc += ((i & 1) ? 1.0 : -1.0) * e[k - i] * pw[i];
        e[k] = acc * (1.0 / k);
    }
    // char poly: X^D - e1 X^{D-1} + e2 X^{D-2} - ... ; r_{D-i} = (-1)^{i+1} e_i
#pragma unroll
    for (int i = 1; i <= D; ++i) r[D - i] = ((i & 1) ? 1.0 : -1.0) * e[i];
}

// One step a <- X a in the algebra spanned by I, X, .., X^{D-1}
// (coefficient vectors; X^D reduced by the characteristic polynomial).
template <int D>
__device__ __forceinline__ void ch_step(double (&a)[D], const double (&r)[D]) {
    const double top = a[D - 1];
#pragma unroll
    for (int i = D - 1; i >= 1; --i) a[i] = fma(top, r[i], a[i - 1]);
    a[0] = top * r[0];
}

// Coefficients of the degree-m Taylor polynomial of exp(-i X) in the basis
// I, X, .., X^{D-1}: sum_{k<=m} (-i)^k X^k / k!, real and imaginary parts.
// With EXCESS the k = 0 term (the identity) is left out.
template <int D, bool EXCESS>
__device__ __forceinline__ void ch_taylor(const double (&r)[D], int m, double (&cre)[D],
                                          double (&cim)[D]) {
    double a[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        a[i] = (i == 0) ? 1.0 : 0.0;
        cre[i] = EXCESS ? 0.0 : a[i];
        cim[i] = 0.0;
    }
    // k = 2q + 1 (sin part) then k = 2q + 2 (cos part)
    for (int q = 0; 2 * q + 1 <= m; ++q) {
        ch_step<D>(a, r);
        const double sc = sin_coef(q);
#pragma unroll
        for (int i = 0; i < D; ++i) cim[i] = fma(-sc, a[i], cim[i]);
        if (2 * q + 2 > m) break;
        ch_step<D>(a, r);
        const double cc = cos_coef(q + 1);
#pragma unroll
        for (int i = 0; i < D; ++i) cre[i] = fma(cc, a[i], cre[i]);
    }
}

// tr(A B) of Hermitian A, B in upper-triangle storage (real).
template <int D, typename T>
__device__ __forceinline__ double herm_trace_prod(const Herm<D, T>& a, const Herm<D, T>& b) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = i; j < D; ++j) {
            const int e = hidx<D>(i, j);
            const double v = (double)a.re[e] * (double)b.re[e] + (double)a.im[e] * (double)b.im[e];
            t += (i == j) ? v : 2.0 * v;
        }
    return t;
}

// exp(-i X) of a pre-scaled Hermitian X by the degree-m Taylor polynomial,
// evaluated in the algebra generated by X: by Cayley-Hamilton every power
// X^k with k >= D is a combination of I, X, .., X^{D-1}, so the polynomial
// is carried as D complex coefficients (scalar recurrences) and the matrix
// is formed once from the powers X^0..X^{D-1}.  The result is the same
// truncated series as the matrix evaluation; only the order of operations
// differs.  With EXCESS the result is exp(-i X) - I (accurate relative to
// ||X||).
template <int D, typename T, bool EXCESS>
__device__ __forceinline__ Mat<D, T> taylor_exp_ch(const Herm<D, T>& x, int m) {
    static_assert(D == 2 || D == 4, "algebra evaluation for D = 2 and 4");
    double pw[D + 1];
    double tr1 = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) tr1 += (double)x.re[hidx<D>(i, i)];
    pw[0] = (double)D;
    pw[1] = tr1;
    pw[2] = herm_trace_prod<D, T>(x, x);
    Herm<D, T> x2, x3;
    if constexpr (D == 4) {
        x2 = herm_mul(x, x);
        x3 = herm_mul(x, x2);
        pw[3] = herm_trace_prod<D, T>(x, x2);
        pw[4] = herm_trace_prod<D, T>(x, x3);
    }
    double r[D], cre[D], cim[D];
    ch_coeffs<D>(pw, r);
    ch_taylor<D, EXCESS>(r, m, cre, cim);
    // U = sum_i c_i X^i; (X^i)_{ba} = conj((X^i)_{ab})
    Mat<D, T> U;
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = a; b < D; ++b) {
            const int e = hidx<D>(a, b);
            double xr[D], xi[D];
            xr[0] = (a == b) ? 1.0 : 0.0;
            xi[0] = 0.0;
            xr[1] = x.re[e];
            xi[1] = x.im[e];
            if constexpr (D == 4) {
                xr[2] = x2.re[e];
                xi[2] = x2.im[e];
                xr[3] = x3.re[e];
                xi[3] = x3.im[e];
            }
            // sum_i c_i x_i and sum_i c_i conj(x_i)
            double pr = 0.0, pi = 0.0, qr = 0.0, qi = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const double rr = cre[i] * xr[i], ii = cim[i] * xi[i];
                const double ri = cre[i] * xi[i], ir = cim[i] * xr[i];
                pr += rr - ii;
                pi += ri + ir;
                qr += rr + ii;
                qi += ir - ri;
            }
            U.re[a * D + b] = (T)pr;
            U.im[a * D + b] = (T)pi;
            if (a != b) {
                U.re[b * D + a] = (T)qr;
                U.im[b * D + a] = (T)qi;
            }
        }
    return U;
}

// The control samples one slice needs: K values (order 2) or the three
// Simpson samples of each control (order 4), K <= KB.  Loaded for the next
// slice while the current one is exponentiated; every load is issued
// unconditionally (controls k >= K re-read control K-1) so the loads of a
// slice go out back to back.
template <int ORD, int KB>
struct SampleSet {
    double v[ORD == 2 ? KB : 3 * KB];
};

template <int ORD, int KB>
__device__ __forceinline__ SampleSet<ORD, KB> load_samples(const PropParams& p, int64_t j) {
    SampleSet<ORD, KB> s;
    const double* c = p.samples;
    const int64_t S = p.n_samples;
    if (p.K == 0) {
#pragma unroll
        for (int q = 0; q < (ORD == 2 ? KB : 3 * KB); ++q) s.v[q] = 0.0;
        return s;
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        const int kk = min(k, p.K - 1);
        if constexpr (ORD == 2) {
            s.v[k] = c[(int64_t)kk * S + j];
        } else {
            const double* ck = c + (int64_t)kk * S + 2 * j;
            s.v[3 * k + 0] = ck[0];
            s.v[3 * k + 1] = ck[1];
            s.v[3 * k + 2] = ck[2];
        }
    }
    return s;
}

// Expand one slice into the upper triangle of G (FP64): the weights of the
// midpoint rule (order 2) or of eq. magnus_coeffs (order 4, pairs i[H_a,H_b]
// with a < b in lexicographic order after the 2K single-control terms).
template <int D, int ORD, int KB>
__device__ __forceinline__ Herm<D, double> expand_slice(const PropParams& p, const SampleSet<ORD, KB>& x,
                                                        bool valid) {
    Herm<D, double> g;
#pragma unroll
    for (int e = 0; e < Herm<D, double>::NE; ++e) g.re[e] = g.im[e] = 0.0;
    const double h = valid ? p.h : 0.0;
    const int K = p.K;
    auto add = [&](double w, int m) {
        const double* b = p.basis + (int64_t)m * D * D * 2;
#pragma unroll
        for (int r = 0; r < D; ++r)
#pragma unroll
            for (int cc = r; cc < D; ++cc) {
                g.re[hidx<D>(r, cc)] = fma(w, b[(r * D + cc) * 2 + 0], g.re[hidx<D>(r, cc)]);
                g.im[hidx<D>(r, cc)] = fma(w, b[(r * D + cc) * 2 + 1], g.im[hidx<D>(r, cc)]);
            }
    };
    add(h, 0);
    if constexpr (ORD == 2) {
#pragma unroll
        for (int k = 0; k < KB; ++k)
            if (k < K) add(h * x.v[k], 1 + k);
    } else {
        const double h6 = h * (1.0 / 6.0), h12 = h * p.h * (1.0 / 12.0);
#pragma unroll
        for (int k = 0; k < KB; ++k)
            if (k < K) {
                const double a0 = x.v[3 * k], a1 = x.v[3 * k + 1], a2 = x.v[3 * k + 2];
                add(h6 * (a0 + 4.0 * a1 + a2), 1 + k);
                add(h12 * (a2 - a0), 1 + K + k);
            }
#pragma unroll
        for (int a = 0; a < KB; ++a)
#pragma unroll
            for (int b = a + 1; b < KB; ++b)
                if (b < K) {
                    const int q = 1 + 2 * K + a * K - a * (a + 1) / 2 + (b - a - 1);
                    add(h12 * (x.v[3 * a] * x.v[3 * b + 2] - x.v[3 * a + 2] * x.v[3 * b]), q);
                }
    }
    return g;
}

// Upper bound of ||X||_1 for Hermitian X (column sums of moduli; FP32
// square roots and sums, inflated past their rounding).
template <int D>
__device__ __forceinline__ float norm1_bound(const Herm<D, double>& g) {
    float col[D];
#pragma unroll
    for (int i = 0; i < D; ++i) col[i] = fabsf((float)g.re[hidx<D>(i, i)]);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = i + 1; j < D; ++j) {
            const int e = hidx<D>(i, j);
            const float a = __builtin_sqrtf((float)(g.re[e] * g.re[e] + g.im[e] * g.im[e]));
            col[i] += a;
            col[j] += a;
        }
    float nu = col[0];
#pragma unroll
    for (int i = 1; i < D; ++i) nu = fmaxf(nu, col[i]);
    return nu * (1.0f + 0x1p-18f) + 0x1p-100f;
}

// Wave maximum of a non-negative float (DPP within rows, then the rows).
__device__ __forceinline__ float wave_max_f(float x) {
    x = fmaxf(x, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x128, 0xF, 0xF, false)));
    x = fmaxf(x, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x124, 0xF, 0xF, false)));
    x = fmaxf(x, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x122, 0xF, 0xF, false)));
    x = fmaxf(x, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x121, 0xF, 0xF, false)));
    const float a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 0));
    const float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 16));
    const float c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 32));
    const float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 48));
    return fmaxf(fmaxf(a, b), fmaxf(c, d));
}

// Plan for the algebra evaluation, where a higher Taylor degree costs a few
// scalar operations and a squaring costs a matrix product: the fewest
// squarings the largest allowed degree needs, then the smallest candidate
// degree that meets its threshold after those squarings.
__device__ __forceinline__ void plan_valu(const PropParams& p, double nu, int lane, double lane_theta,
                                          int& m_out, int& s_out) {
    const int s = wave_uniform(p.force_s >= 0 ? p.force_s : min(min_squarings(nu, p.theta[p.max_degree]), 62));
    const bool ok = lane_theta < __builtin_inf() && ldexp(nu, -s) <= lane_theta;
    int key = ok ? lane : 1 << 20;
    key = __builtin_amdgcn_readfirstlane(row16_min_i(key));
    m_out = key < kNumCand ? cand_degree(key) : p.max_degree;
    s_out = s;
}

// Store e^{-i mu} U (or e^{-i mu} (I + U) with plus_ident) as slice j,
// cropped to the user dimension.
template <int D, typename T>
__device__ __forceinline__ void store_phased(const PropParams& p, int64_t j, const Mat<D, T>& U, double mu,
                                             bool plus_ident) {
    double sn, cs;
    sincos(mu, &sn, &cs);
    T* out = reinterpret_cast<T*>(p.slices_out) + j * (int64_t)p.du * p.du * 2;
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
        for (int c = 0; c < D; ++c) {
            const double ur = (double)U.re[r * D + c] + ((plus_ident && r == c) ? 1.0 : 0.0);
            const double ui = (double)U.im[r * D + c];
            const T vr = (T)(cs * ur + sn * ui), vi = (T)(cs * ui - sn * ur);
            if (p.du == D) {
                out[(r * D + c) * 2 + 0] = vr;
                out[(r * D + c) * 2 + 1] = vi;
            } else if (r < p.du && c < p.du) {
                out[(r * p.du + c) * 2 + 0] = vr;
                out[(r * p.du + c) * 2 + 1] = vi;
            }
        }
}

// Per-slice output through LDS.  Lane l's slices are `run` apart from lane
// l+1's, so direct stores would touch 64 separate cache lines per
// instruction.  Each lane instead stages R consecutive slices (at least 128
// contiguous bytes) in a per-wave LDS buffer, and the wave then writes the 64
// segments cooperatively, 16 bytes per lane, whole lines per instruction.
template <typename T, int D>
struct Stage {
    static constexpr int SB = D * D * 2 * (int)sizeof(T);   // bytes per slice
    static constexpr int R = SB >= 128 ? 1 : 128 / SB;      // slices per segment
    static constexpr int SEG = R * SB;
    static constexpr int STRIDE = SEG + 16;                  // padded against bank conflicts
    static constexpr int BUF = 64 * STRIDE;                  // bytes per wave
    static constexpr int PIECES = SEG / 16;                  // 16-byte pieces per segment
};

// The phased slice e^{-i mu} (U or I + U) into this lane's staging row.
template <int D, typename T>
__device__ __forceinline__ void stage_phased(char* row, const Mat<D, T>& U, double mu, bool plus_ident) {
    double sn, cs;
    sincos(mu, &sn, &cs);
    T* out = reinterpret_cast<T*>(row);
#pragma unroll
    for (int e = 0; e < D * D; ++e) {
        const double ur = (double)U.re[e] + ((plus_ident && e % (D + 1) == 0) ? 1.0 : 0.0);
        const double ui = (double)U.im[e];
        out[2 * e + 0] = (T)(cs * ur + sn * ui);
        out[2 * e + 1] = (T)(cs * ui - sn * ur);
    }
}

// Write the staged segments of the wave: lane l's `nst` slices starting at
// slice first + l * run, each slice j < N.
template <typename T, int D>
__device__ __forceinline__ void flush_stage(const PropParams& p, const char* buf, int64_t first, int64_t run,
                                            int nst, int lane) {
    using S = Stage<T, D>;
    char* out = reinterpret_cast<char*>(p.slices_out);
#pragma unroll
    for (int q = 0; q < S::PIECES; ++q) {
        const int piece = q * 64 + lane;
        const int seg = piece / S::PIECES, off = piece % S::PIECES;
        const int r = (off * 16) / S::SB;
        const int64_t j = first + (int64_t)seg * run + r;
        if (r < nst && j < p.n_slices) {
            const uint4 v = *reinterpret_cast<const uint4*>(buf + seg * S::STRIDE + off * 16);
            *reinterpret_cast<uint4*>(out + (first + (int64_t)seg * run) * S::SB + off * 16) = v;
        }
    }
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// One slice per lane, all matrices in registers.  A leaf (one wave) covers
// `chunk` consecutive slices: lane l multiplies the run
// [base + l*run, base + (l+1)*run) into its own chain product.
template <typename T, int D, int ORD, int KB>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(D == 2 ? (ORD == 4 && KB >= 4 ? 3 : 4) : 1, 8)))
propagate_valu(PropParams p) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * 4 + wave_uniform((int)(threadIdx.x >> 6));
    if (wave >= p.n_leaves) return;
    extern __shared__ char stage_lds[];
    using S = Stage<T, D>;
    char* sbuf = stage_lds + (threadIdx.x >> 6) * S::BUF;
    char* srow = sbuf + lane * S::STRIDE;
    // staged (coalesced) output when the user dimension is the engine's
    const bool staged = p.slices_out != nullptr && p.du == D;
    const int64_t run = p.chunk / 64;
    const int64_t base = wave * p.chunk + (int64_t)lane * run;
    const double lth = lane_theta_of(p, lane);
    constexpr bool kF64 = std::is_same<T, double>::value;
    // The scalar phases e^{-i mu_j} commute with everything: the chain
    // multiplies the phase-free factors and the lane applies e^{-i sum mu}
    // once at the end of its run.  FP64: Q <- U Q.  Reduced modes: slices as
    // I + E and Q <- Q + E Q with Q in FP64.
    Mat<D, T> Q;
    mat_ident(Q);
    Mat<D, double> Qx;
    mat_ident(Qx);
    double phi = 0.0;
    const int64_t last = p.n_slices - 1;
    SampleSet<ORD, KB> smp = load_samples<ORD, KB>(p, min(base, last));
    for (int64_t i = 0; i < run; ++i) {
        const int64_t j = base + i;
        const bool valid = j < p.n_slices;
        const SampleSet<ORD, KB> cur = smp;
        if (i + 1 < run) smp = load_samples<ORD, KB>(p, min(j + 1, last));
        Herm<D, double> g = expand_slice<D, ORD, KB>(p, cur, valid);
        // shift by the mean eigenvalue: exp(-i G) = e^{-i mu} exp(-i (G - mu I))
        double mu = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) mu += g.re[hidx<D>(a, a)];
        mu *= 1.0 / D;
#pragma unroll
        for (int a = 0; a < D; ++a) g.re[hidx<D>(a, a)] -= mu;
        const double nu = (double)wave_max_f(norm1_bound<D>(g));
        int m, s;
        plan_valu(p, nu, lane, lth, m, s);
        Herm<D, T> x;
#pragma unroll
        for (int e = 0; e < Herm<D, T>::NE; ++e) {
            x.re[e] = (T)ldexp(g.re[e], -s);
            x.im[e] = (T)ldexp(g.im[e], -s);
        }
        if constexpr (kF64) {
            Mat<D, T> U = taylor_exp_ch<D, T, false>(x, m);
            for (int k = 0; k < s; ++k) U = mat_mul(U, U);
            if (valid) {
                if (staged) stage_phased<D, T>(srow + (i % S::R) * S::SB, U, mu, false);
                else if (p.slices_out) store_phased<D, T>(p, j, U, mu, false);
                Q = mat_mul(U, Q);
                phi += mu;
            }
        } else {
            Mat<D, T> E = taylor_exp_ch<D, T, true>(x, m);
            if (s > 0) {
                // (I + E)^2 - I = 2E + E E, in FP64
                Mat<D, double> Ed = mat_convert<D, double>(E);
                for (int k = 0; k < s; ++k) {
                    const Mat<D, double> P = mat_mul(Ed, Ed);
#pragma unroll
                    for (int e = 0; e < D * D; ++e) {
                        Ed.re[e] = fma(2.0, Ed.re[e], P.re[e]);
                        Ed.im[e] = fma(2.0, Ed.im[e], P.im[e]);
                    }
                }
                E = mat_convert<D, T>(Ed);
            }
            if (valid) {
                if (staged) stage_phased<D, T>(srow + (i % S::R) * S::SB, E, mu, true);
                else if (p.slices_out) store_phased<D, T>(p, j, E, mu, true);
                const Mat<D, T> P = mat_mul(E, mat_convert<D, T>(Qx));
#pragma unroll
                for (int e = 0; e < D * D; ++e) {
                    Qx.re[e] += (double)P.re[e];
                    Qx.im[e] += (double)P.im[e];
                }
                phi += mu;
            }
        }
        if (staged && ((i % S::R) == S::R - 1 || i == run - 1)) {
            const int nst = (int)(i % S::R) + 1;
            wave_lds_sync();
            flush_stage<T, D>(p, sbuf, wave * p.chunk + (i - (i % S::R)), run, nst, lane);
            wave_lds_sync();
        }
    }
    if constexpr (kF64) Qx = Q;
    {
        double sn, cs;
        sincos(phi, &sn, &cs);
#pragma unroll
        for (int e = 0; e < D * D; ++e) {
            const double r = Qx.re[e], im = Qx.im[e];
            Qx.re[e] = cs * r + sn * im;
            Qx.im[e] = cs * im - sn * r;
        }
    }
    // product over the wave's 64 consecutive runs: lane l+delta holds later slices
    Mat<D, double> W = Qx;
#pragma unroll
    for (int delta = 1; delta < 64; delta <<= 1) {
        const Mat<D, double> later = mat_shfl_down<D>(W, delta);
        const Mat<D, double> prod = mat_mul(later, W);
        if ((lane & (2 * delta - 1)) == 0) W = prod;
    }
    // lane 0 holds the wave's product; make it uniform
#pragma unroll
    for (int e = 0; e < D * D; ++e) {
        W.re[e] = wave_uniform(__shfl(W.re[e], 0));
        W.im[e] = wave_uniform(__shfl(W.im[e], 0));
    }
    // ticketed pairwise tree over the waves' products (FP64)
    const int64_t NN = (int64_t)D * D * 2;
    int64_t idx = wave, cnt = p.n_leaves, off = 0;
    while (cnt > 1) {
        const int64_t pcnt = (cnt + 1) >> 1, poff = off + cnt, par = idx >> 1;
        const bool carry = (idx == cnt - 1) && (cnt & 1);
        if (!carry) {
            double* node = p.nodes + (off + idx) * NN;
            if (lane == 0) {
#pragma unroll
                for (int e = 0; e < D * D; ++e) {
                    node[2 * e + 0] = W.re[e];
                    node[2 * e + 1] = W.im[e];
                }
            }
            __threadfence();
            unsigned v = 0;
            if (lane == 0) v = atomicAdd(&p.counters[poff + par], 1u);
            const unsigned t = (unsigned)wave_uniform((int)__shfl(v, 0));
            if (t == 0) return;
            __threadfence();
            if (lane == 0) atomicExch(&p.counters[poff + par], 0u);
            const double* sib = p.nodes + (off + (idx ^ 1)) * NN;
            Mat<D, double> O;
#pragma unroll
            for (int e = 0; e < D * D; ++e) {
                O.re[e] = sib[2 * e + 0];
                O.im[e] = sib[2 * e + 1];
            }
            W = (idx & 1) ? mat_mul(W, O) : mat_mul(O, W);
        }
        idx = par;
        off = poff;
        cnt = pcnt;
    }
    if (lane == 0) {
#pragma unroll
        for (int r = 0; r < D; ++r)
#pragma unroll
            for (int c = 0; c < D; ++c)
                if (r < p.du && c < p.du) {
                    p.U_out[(r * p.du + c) * 2 + 0] = W.re[r * D + c];
                    p.U_out[(r * p.du + c) * 2 + 1] = W.im[r * D + c];
                }
    }
}

template <typename T, int D, int ORD, int KB>
hipError_t launch_valu_k(const PropParams& p, hipStream_t stream) {
    const int64_t blocks = (p.n_leaves + 3) / 4;
    const size_t lds = 4 * (size_t)Stage<T, D>::BUF;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)propagate_valu<T, D, ORD, KB>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL((propagate_valu<T, D, ORD, KB>), dim3((unsigned)blocks), dim3(256), lds, stream, p);
    return hipGetLastError();
}

// Control-count buckets keep the per-lane sample registers small.
template <typename T, int D, int ORD>
hipError_t launch_valu_ord(const PropParams& p, hipStream_t stream) {
    if (p.K <= 1) return launch_valu_k<T, D, ORD, 1>(p, stream);
    if (p.K <= 2) return launch_valu_k<T, D, ORD, 2>(p, stream);
    if (p.K <= 4) return launch_valu_k<T, D, ORD, 4>(p, stream);
    return launch_valu_k<T, D, ORD, kMaxCtrl>(p, stream);
}

template <typename T, int D>
hipError_t launch_valu_one(const PropParams& p, hipStream_t stream) {
    return p.order == 2 ? launch_valu_ord<T, D, 2>(p, stream) : launch_valu_ord<T, D, 4>(p, stream);
}

}  // namespace

hipError_t launch_valu(int D, bool fp64, const PropParams& p, hipStream_t stream) {
    switch (D) {
        case 2: return fp64 ? launch_valu_one<double, 2>(p, stream) : launch_valu_one<float, 2>(p, stream);
        case 4: return fp64 ? launch_valu_one<double, 4>(p, stream) : launch_valu_one<float, 4>(p, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace pm
