// VALU engine for dimensions 2 and 4 (instantiated per element type and
// dimension in the engine_valu_*.hip units): one slice per lane, all
// matrices in registers.  Lane l of a wave runs `chunk/64` consecutive
// slices and keeps its own chain product; the 64 lane products are then
// multiplied by a pairwise tree across lanes (register shuffles), the four
// waves of a block are combined in LDS, and the block's product enters the
// ticketed FP64 tree shared with the MFMA engine's design.
//
// Per slice: expand G = sum_m w_m B_m (FP64; the block keeps the basis in
// LDS), shift by the mean eigenvalue mu = tr G / D (exp(-i G) =
// e^{-i mu} exp(-i (G - mu I)); the chain collects the phases and applies
// them once per run), bound the 1-norm of the shifted matrix, plan once per
// wave (maximum over its lanes), and evaluate the truncated Taylor series of
// exp(-i X), X = (G - mu I)/2^s, in the D-dimensional algebra spanned by
// I, X, .., X^{D-1} (Cayley-Hamilton: the series becomes D scalar
// recurrences; D = 4 needs the matrix power X^2 only), then square s times
// in FP64.  Per-slice output goes through a per-wave LDS staging buffer and
// leaves as whole cache lines.
#pragma once

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

// Q <- U Q, one column of Q at a time (a column of the product depends only
// on the same column of Q), so no second full matrix is live.
template <int D, typename T>
__device__ __forceinline__ void mat_lmul_inplace(const Mat<D, T>& u, Mat<D, T>& q) {
#pragma unroll
    for (int j = 0; j < D; ++j) {
        T cr[D], ci[D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            cr[k] = q.re[k * D + j];
            ci[k] = q.im[k * D + j];
        }
#pragma unroll
        for (int i = 0; i < D; ++i) {
            T sr = 0, si = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const T ar = u.re[i * D + k], ai = u.im[i * D + k];
                sr = fma(ar, cr[k], sr);
                sr = fma(-ai, ci[k], sr);
                si = fma(ar, ci[k], si);
                si = fma(ai, cr[k], si);
            }
            q.re[i * D + j] = sr;
            q.im[i * D + j] = si;
        }
    }
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
// With EXCESS the k = 0 term (the identity) is left out.  Unrolled to the
// largest degree so the series coefficients are immediates; the degree m is
// wave-uniform, so the early exits are scalar branches.
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
#pragma unroll
    for (int q = 0; q <= kMaxDeg / 2; ++q) {
        if (2 * q + 1 > m) break;
        ch_step<D>(a, r);
        const double sc = sin_coef(q);
#pragma unroll
        for (int i = 0; i < D; ++i) cim[i] = fma(-sc, a[i], cim[i]);
        if (2 * q + 2 > m || q + 1 > 10) break;
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
// Clenshaw recurrence of the Chebyshev series in the algebra:
// D_k = a_k I + 2 X D_{k+1} - D_{k+2} on complex coefficient vectors,
// a_k = (-i)^k J_k(theta) from the table row jk; result D_0 - D_2.
template <int D>
__device__ __forceinline__ void ch_clenshaw(const double (&r)[D], int m, const double* jk, double (&cre)[D],
                                            double (&cim)[D]) {
    double d1r[D], d1i[D], d2r[D], d2i[D], kr[D], ki[D];
#pragma unroll
    for (int i = 0; i < D; ++i) d1r[i] = d1i[i] = d2r[i] = d2i[i] = kr[i] = ki[i] = 0.0;
#pragma unroll
    for (int k = kMaxCheb; k >= 0; --k) {
        if (k > m) continue;
        double pr[D], pi[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            pr[i] = d1r[i];
            pi[i] = d1i[i];
        }
        ch_step<D>(pr, r);
        ch_step<D>(pi, r);
        const double jv = jk[k];
        const int q = k & 3;
        double dr[D], di[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            dr[i] = fma(2.0, pr[i], -d2r[i]);
            di[i] = fma(2.0, pi[i], -d2i[i]);
        }
        dr[0] += q == 0 ? jv : (q == 2 ? -jv : 0.0);
        di[0] += q == 1 ? -jv : (q == 3 ? jv : 0.0);
        if (k == 0) {
#pragma unroll
            for (int i = 0; i < D; ++i) {
                kr[i] = d2r[i];
                ki[i] = d2i[i];
            }
        }
#pragma unroll
        for (int i = 0; i < D; ++i) {
            d2r[i] = d1r[i];
            d2i[i] = d1i[i];
            d1r[i] = dr[i];
            d1i[i] = di[i];
        }
    }
#pragma unroll
    for (int i = 0; i < D; ++i) {
        cre[i] = d1r[i] - kr[i];
        cim[i] = d1i[i] - ki[i];
    }
}

enum { EXP_TAYLOR = 0, EXP_TAYLOR_EXCESS = 1, EXP_CHEBYSHEV = 2 };

// exp(-i X) of a pre-scaled Hermitian X, evaluated in the algebra generated
// by X: by Cayley-Hamilton every power X^k with k >= D is a combination of
// I, X, .., X^{D-1}, so the polynomial is carried as D complex coefficients
// (scalar recurrences) and the matrix is formed once from the powers
// X^0..X^{D-1}.  KIND: the degree-m Taylor series (EXP_TAYLOR), the same
// without its identity term (EXP_TAYLOR_EXCESS: exp(-i X) - I, accurate
// relative to ||X||), or the degree-m Chebyshev series on [-theta, theta]
// (EXP_CHEBYSHEV; X is first divided by theta).  The results are the same
// truncated series as the matrix evaluations; only the order of operations
// differs.
template <int D, typename T, int KIND>
__device__ __forceinline__ Mat<D, T> exp_ch(Herm<D, T> x, int m, const double* jk = nullptr, double theta = 1.0) {
    static_assert(D == 2 || D == 4, "algebra evaluation for D = 2 and 4");
    if constexpr (KIND == EXP_CHEBYSHEV) {
        const T inv = (T)(1.0 / theta);
#pragma unroll
        for (int e = 0; e < Herm<D, T>::NE; ++e) {
            x.re[e] *= inv;
            x.im[e] *= inv;
        }
    }
    double pw[D + 1];
    double tr1 = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) tr1 += (double)x.re[hidx<D>(i, i)];
    pw[0] = (double)D;
    pw[1] = tr1;
    pw[2] = herm_trace_prod<D, T>(x, x);
    Herm<D, T> x2;
    if constexpr (D == 4) {
        // tr X^3 = <X, X^2>_F and tr X^4 = <X^2, X^2>_F; X^3 is never stored
        x2 = herm_mul(x, x);
        pw[3] = herm_trace_prod<D, T>(x, x2);
        pw[4] = herm_trace_prod<D, T>(x2, x2);
    }
    double r[D], cre[D], cim[D];
    ch_coeffs<D>(pw, r);
    if constexpr (KIND == EXP_CHEBYSHEV) ch_clenshaw<D>(r, m, jk, cre, cim);
    else ch_taylor<D, KIND == EXP_TAYLOR_EXCESS>(r, m, cre, cim);
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
                // (X^3)_{ab} = sum_k X_{ak} (X^2)_{kb}
                double tr = 0.0, ti = 0.0;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const double ar = x.gre(a, k), ai = x.gim(a, k);
                    const double br = x2.gre(k, b), bi = x2.gim(k, b);
                    tr = fma(ar, br, fma(-ai, bi, tr));
                    ti = fma(ar, bi, fma(ai, br, ti));
                }
                xr[3] = tr;
                xi[3] = ti;
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

// The control samples one exponent needs: K values (order 2) or the three
// Simpson samples of each control (order 4; for the commutator-free scheme
// those of slice j >> 1, mirrored for its second factor), K <= KB.  Loaded for the next
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
        } else if constexpr (ORD == kOrderCF4) {
            const double* ck = c + (int64_t)kk * S + (j & ~(int64_t)1);
            const bool second = (j & 1) != 0;
            s.v[3 * k + 0] = ck[second ? 2 : 0];
            s.v[3 * k + 1] = ck[1];
            s.v[3 * k + 2] = ck[second ? 0 : 2];
        } else {
            const double* ck = c + (int64_t)kk * S + 2 * j;
            s.v[3 * k + 0] = ck[0];
            s.v[3 * k + 1] = ck[1];
            s.v[3 * k + 2] = ck[2];
        }
    }
    return s;
}

// Midpoint-rule samples (order 2) in blocks of SB consecutive slices per
// lane.  A lane's slices are a contiguous run, `run` samples away from the
// next lane's, so a load for one slice touches a different line in every
// lane; issued slice by slice, each line is fetched again for every piece
// of it once other traffic (the per-slice output) has evicted it in between.
// Here a lane reads the SB samples of a control that its next SB slices
// need at once, as SB / 2 contiguous 16-byte pieces, one block ahead of
// their use.  Piece q holds the samples a, a + 1 (a = first + 2 q); a piece
// that would pass the last sample is moved back to the last two, and a
// slice past the end takes some sample (its exponent is zero).
template <int KB, int SB>
struct SampleBlock {
    double v[KB][SB];
};

template <int KB, int SB>
__device__ __forceinline__ void load_block(const PropParams& p, int64_t first, SampleBlock<KB, SB>& b) {
    static_assert(SB % 2 == 0, "whole 16-byte pieces");
    const int64_t S = p.n_samples;
    if (p.K == 0 || S < 2) {
        // no samples, or a single one (N = 1): every slice reads sample 0
#pragma unroll
        for (int k = 0; k < KB; ++k)
#pragma unroll
            for (int r = 0; r < SB; ++r) b.v[k][r] = p.K == 0 ? 0.0 : p.samples[(int64_t)min(k, p.K - 1) * S];
        return;
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        const double* row = p.samples + (int64_t)min(k, p.K - 1) * S;
#pragma unroll
        for (int q = 0; q < SB / 2; ++q) {
            const int64_t a = first + 2 * q;
            const bool inner = a < S - 1;
            struct alignas(8) Pair { double x, y; } v;
            __builtin_memcpy(&v, row + (inner ? a : S - 2), sizeof(v));
            b.v[k][2 * q] = inner ? v.x : v.y;
            b.v[k][2 * q + 1] = v.y;
        }
    }
}

// Expand one slice into the upper triangle of G (FP64): the weights of the
// midpoint rule (order 2) or of eq. magnus_coeffs (order 4, pairs i[H_a,H_b]
// with a < b in lexicographic order after the 2K single-control terms).
template <int D, int ORD, int KB>
__device__ __forceinline__ Herm<D, double> expand_slice(const PropParams& p, const double* basis,
                                                        const SampleSet<ORD, KB>& x, bool valid) {
    Herm<D, double> g;
#pragma unroll
    for (int e = 0; e < Herm<D, double>::NE; ++e) g.re[e] = g.im[e] = 0.0;
    const double h = valid ? p.h : 0.0;
    const int K = p.K;
    auto add = [&](double w, int m) {
        const double* b = basis + m * D * D * 2;
#pragma unroll
        for (int r = 0; r < D; ++r)
#pragma unroll
            for (int cc = r; cc < D; ++cc) {
                g.re[hidx<D>(r, cc)] = fma(w, b[(r * D + cc) * 2 + 0], g.re[hidx<D>(r, cc)]);
                g.im[hidx<D>(r, cc)] = fma(w, b[(r * D + cc) * 2 + 1], g.im[hidx<D>(r, cc)]);
            }
    };
    if constexpr (ORD == kOrderCF4) {
        // one factor of the commutator-free step: (h/2) H0 + (h/12)(3 s0 + 4 s1 - s2) H_k
        add(0.5 * h, 0);
        const double h12 = h * (1.0 / 12.0);
#pragma unroll
        for (int k = 0; k < KB; ++k)
            if (k < K) add(h12 * (3.0 * x.v[3 * k] + 4.0 * x.v[3 * k + 1] - x.v[3 * k + 2]), 1 + k);
        return g;
    }
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
            // hardware square root (within 1 ulp; the inflation below covers it)
            const float a = __builtin_amdgcn_sqrtf((float)(g.re[e] * g.re[e] + g.im[e] * g.im[e]));
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

// (cos mu, sin mu) by the Taylor series on mu / 2^s, |mu / 2^s| <= 1/2
// (remainder below 2^-60), then s double-angle steps: a few dozen FP64
// operations where a library sincos costs several times that.
__device__ __forceinline__ void phase_cs(double mu, double& cs, double& sn) {
    int e = 0;
    (void)frexp(mu, &e);            // |mu| < 2^e
    const int s = max(0, e + 1);    // |mu| / 2^s < 1/2
    const double x = ldexp(mu, -s), y = x * x;
    double c = 1.0 / 20922789888000.0, t = 1.0 / 1307674368000.0;   // 1/16!, 1/15!
    c = fma(c, -y, 1.0 / 87178291200.0);
    t = fma(t, -y, 1.0 / 6227020800.0);
    c = fma(c, -y, 1.0 / 479001600.0);
    t = fma(t, -y, 1.0 / 39916800.0);
    c = fma(c, -y, 1.0 / 3628800.0);
    t = fma(t, -y, 1.0 / 362880.0);
    c = fma(c, -y, 1.0 / 40320.0);
    t = fma(t, -y, 1.0 / 5040.0);
    c = fma(c, -y, 1.0 / 720.0);
    t = fma(t, -y, 1.0 / 120.0);
    c = fma(c, -y, 1.0 / 24.0);
    t = fma(t, -y, 1.0 / 6.0);
    c = fma(c, -y, 0.5);
    t = fma(t, -y, 1.0);
    c = fma(c, -y, 1.0);
    double sv = t * x;
    for (int k = 0; k < s; ++k) {
        const double c2 = fma(c, c, -sv * sv);
        sv = 2.0 * c * sv;
        c = c2;
    }
    cs = c;
    sn = sv;
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
typedef unsigned v4u __attribute__((ext_vector_type(4)));

template <typename T, int D>
struct Stage {
    static constexpr int SB = D * D * 2 * (int)sizeof(T);   // bytes per slice
    static constexpr int R = SB >= 128 ? 1 : 128 / SB;      // slices per segment: whole 128-byte
                                                             // lines (R divides the runs' blocks)
    static constexpr int SEG = R * SB;
    static constexpr int STRIDE = SEG + 16;                  // padded against bank conflicts
    static constexpr int BUF = 64 * STRIDE;                  // bytes per wave
    static constexpr int PIECES = SEG / 16;                  // 16-byte pieces per segment
};

// The phased slice e^{-i mu} (U or I + U) into this lane's staging row.
// A wave whose slices all have mu = 0 (traceless Hamiltonians) skips the
// rotation, which would multiply by exactly 1 and 0.
template <int D, typename T>
__device__ __forceinline__ void stage_phased(char* row, const Mat<D, T>& U, double mu, bool plus_ident,
                                             bool phased) {
    T* out = reinterpret_cast<T*>(row);
    if (!phased) {
#pragma unroll
        for (int e = 0; e < D * D; ++e) {
            out[2 * e + 0] = (plus_ident && e % (D + 1) == 0) ? (T)((double)U.re[e] + 1.0) : U.re[e];
            out[2 * e + 1] = U.im[e];
        }
        return;
    }
    double sn, cs;
    phase_cs(mu, cs, sn);
#pragma unroll
    for (int e = 0; e < D * D; ++e) {
        const double ur = (double)U.re[e] + ((plus_ident && e % (D + 1) == 0) ? 1.0 : 0.0);
        const double ui = (double)U.im[e];
        out[2 * e + 0] = (T)(cs * ur + sn * ui);
        out[2 * e + 1] = (T)(cs * ui - sn * ur);
    }
}

// Write the staged segments of the wave: lane l's R slices starting at
// slice first + l * run.  Buffer stores with the range limited to the
// slices that exist: pieces past the end are dropped by the hardware range
// check, so the stores need no branches (and the compiler's wait counts stay
// exact, letting the stores overlap the next slices' arithmetic).  D = 4 and
// the FP64 D = 2 kernel mark them non-temporal: at D = 4 measured 5 % faster;
// at D = 2 in FP64 the same time, but the output stream no longer evicts the
// sample lines that lanes are still reading (HBM reads 1.61 -> 0.62 GB per
// launch of 2^26 slices, the samples being 0.54 GB).
template <typename T, int D>
__device__ __forceinline__ void flush_stage(const PropParams& p, const char* buf, int64_t first, int64_t run,
                                            int lane) {
    using S = Stage<T, D>;
    constexpr bool kNT = D == 4 || std::is_same<T, double>::value;
    const int64_t avail = p.n_slices - first;
    const int64_t span = 64 * run;
    const unsigned nrec = (unsigned)((avail < span ? (avail > 0 ? avail : 0) : span) * S::SB);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        reinterpret_cast<char*>(p.slices_out) + first * S::SB, (short)0, (int)nrec, 0x00020000);
#pragma unroll
    for (int q = 0; q < S::PIECES; ++q) {
        const int piece = q * 64 + lane;
        const int seg = piece / S::PIECES, off = piece % S::PIECES;
        const v4u v = *reinterpret_cast<const v4u*>(buf + seg * S::STRIDE + off * 16);
        __builtin_amdgcn_raw_buffer_store_b128(v, rs, (int)(seg * run * S::SB + off * 16), 0, kNT ? 2 : 0);
    }
}

// Order this wave's LDS writes before its reads of other lanes' rows (and
// the reverse): a wave's LDS operations execute in order, so only the
// compiler must be kept from moving them across this point.
// As many buffer stores as a flush issues, to a zero-length range (all
// dropped): placed after the first sample loads so that the loop is entered
// with the same pending memory operations as it is re-entered after a flush,
// which keeps the compiler's wait before the first use of the samples at
// "all but the flush's stores" instead of "everything".
template <typename T, int D>
__device__ __forceinline__ void dummy_flush(const PropParams& p, int lane) {
    using S = Stage<T, D>;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(p.slices_out, (short)0, 0, 0x00020000);
    const v4u z = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int q = 0; q < S::PIECES; ++q) __builtin_amdgcn_raw_buffer_store_b128(z, rs, (q * 64 + lane) * 16, 0, 0);
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// One slice per lane, all matrices in registers.  A leaf (one wave) covers
// `chunk` consecutive slices: lane l multiplies the run
// [base + l*run, base + (l+1)*run) into its own chain product.
// Output modes of the kernel: no per-slice output, staged (coalesced)
// output when the user dimension equals D, or direct per-lane stores for the
// embedded dimensions 1 and 3.
enum { OUT_NONE = 0, OUT_STAGED = 1, OUT_DIRECT = 2 };

template <typename T, int D, int ORD, int KB, int OUT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(D == 2 ? 2 : 1, 8)))
propagate_valu(PropParams p) {
    const int lane = threadIdx.x & 63;
    const int wib = wave_uniform((int)(threadIdx.x >> 6));
    // wave = chain; waves past the last chain run no slices (identity)
    const int64_t wave = (int64_t)blockIdx.x * 4 + wib;
    extern __shared__ char stage_lds[];
    using S = Stage<T, D>;
    // the block's copy of the basis (after the four staging buffers)
    double* lbasis = reinterpret_cast<double*>(stage_lds + 4 * S::BUF);
    block_copy_to_lds(lbasis, p.basis, p.M * D * D * 2);
    __syncthreads();
    char* sbuf = stage_lds + wib * S::BUF;
    char* srow = sbuf + lane * S::STRIDE;
    // a lane's run is a multiple of 16 slices (two sample blocks, 2 S::R)
    const int64_t cfirst = chain_first(p, wave);
    const int64_t run = wave < p.n_chains ? (chain_first(p, wave + 1) - cfirst) / 64 : 0;
    const int64_t base = cfirst + (int64_t)lane * run;
    const double lth = lane_theta_of(p, lane);
    const double lcth = lane_ctheta_of(p, lane);
    constexpr bool kF64 = std::is_same<T, double>::value;
    const bool cheb = kF64 && p.method == PM_EXPM_CHEBYSHEV;
    // The scalar phases e^{-i mu_j} commute with everything: the chain
    // multiplies the phase-free factors and the lane applies e^{-i sum mu}
    // once at the end of its run.  FP64: Q <- U Q.  Reduced modes: slices as
    // I + E and Q <- Q + E Q with Q in FP64.  Slices past the end have G = 0,
    // whose factor is exactly I (E = 0), so they multiply in unconditionally.
    Mat<D, T> Q;
    mat_ident(Q);
    Mat<D, double> Qx;
    mat_ident(Qx);
    double phi = 0.0;
    const int64_t last = p.n_slices - 1;
    // One slice: expand, shift, plan, exponentiate, stage or store, chain.
    auto step = [&](const SampleSet<ORD, KB>& cur, int64_t j, int r) {
        const bool valid = j < p.n_slices;
        Herm<D, double> g = expand_slice<D, ORD, KB>(p, lbasis, cur, valid);
        // shift by the mean eigenvalue: exp(-i G) = e^{-i mu} exp(-i (G - mu I))
        double mu = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) mu += g.re[hidx<D>(a, a)];
        mu *= 1.0 / D;
#pragma unroll
        for (int a = 0; a < D; ++a) g.re[hidx<D>(a, a)] -= mu;
        const bool phased = __ballot(mu != 0.0) != 0;
        const double nu = (double)wave_max_f(norm1_bound<D>(g));
        int m, s;
        if (cheb) plan_cheb_lanes(p, nu, lane, lcth, m, s);
        else plan_valu(p, nu, lane, lth, m, s);
        Herm<D, T> x;
#pragma unroll
        for (int e = 0; e < Herm<D, T>::NE; ++e) {
            x.re[e] = (T)ldexp(g.re[e], -s);
            x.im[e] = (T)ldexp(g.im[e], -s);
        }
        if constexpr (kF64) {
            Mat<D, T> U = cheb ? exp_ch<D, T, EXP_CHEBYSHEV>(x, m, p.cheb_j + m * (kMaxCheb + 1), p.ctheta[m])
                               : exp_ch<D, T, EXP_TAYLOR>(x, m);
            for (int k = 0; k < s; ++k) U = mat_mul(U, U);
            if constexpr (OUT == OUT_STAGED) stage_phased<D, T>(srow + r * S::SB, U, mu, false, phased);
            if constexpr (OUT == OUT_DIRECT)
                if (valid) store_phased<D, T>(p, j, U, mu, false);
            mat_lmul_inplace<D, T>(U, Q);
        } else {
            Mat<D, T> E = exp_ch<D, T, EXP_TAYLOR_EXCESS>(x, m);
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
            if constexpr (OUT == OUT_STAGED) stage_phased<D, T>(srow + r * S::SB, E, mu, true, phased);
            if constexpr (OUT == OUT_DIRECT)
                if (valid) store_phased<D, T>(p, j, E, mu, true);
            const Mat<D, T> P = mat_mul(E, mat_convert<D, T>(Qx));
#pragma unroll
            for (int e = 0; e < D * D; ++e) {
                Qx.re[e] += (double)P.re[e];
                Qx.im[e] += (double)P.im[e];
            }
        }
        phi += mu;
    };
    // The staged output of the R slices of the run that end at step i1.
    auto flush = [&](int64_t i1) {
        if constexpr (OUT == OUT_STAGED) {
            wave_lds_sync();
            flush_stage<T, D>(p, sbuf, cfirst + i1 - S::R, run, lane);
            wave_lds_sync();
        }
    };
    if constexpr (ORD == 2) {
        // Samples in blocks of SB slices, one block ahead (load_block): the
        // FP64 two-dimensional kernel with output runs its blocks unrolled
        // (UNR), everything else one slice per pass of a loop.  Blocks of 8
        // (64 bytes per control) where the controls are few; 4 in the
        // unrolled kernel, whose 16 unrolled slices of 8 would hold more
        // registers.
        constexpr bool UNR = D == 2 && kF64 && OUT == OUT_STAGED;
        constexpr int SB0 = KB > 2 ? 2 : (UNR ? 4 : 8);
        constexpr int SB = (OUT == OUT_STAGED && SB0 < S::R) ? S::R : SB0;
        static_assert(OUT != OUT_STAGED || SB % S::R == 0, "segments inside a block");
        using Blk = SampleBlock<KB, SB>;
        auto slice_of = [&](const Blk& b, int r) {
            SampleSet<2, KB> x;
#pragma unroll
            for (int k = 0; k < KB; ++k) x.v[k] = b.v[k][r];
            return x;
        };
        if constexpr (UNR) {
            // Two blocks in alternating registers, each run straight through:
            // a block's loads are issued before the previous block's output
            // stores, so waiting for them never waits for those stores (the
            // zero-length stores before the loop give its first pass the
            // same count of younger stores as every later pass).
            auto block = [&](const Blk& b, int64_t i0) {
#pragma unroll
                for (int r = 0; r < SB; ++r) {
                    step(slice_of(b, r), base + i0 + r, r % S::R);
                    if ((r + 1) % S::R == 0) flush(i0 + r + 1);
                    // the slices' exponentials are independent: keep the
                    // scheduler from overlapping them (their registers
                    // would spill)
                    __builtin_amdgcn_sched_barrier(0);
                }
            };
            Blk A, B;
            load_block<KB, SB>(p, base, A);
            if constexpr (OUT == OUT_STAGED)
#pragma unroll
                for (int q = 0; q < SB / S::R; ++q) dummy_flush<T, D>(p, lane);
            for (int64_t i0 = 0; i0 < run; i0 += 2 * SB) {
                load_block<KB, SB>(p, base + i0 + SB, B);
                block(A, i0);
                load_block<KB, SB>(p, base + i0 + 2 * SB, A);
                block(B, i0 + SB);
            }
        } else {
            // One slice per pass of a loop (D = 4: an unrolled block would
            // not fit the instruction cache; D = 2 without output or in FP32:
            // as fast, fewer registers); the current block shifts down by one
            // slot per slice and takes over the next block, loaded a block
            // earlier, when it is used up.
            Blk A, B;
            load_block<KB, SB>(p, base, A);
            load_block<KB, SB>(p, base + SB, B);
            for (int64_t i = 0; i < run; ++i) {
                const SampleSet<2, KB> cur = slice_of(A, 0);
#pragma unroll
                for (int k = 0; k < KB; ++k)
#pragma unroll
                    for (int r = 0; r + 1 < SB; ++r) A.v[k][r] = A.v[k][r + 1];
                step(cur, base + i, (int)(i % S::R));
                if ((i + 1) % S::R == 0) flush(i + 1);
                if ((i + 1) % SB == 0) {
                    A = B;
                    load_block<KB, SB>(p, base + i + 1 + SB, B);
                }
            }
        }
    } else {
        // Orders 4 and CF4: R slices' samples per group, one group ahead.
        auto group = [&](const SampleSet<ORD, KB> (&cur)[S::R], int64_t i0) {
#pragma unroll
            for (int r = 0; r < S::R; ++r) step(cur[r], base + i0 + r, r);
            flush(i0 + S::R);
        };
        auto load_group = [&](SampleSet<ORD, KB> (&dst)[S::R], int64_t i0) {
#pragma unroll
            for (int r = 0; r < S::R; ++r) dst[r] = load_samples<ORD, KB>(p, min(base + i0 + r, last));
        };
        if constexpr (D == 2) {
            SampleSet<ORD, KB> A[S::R], B[S::R];
            load_group(A, 0);
            if constexpr (OUT == OUT_STAGED) dummy_flush<T, D>(p, lane);
            for (int64_t i0 = 0; i0 < run; i0 += 2 * S::R) {
                load_group(B, i0 + S::R);
                group(A, i0);
                load_group(A, i0 + 2 * S::R);
                group(B, i0 + S::R);
            }
        } else {
            // D = 4 keeps one sample set in flight; S::R = 1 here.
            SampleSet<ORD, KB> A[S::R];
            load_group(A, 0);
            for (int64_t i0 = 0; i0 < run; i0 += S::R) {
                const SampleSet<ORD, KB> cur = A[0];
                load_group(A, i0 + S::R);
                const SampleSet<ORD, KB> C[S::R] = {cur};
                group(C, i0);
            }
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
    // the block's four consecutive chains, combined in LDS (later chain on
    // the left): the block is one leaf of the tree
    double* comb = reinterpret_cast<double*>(stage_lds);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int e = 0; e < D * D; ++e) {
            comb[(wib * D * D + e) * 2 + 0] = W.re[e];
            comb[(wib * D * D + e) * 2 + 1] = W.im[e];
        }
    }
    __syncthreads();
    if (wib != 0) return;
#pragma unroll
    for (int w = 1; w < 4; ++w) {
        Mat<D, double> O;
#pragma unroll
        for (int e = 0; e < D * D; ++e) {
            O.re[e] = comb[(w * D * D + e) * 2 + 0];
            O.im[e] = comb[(w * D * D + e) * 2 + 1];
        }
        W = mat_mul(O, W);
    }
    // ticketed product tree with fan-in kFanIn over the blocks' products
    // (FP64): a block publishes its node with a release fence before the
    // group's ticket; only the group's last arrival acquires, multiplies the
    // group's nodes (later on the left) and goes on
    const int64_t NN = (int64_t)D * D * 2;
    auto load_node = [&](int64_t at) {
        const double* nd = p.nodes + at * NN;
        Mat<D, double> O;
#pragma unroll
        for (int e = 0; e < D * D; ++e) {
            O.re[e] = nd[2 * e + 0];
            O.im[e] = nd[2 * e + 1];
        }
        return O;
    };
    int64_t idx = blockIdx.x, cnt = p.n_leaves, off = 0;
    while (cnt > 1) {
        const int64_t pcnt = (cnt + kFanIn - 1) / kFanIn, poff = off + cnt, grp = idx / kFanIn;
        const int64_t first = grp * kFanIn;
        const int64_t members = min(cnt, first + kFanIn) - first;
        if (members > 1) {
            double* node = p.nodes + (off + idx) * NN;
            if (lane == 0) {
#pragma unroll
                for (int e = 0; e < D * D; ++e) {
                    node[2 * e + 0] = W.re[e];
                    node[2 * e + 1] = W.im[e];
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            unsigned v = 0;
            if (lane == 0) v = atomicAdd(&p.counters[poff + grp], 1u);
            const unsigned t = (unsigned)wave_uniform((int)__shfl(v, 0));
            if (t != (unsigned)(members - 1)) return;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            if (lane == 0) atomicExch(&p.counters[poff + grp], 0u);
            const int64_t lastn = first + members - 1;
            Mat<D, double> P = lastn == idx ? W : load_node(off + lastn);
            for (int64_t k = lastn - 1; k >= first; --k) P = mat_mul(P, k == idx ? W : load_node(off + k));
            W = P;
        }
        idx = grp;
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

template <typename T, int D, int ORD, int KB, int OUT>
hipError_t launch_valu_k(const PropParams& p, hipStream_t stream) {
    const int64_t blocks = p.n_leaves;   // a block of four chains is a leaf
    const size_t lds = 4 * (size_t)Stage<T, D>::BUF + sizeof(double) * (size_t)p.M * D * D * 2;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)propagate_valu<T, D, ORD, KB, OUT>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)(4 * (size_t)Stage<T, D>::BUF + sizeof(double) * kMaxBasis * D * D * 2));
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL((propagate_valu<T, D, ORD, KB, OUT>), dim3((unsigned)blocks), dim3(256), lds, stream, p);
    return hipGetLastError();
}

// Control-count buckets keep the per-lane sample registers small; the
// direct-store variant (dimensions 1 and 3 with per-slice output) takes the
// general bucket only.
template <typename T, int D, int ORD>
hipError_t launch_valu_ord(const PropParams& p, hipStream_t stream) {
    if (p.slices_out && p.du != D) return launch_valu_k<T, D, ORD, kMaxCtrl, OUT_DIRECT>(p, stream);
    if (p.slices_out) {
        if (p.K <= 1) return launch_valu_k<T, D, ORD, 1, OUT_STAGED>(p, stream);
        if (p.K <= 2) return launch_valu_k<T, D, ORD, 2, OUT_STAGED>(p, stream);
        return launch_valu_k<T, D, ORD, kMaxCtrl, OUT_STAGED>(p, stream);
    }
    if (p.K <= 1) return launch_valu_k<T, D, ORD, 1, OUT_NONE>(p, stream);
    if (p.K <= 2) return launch_valu_k<T, D, ORD, 2, OUT_NONE>(p, stream);
    return launch_valu_k<T, D, ORD, kMaxCtrl, OUT_NONE>(p, stream);
}

// The commutator-free scheme has no per-slice output (the host rejects it).
template <typename T, int D>
hipError_t launch_valu_cf4(const PropParams& p, hipStream_t stream) {
    if (p.slices_out) return hipErrorInvalidValue;
    if (p.K <= 2) return launch_valu_k<T, D, kOrderCF4, 2, OUT_NONE>(p, stream);
    return launch_valu_k<T, D, kOrderCF4, kMaxCtrl, OUT_NONE>(p, stream);
}

template <typename T, int D>
hipError_t launch_valu_one(const PropParams& p, hipStream_t stream) {
    if (p.order == kOrderCF4) return launch_valu_cf4<T, D>(p, stream);
    return p.order == 2 ? launch_valu_ord<T, D, 2>(p, stream) : launch_valu_ord<T, D, 4>(p, stream);
}

}  // namespace
}  // namespace pm
