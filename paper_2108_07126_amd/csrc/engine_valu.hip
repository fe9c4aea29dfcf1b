// VALU engine for dimensions 2 and 4: one slice per lane, all matrices in
// registers.  Lane l of a wave runs `chunk` consecutive slices
// [base + l*chunk, base + (l+1)*chunk) and keeps its own chain product; the
// 64 lane products are then multiplied by a pairwise tree across lanes
// (register shuffles), and the wave's product enters the same ticketed FP64
// tree as the MFMA engine's teams.
//
// Per slice: expand G = sum_m w_m B_m (FP64; the basis is wave-uniform and
// read through the scalar cache), 1-norm, planning with the wave maximum of
// the norms (one (m, s) per wave step keeps the lanes in lockstep), then
// exp(-i G) = C(Y) - i G S'(Y) with Y = G^2.  Every factor before U is a
// real polynomial in G, hence Hermitian and commuting with G, so only upper
// triangles are formed.
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
__device__ __forceinline__ void herm_ident(Herm<D, T>& a) {
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = i; j < D; ++j) {
            a.re[hidx<D>(i, j)] = (i == j) ? T(1) : T(0);
            a.im[hidx<D>(i, j)] = T(0);
        }
}

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

template <int D, typename T>
__device__ __forceinline__ void herm_axpy(Herm<D, T>& y, double a, const Herm<D, T>& x) {
    const T ta = (T)a;
#pragma unroll
    for (int e = 0; e < Herm<D, T>::NE; ++e) {
        y.re[e] += ta * x.re[e];
        y.im[e] += ta * x.im[e];
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

// exp(-i G) of a pre-scaled Hermitian G by the degree-m Taylor polynomial.
template <int D, typename T>
__device__ __forceinline__ Mat<D, T> taylor_exp(const Herm<D, T>& g, int m) {
    Herm<D, T> C, S;
    herm_ident(C);
    if (m <= 1) {
        S = g;
    } else {
        const int qc = m / 2, qs = (m - 1) / 2;
        const Herm<D, T> Y = herm_mul(g, g);
        Herm<D, T> Sp;
        herm_ident(Sp);
        herm_axpy(C, cos_coef(1), Y);
        if (qs >= 1) herm_axpy(Sp, sin_coef(1), Y);
        Herm<D, T> P = Y;
        for (int k = 2; k <= qc; ++k) {
            P = herm_mul(P, Y);
            herm_axpy(C, cos_coef(k), P);
            if (k <= qs) herm_axpy(Sp, sin_coef(k), P);
        }
        S = (qs >= 1) ? herm_mul(g, Sp) : g;
    }
    Mat<D, T> U;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            U.re[i * D + j] = C.gre(i, j) + S.gim(i, j);
            U.im[i * D + j] = C.gim(i, j) - S.gre(i, j);
        }
    return U;
}

// Basis layout of this engine: [m][D][D] interleaved complex, padded to D.
template <typename T, int D>
__global__ void __launch_bounds__(256) propagate_valu(PropParams p) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * 4 + wave_uniform((int)(threadIdx.x >> 6));
    if (wave >= p.n_leaves) return;
    // a leaf covers chunk slices; its 64 lanes split them into runs of `run`
    const int64_t run = p.chunk / 64;
    const int64_t base = wave * p.chunk + (int64_t)lane * run;
    Mat<D, T> Q;
    mat_ident(Q);
    for (int64_t i = 0; i < run; ++i) {
        const int64_t j = base + i;
        const bool valid = j < p.n_slices;
        Herm<D, double> g;
#pragma unroll
        for (int e = 0; e < Herm<D, double>::NE; ++e) g.re[e] = g.im[e] = 0.0;
        if (valid) {
            for (int m = 0; m < p.M; ++m) {
                const double w = slice_weight(p, j, m);
                const double* b = p.basis + (int64_t)m * D * D * 2;
#pragma unroll
                for (int r = 0; r < D; ++r)
#pragma unroll
                    for (int c = r; c < D; ++c) {
                        g.re[hidx<D>(r, c)] = fma(w, b[(r * D + c) * 2 + 0], g.re[hidx<D>(r, c)]);
                        g.im[hidx<D>(r, c)] = fma(w, b[(r * D + c) * 2 + 1], g.im[hidx<D>(r, c)]);
                    }
            }
        }
        double nu = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) {
            double cs = 0.0;
#pragma unroll
            for (int r = 0; r < D; ++r) {
                const double a = g.gre(r, c), b = g.gim(r, c);
                cs += sqrt(a * a + b * b);
            }
            nu = fmax(nu, cs);
        }
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) nu = fmax(nu, __shfl_xor(nu, off));
        nu = wave_uniform(nu);
        int m, s;
        plan_expm(p, nu, m, s);
        m = wave_uniform(m);
        s = wave_uniform(s);
        Herm<D, T> gt;
#pragma unroll
        for (int e = 0; e < Herm<D, T>::NE; ++e) {
            gt.re[e] = (T)ldexp(g.re[e], -s);
            gt.im[e] = (T)ldexp(g.im[e], -s);
        }
        Mat<D, T> U = taylor_exp<D, T>(gt, m);
        if (s > 0) {
            Mat<D, double> Ud = mat_convert<D, double>(U);
            for (int k = 0; k < s; ++k) Ud = mat_mul(Ud, Ud);
            U = mat_convert<D, T>(Ud);
        }
        if (valid) {
            if (p.slices_out) {
                T* out = reinterpret_cast<T*>(p.slices_out) + j * (int64_t)p.du * p.du * 2;
#pragma unroll
                for (int r = 0; r < D; ++r)
#pragma unroll
                    for (int c = 0; c < D; ++c)
                        if (r < p.du && c < p.du) {
                            out[(r * p.du + c) * 2 + 0] = U.re[r * D + c];
                            out[(r * p.du + c) * 2 + 1] = U.im[r * D + c];
                        }
            }
            Q = mat_mul(U, Q);
        }
    }
    // product over the wave's 64 consecutive runs: lane l+delta holds later slices
    Mat<D, double> W = mat_convert<D, double>(Q);
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

template <typename T, int D>
hipError_t launch_valu_one(const PropParams& p, hipStream_t stream) {
    const int64_t blocks = (p.n_leaves + 3) / 4;
    hipLaunchKernelGGL((propagate_valu<T, D>), dim3((unsigned)blocks), dim3(256), 0, stream, p);
    return hipGetLastError();
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
