// Tile machinery of the MFMA engines: one wave owns a 16x16 tile of every
// D x D complex matrix (accumulator layout of the 16x16x4 MFMA products);
// complex products stage both operands in LDS slots.  Shared by the
// propagation and gradient kernels.
#pragma once

#include <type_traits>

#include "engine_common.h"

namespace pm {
namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

template <typename T> struct V4;
template <> struct V4<double> { using type = d4_t; };
template <> struct V4<float> { using type = f4_t; };

__device__ __forceinline__ d4_t mfma16(double a, double b, d4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma16(float a, float b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T>
struct Tile {
    T re[4], im[4];
};

// Row (within a 16x16 tile) of accumulator register r in lane group g.  The
// FP32 16x16x4 product leaves rows 4g..4g+3 in a lane; the FP64 one
// interleaves them as g, g+4, g+8, g+12.  Column = lane & 15 for both.
template <typename T> __device__ __forceinline__ int crow(int g, int r);
template <> __device__ __forceinline__ int crow<double>(int g, int r) { return g + 4 * r; }
template <> __device__ __forceinline__ int crow<float>(int g, int r) { return 4 * g + r; }

template <int D_, int NT_>
struct Geo {
    static constexpr int D = D_;
    static constexpr int TD = D / 16;
    static constexpr int TW = TD * TD;   // waves per team
    static constexpr int NT = NT_;       // teams per block
    static constexpr int THREADS = 64 * TW * NT;
    static constexpr int LD = D + 1;     // padded LDS row stride
    static constexpr int PLANE = D * LD;
    static constexpr int SLOT = 2 * PLANE;   // in doubles (a float slot uses the front half)
    static_assert(TW == 1 || NT == 1, "multi-wave teams own their whole block");
};

// Per-wave coordinates.
struct Lane {
    int lane, g, j, TI, TJ, wt;
};

template <class G>
__device__ __forceinline__ void team_sync() {
    if constexpr (G::TW == 1) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    } else {
        __syncthreads();
    }
}

template <typename T>
__device__ __forceinline__ Tile<T> ident(const Lane& L) {
    Tile<T> t;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        t.re[r] = (16 * L.TI + crow<T>(L.g, r) == 16 * L.TJ + L.j) ? T(1) : T(0);
        t.im[r] = T(0);
    }
    return t;
}

template <typename T>
__device__ __forceinline__ void axpy(Tile<T>& y, double a, const Tile<T>& x) {
    const T ta = (T)a;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        y.re[r] += ta * x.re[r];
        y.im[r] += ta * x.im[r];
    }
}

template <class G, typename T>
__device__ __forceinline__ void slot_store(double* slot, const Tile<T>& t, const Lane& L) {
    T* re = reinterpret_cast<T*>(slot);
    T* im = re + G::PLANE;
    const int col = 16 * L.TJ + L.j;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 16 * L.TI + crow<T>(L.g, r);
        re[row * G::LD + col] = t.re[r];
        im[row * G::LD + col] = t.im[r];
    }
}

// Change a tile's element type; the register layouts differ between FP32
// and FP64 accumulators, so the values travel through an LDS slot.
template <class G, typename Tdst, typename Tsrc>
__device__ __forceinline__ Tile<Tdst> relayout(const Tile<Tsrc>& t, double* slot, const Lane& L) {
    if constexpr (std::is_same<Tdst, Tsrc>::value) {
        return t;
    } else {
        team_sync<G>();
        slot_store<G, Tsrc>(slot, t, L);
        team_sync<G>();
        const Tsrc* re = reinterpret_cast<const Tsrc*>(slot);
        const Tsrc* im = re + G::PLANE;
        const int col = 16 * L.TJ + L.j;
        Tile<Tdst> o;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * L.TI + crow<Tdst>(L.g, r);
            o.re[r] = (Tdst)re[row * G::LD + col];
            o.im[r] = (Tdst)im[row * G::LD + col];
        }
        return o;
    }
}

// Tile (TI, TJ) of A * B, A and B complex D x D in LDS slots.
template <class G, typename T>
__device__ __forceinline__ Tile<T> slot_mul(const double* A, const double* B, const Lane& L) {
    using V = typename V4<T>::type;
    const T* Are = reinterpret_cast<const T*>(A);
    const T* Aim = Are + G::PLANE;
    const T* Bre = reinterpret_cast<const T*>(B);
    const T* Bim = Bre + G::PLANE;
    // Re = sum Ar Br + (-Ai) Bi and Im = sum Ar Bi + Ai Br accumulate in two
    // interleaved chains, so no combine step follows the MFMAs.
    V acc_re = {0, 0, 0, 0}, acc_im = {0, 0, 0, 0};
    const int arow = (16 * L.TI + L.j) * G::LD;
    const int bcol = 16 * L.TJ + L.j;
#pragma unroll
    for (int kb = 0; kb < G::D / 4; ++kb) {
        const int k = 4 * kb + L.g;
        const T ar = Are[arow + k], ai = Aim[arow + k];
        const T br = Bre[k * G::LD + bcol], bi = Bim[k * G::LD + bcol];
        acc_re = mfma16(ar, br, acc_re);
        acc_im = mfma16(ar, bi, acc_im);
        acc_re = mfma16(-ai, bi, acc_re);
        acc_im = mfma16(ai, br, acc_im);
    }
    Tile<T> out;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        out.re[r] = acc_re[r];
        out.im[r] = acc_im[r];
    }
    return out;
}

// ||G||_1 of the Hermitian G, taken as its max row sum (equal for Hermitian
// matrices), FP64 sums of entry bounds; same value in every lane.  A row of a
// tile lives in the 16 lanes of one lane group (one register), so row sums
// are DPP rotations; tiles of a row are added through LDS.
template <class G, typename T>
__device__ __forceinline__ double team_norm1(const double* gre, const double* gim, const Lane& L,
                                             double* red) {
    double rs[4];
    if constexpr (G::TW == 1) {
        float fs[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) fs[r] = row16_sum_f(abs_bound_f(gre[r], gim[r]));
        return rows_max_f(fmaxf(fmaxf(fs[0], fs[1]), fmaxf(fs[2], fs[3])));
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) rs[r] = row16_sum(abs_bound(gre[r], gim[r]));
        if (L.j == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) red[L.TJ * G::D + 16 * L.TI + crow<T>(L.g, r)] = rs[r];
        }
        __syncthreads();
        double tot = 0.0;
        if (L.lane < G::D) {
#pragma unroll
            for (int tj = 0; tj < G::TD; ++tj) tot += red[tj * G::D + L.lane];
        }
        __syncthreads();
        return rows_max(row16_max(tot));
    }
}

// exp(-i G) for a (pre-scaled) Hermitian tile set by the degree-m Taylor
// polynomial, split as C(Y) - i G S'(Y).  Uses slots s0, s1.
template <class G, typename T>
__device__ Tile<T> taylor_exp(const Tile<T>& Gt, int m, const Lane& L, double* s0, double* s1) {
    Tile<T> C = ident<T>(L);
    Tile<T> S;
    if (m <= 1) {
        S = Gt;
    } else {
        const int qc = m / 2;        // highest power of Y in C
        const int qs = (m - 1) / 2;  // highest power of Y in S'
        team_sync<G>();
        slot_store<G, T>(s0, Gt, L);
        team_sync<G>();
        Tile<T> P = slot_mul<G, T>(s0, s0, L);   // Y = G G
        Tile<T> Sp = ident<T>(L);
        axpy(C, cos_coef(1), P);
        if (qs >= 1) axpy(Sp, sin_coef(1), P);
        if (qc >= 2) {
            team_sync<G>();
            slot_store<G, T>(s1, P, L);   // Y stays in s1
            team_sync<G>();
            for (int k = 2; k <= qc; ++k) {
                if (k == 2) {
                    P = slot_mul<G, T>(s1, s1, L);
                } else {
                    team_sync<G>();
                    slot_store<G, T>(s0, P, L);
                    team_sync<G>();
                    P = slot_mul<G, T>(s0, s1, L);
                }
                axpy(C, cos_coef(k), P);
                if (k <= qs) axpy(Sp, sin_coef(k), P);
            }
        }
        if (qs >= 1) {
            team_sync<G>();
            slot_store<G, T>(s0, Gt, L);
            slot_store<G, T>(s1, Sp, L);
            team_sync<G>();
            S = slot_mul<G, T>(s0, s1, L);
        } else {
            S = Gt;
        }
    }
    Tile<T> U;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        U.re[r] = C.re[r] + S.im[r];
        U.im[r] = C.im[r] - S.re[r];
    }
    return U;
}

template <class G, typename T>
__device__ __forceinline__ Tile<T> square_n(Tile<T> U, int s, const Lane& L, double* s0) {
    for (int i = 0; i < s; ++i) {
        team_sync<G>();
        slot_store<G, T>(s0, U, L);
        team_sync<G>();
        U = slot_mul<G, T>(s0, s0, L);
    }
    return U;
}

template <class G, typename T>
__device__ __forceinline__ void store_slice(const PropParams& p, int64_t j, const Tile<T>& U,
                                            const Lane& L) {
    T* out = reinterpret_cast<T*>(p.slices_out) + j * (int64_t)p.du * p.du * 2;
    const int col = 16 * L.TJ + L.j;
    if (col >= p.du) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 16 * L.TI + crow<T>(L.g, r);
        if (row < p.du) {
            out[(row * p.du + col) * 2 + 0] = U.re[r];
            out[(row * p.du + col) * 2 + 1] = U.im[r];
        }
    }
}

template <class G>
__device__ __forceinline__ void node_store(double* node, const Tile<double>& t, const Lane& L) {
    const int col = 16 * L.TJ + L.j;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 16 * L.TI + crow<double>(L.g, r);
        node[(row * G::D + col) * 2 + 0] = t.re[r];
        node[(row * G::D + col) * 2 + 1] = t.im[r];
    }
}

template <class G>
__device__ __forceinline__ Tile<double> node_load(const double* node, const Lane& L) {
    Tile<double> t;
    const int col = 16 * L.TJ + L.j;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 16 * L.TI + crow<double>(L.g, r);
        t.re[r] = node[(row * G::D + col) * 2 + 0];
        t.im[r] = node[(row * G::D + col) * 2 + 1];
    }
    return t;
}

}  // namespace
}  // namespace pm
