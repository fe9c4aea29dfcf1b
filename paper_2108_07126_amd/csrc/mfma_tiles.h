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
    // Several multi-wave teams in one block synchronise block-wide, so they
    // must run the same control flow (the batched engine's lockstep packets).
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

// The identity in the register layout of T-kernels, held as FP64 values
// (the reduced-precision kernels keep their chain products this way).
template <typename T>
__device__ __forceinline__ Tile<double> ident_as(const Lane& L) {
    Tile<double> t;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        t.re[r] = (16 * L.TI + crow<T>(L.g, r) == 16 * L.TJ + L.j) ? 1.0 : 0.0;
        t.im[r] = 0.0;
    }
    return t;
}

template <typename T>
__device__ __forceinline__ Tile<T> plus_ident(const Tile<T>& e, const Lane& L) {
    Tile<T> t = e;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (16 * L.TI + crow<T>(L.g, r) == 16 * L.TJ + L.j) t.re[r] += T(1);
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

// FP64 values moved from the row layout of LSrc-kernels to that of
// LDst-kernels (through an LDS slot).
template <class G, typename LSrc, typename LDst>
__device__ __forceinline__ Tile<double> relayout_rows(const Tile<double>& t, double* slot, const Lane& L) {
    if constexpr (std::is_same<LSrc, LDst>::value) {
        return t;
    } else {
        double* re = slot;
        double* im = slot + G::PLANE;
        const int col = 16 * L.TJ + L.j;
        team_sync<G>();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * L.TI + crow<LSrc>(L.g, r);
            re[row * G::LD + col] = t.re[r];
            im[row * G::LD + col] = t.im[r];
        }
        team_sync<G>();
        Tile<double> o;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * L.TI + crow<LDst>(L.g, r);
            o.re[r] = re[row * G::LD + col];
            o.im[r] = im[row * G::LD + col];
        }
        return o;
    }
}

// Tile (TI, TJ) of A * B, A and B complex D x D in LDS slots: four real
// products (the FP32 mode's complex product).
template <class G, typename T>
__device__ __forceinline__ Tile<T> slot_mul4(const double* A, const double* B, const Lane& L) {
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

// Complex product as three real products (3M): T1 = Ar Br, T2 = Ai Bi,
// T3 = (Ar + Ai)(Br + Bi); Re = T1 - T2, Im = T3 - T1 - T2.  FP64 products
// always take this form (three MFMA chains instead of four; the imaginary
// part's rounding bound doubles, which FP64 absorbs), FP32 ones in the 3M
// mode.
template <class G, typename T>
__device__ __forceinline__ Tile<T> slot_mul_3m(const double* A, const double* B, const Lane& L) {
    using V = typename V4<T>::type;
    const T* Are = reinterpret_cast<const T*>(A);
    const T* Aim = Are + G::PLANE;
    const T* Bre = reinterpret_cast<const T*>(B);
    const T* Bim = Bre + G::PLANE;
    V t1 = {0, 0, 0, 0}, t2 = {0, 0, 0, 0}, t3 = {0, 0, 0, 0};
    const int arow = (16 * L.TI + L.j) * G::LD;
    const int bcol = 16 * L.TJ + L.j;
#pragma unroll
    for (int kb = 0; kb < G::D / 4; ++kb) {
        const int k = 4 * kb + L.g;
        const T ar = Are[arow + k], ai = Aim[arow + k];
        const T br = Bre[k * G::LD + bcol], bi = Bim[k * G::LD + bcol];
        t1 = mfma16(ar, br, t1);
        t2 = mfma16(ai, bi, t2);
        t3 = mfma16(ar + ai, br + bi, t3);
    }
    Tile<T> out;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        out.re[r] = t1[r] - t2[r];
        out.im[r] = t3[r] - t1[r] - t2[r];
    }
    return out;
}

// The engines' complex product: 3M in FP64, four real products in FP32.
template <class G, typename T>
__device__ __forceinline__ Tile<T> slot_mul(const double* A, const double* B, const Lane& L) {
    if constexpr (std::is_same<T, double>::value) return slot_mul_3m<G, double>(A, B, L);
    else return slot_mul4<G, T>(A, B, L);
}

typedef short s4_t __attribute__((ext_vector_type(4)));

// x = hi + lo with hi = bf16(x), lo = bf16(x - hi) (round to nearest even).
__device__ __forceinline__ void split_bf16x4(const float* x, s4_t& hi, s4_t& lo) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const __bf16 h = (__bf16)x[q];
        const __bf16 l = (__bf16)(x[q] - (float)h);
        hi[q] = (short)__builtin_bit_cast(unsigned short, h);
        lo[q] = (short)__builtin_bit_cast(unsigned short, l);
    }
}

__device__ __forceinline__ f4_t mfma_bf16(s4_t a, s4_t b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// 3M complex product on BF16 hi/lo split operands with FP32 accumulation:
// each real product a b is taken as a_hi b_hi + a_hi b_lo + a_lo b_hi (the
// a_lo b_lo term is below FP32 rounding of the result's scale).  The 16x16x16
// BF16 MFMA takes four consecutive k per lane group: A[i][16 kb + 4 g + q],
// B[16 kb + 4 g + q][j].
template <class G>
__device__ __forceinline__ Tile<float> slot_mul_bf16s(const double* A, const double* B, const Lane& L) {
    const float* Are = reinterpret_cast<const float*>(A);
    const float* Aim = Are + G::PLANE;
    const float* Bre = reinterpret_cast<const float*>(B);
    const float* Bim = Bre + G::PLANE;
    f4_t t1 = {0, 0, 0, 0}, t2 = {0, 0, 0, 0}, t3 = {0, 0, 0, 0};
    const int arow = (16 * L.TI + L.j) * G::LD;
    const int bcol = 16 * L.TJ + L.j;
#pragma unroll
    for (int kb = 0; kb < G::D / 16; ++kb) {
        float ar[4], ai[4], as[4], br[4], bi[4], bs[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = 16 * kb + 4 * L.g + q;
            ar[q] = Are[arow + k];
            ai[q] = Aim[arow + k];
            br[q] = Bre[k * G::LD + bcol];
            bi[q] = Bim[k * G::LD + bcol];
            as[q] = ar[q] + ai[q];
            bs[q] = br[q] + bi[q];
        }
        s4_t arh, arl, aih, ail, ash, asl, brh, brl, bih, bil, bsh, bsl;
        split_bf16x4(ar, arh, arl);
        split_bf16x4(ai, aih, ail);
        split_bf16x4(as, ash, asl);
        split_bf16x4(br, brh, brl);
        split_bf16x4(bi, bih, bil);
        split_bf16x4(bs, bsh, bsl);
        t1 = mfma_bf16(arh, brh, t1);
        t2 = mfma_bf16(aih, bih, t2);
        t3 = mfma_bf16(ash, bsh, t3);
        t1 = mfma_bf16(arh, brl, t1);
        t2 = mfma_bf16(aih, bil, t2);
        t3 = mfma_bf16(ash, bsl, t3);
        t1 = mfma_bf16(arl, brh, t1);
        t2 = mfma_bf16(ail, bih, t2);
        t3 = mfma_bf16(asl, bsh, t3);
    }
    Tile<float> out;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        out.re[r] = t1[r] - t2[r];
        out.im[r] = t3[r] - t1[r] - t2[r];
    }
    return out;
}

// Complex products of one-wave tiles without leaving the lane.  In the
// accumulator layout of the 16x16x4 MFMA a lane holds four rows of its
// column (rows g + 4r in FP64, 4g + r in FP32, lane 16 g + j, column j), so
// register r of B is B's k-slice r as the next MFMA wants it (k running
// over the four rows that register r holds across the lane groups).  The
// A-slice needs A[j][k] for those k, i.e. the transpose of what the lane
// holds; for a Hermitian A that is conj(A[k][j]), register r of the lane
// itself.  reg_mul takes the A-slices as (a_r - i a_i)[r]:
//     sum_r (a_r - i a_i)[r] B[r]
// by 3M: t1 = a_r Br, t2 = a_i Bi, t3 = (a_r - a_i)(Br + Bi);
// Re = t1 + t2, Im = t3 - t1 + t2.
template <typename T>
__device__ __forceinline__ Tile<T> reg_mul(const T (&ar)[4], const T (&ai)[4], const Tile<T>& B) {
    using V = typename V4<T>::type;
    V t1 = {0, 0, 0, 0}, t2 = {0, 0, 0, 0}, t3 = {0, 0, 0, 0};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        t1 = mfma16(ar[r], B.re[r], t1);
        t2 = mfma16(ai[r], B.im[r], t2);
        t3 = mfma16(ar[r] - ai[r], B.re[r] + B.im[r], t3);
    }
    Tile<T> out;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        out.re[r] = t1[r] + t2[r];
        out.im[r] = t3[r] - t1[r] + t2[r];
    }
    return out;
}

// The same product as four real products (the FP32 mode): with a = a_r - i a_i,
// Re = sum a_r Br + a_i Bi and Im = sum a_r Bi - a_i Br in two chains.
__device__ __forceinline__ Tile<float> reg_mul4(const float (&ar)[4], const float (&ai)[4], const Tile<float>& B) {
    f4_t acc_re = {0, 0, 0, 0}, acc_im = {0, 0, 0, 0};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        acc_re = mfma16(ar[r], B.re[r], acc_re);
        acc_im = mfma16(ar[r], B.im[r], acc_im);
        acc_re = mfma16(ai[r], B.im[r], acc_re);
        acc_im = mfma16(-ai[r], B.re[r], acc_im);
    }
    Tile<float> out;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        out.re[r] = acc_re[r];
        out.im[r] = acc_im[r];
    }
    return out;
}

// The same product as 3M on BF16 hi/lo split operands (the BF16-split
// mode): the 16x16x16 BF16 MFMA takes four consecutive k per lane group,
// A[j][4 g + q] and B[4 g + q][j], which for one 16-wide tile are again the
// lane's own four registers (rows 4 g + q of the FP32 accumulator layout).
__device__ __forceinline__ Tile<float> reg_mul_bf16s(const float (&ar)[4], const float (&ai)[4],
                                                     const Tile<float>& B) {
    float as[4], bs[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        as[q] = ar[q] - ai[q];
        bs[q] = B.re[q] + B.im[q];
    }
    s4_t arh, arl, aih, ail, ash, asl, brh, brl, bih, bil, bsh, bsl;
    split_bf16x4(ar, arh, arl);
    split_bf16x4(ai, aih, ail);
    split_bf16x4(as, ash, asl);
    split_bf16x4(B.re, brh, brl);
    split_bf16x4(B.im, bih, bil);
    split_bf16x4(bs, bsh, bsl);
    f4_t t1 = {0, 0, 0, 0}, t2 = {0, 0, 0, 0}, t3 = {0, 0, 0, 0};
    t1 = mfma_bf16(arh, brh, t1);
    t2 = mfma_bf16(aih, bih, t2);
    t3 = mfma_bf16(ash, bsh, t3);
    t1 = mfma_bf16(arh, brl, t1);
    t2 = mfma_bf16(aih, bil, t2);
    t3 = mfma_bf16(ash, bsl, t3);
    t1 = mfma_bf16(arl, brh, t1);
    t2 = mfma_bf16(ail, bih, t2);
    t3 = mfma_bf16(asl, bsh, t3);
    Tile<float> out;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        out.re[r] = t1[r] + t2[r];
        out.im[r] = t3[r] - t1[r] + t2[r];
    }
    return out;
}

// Register product in the engine's product mode: FP64 and FP32-3M as 3M,
// FP32 as four real products, BF16 split as split 3M.
template <typename T, int PMODE>
__device__ __forceinline__ Tile<T> reg_mulP(const T (&ar)[4], const T (&ai)[4], const Tile<T>& B) {
    if constexpr (std::is_same<T, double>::value || PMODE == 1) return reg_mul<T>(ar, ai, B);
    else if constexpr (PMODE == 0) return reg_mul4(ar, ai, B);
    else return reg_mul_bf16s(ar, ai, B);
}

// A B for a Hermitian A (the A-slices are conj of the lane's own registers).
template <typename T, int PMODE = 0>
__device__ __forceinline__ Tile<T> reg_mul_herm(const Tile<T>& A, const Tile<T>& B) {
    return reg_mulP<T, PMODE>(A.re, A.im, B);
}

// (C - i P) B for Hermitian C and P: the A-slice of C - i P at (j, k) is
// conj(C[k][j]) - i conj(P[k][j]) = (C_re - P_im) - i (C_im + P_re) of the
// lane's own registers.
template <typename T, int PMODE = 0>
__device__ __forceinline__ Tile<T> reg_mul_cp(const Tile<T>& C, const Tile<T>& P, const Tile<T>& B) {
    T ar[4], ai[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        ar[r] = C.re[r] - P.im[r];
        ai[r] = C.im[r] + P.re[r];
    }
    return reg_mulP<T, PMODE>(ar, ai, B);
}

// C - i P as one tile.
template <typename T>
__device__ __forceinline__ Tile<T> combine_cp(const Tile<T>& C, const Tile<T>& P) {
    Tile<T> U;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        U.re[r] = C.re[r] + P.im[r];
        U.im[r] = C.im[r] - P.re[r];
    }
    return U;
}

// The degree-m Taylor polynomial of exp(-i G) for a (pre-scaled) Hermitian
// one-wave tile, returned as the Hermitian pair exp(-i G) = C - i P with
// C = C(Y) and P = G S'(Y), Y = G^2 (the cos / sin split of taylor_exp):
// every product has a Hermitian left factor, so all of them stay in
// registers.  With EXCESS the identity term of C is left out (C - i P is
// then exp(-i G) - I, accurate relative to ||G||).
template <typename T, int PMODE = 0, bool EXCESS = false>
__device__ __forceinline__ void taylor_parts_reg(const Tile<T>& Gt, int m, const Lane& L, Tile<T>& C, Tile<T>& P) {
    if constexpr (EXCESS) {
#pragma unroll
        for (int r = 0; r < 4; ++r) C.re[r] = C.im[r] = T(0);
    } else {
        C = ident<T>(L);
    }
    if (m <= 1) {
        P = Gt;
        return;
    }
    const int qc = m / 2;        // highest power of Y in C
    const int qs = (m - 1) / 2;  // highest power of Y in S'
    const Tile<T> Y = reg_mul_herm<T, PMODE>(Gt, Gt);
    Tile<T> Sp = ident<T>(L);
    axpy(C, cos_coef(1), Y);
    if (qs >= 1) axpy(Sp, sin_coef(1), Y);
    Tile<T> Yk = Y;
    for (int k = 2; k <= qc; ++k) {
        Yk = reg_mul_herm<T, PMODE>(Y, Yk);
        axpy(C, cos_coef(k), Yk);
        if (k <= qs) axpy(Sp, sin_coef(k), Yk);
    }
    P = qs >= 1 ? reg_mul_herm<T, PMODE>(Gt, Sp) : Gt;
}

// Product modes of the FP32 kernels: 0 four real products, 1 3M, 2 BF16-split 3M.
template <class G, typename T, int PMODE>
__device__ __forceinline__ Tile<T> mulT(const double* A, const double* B, const Lane& L) {
    if constexpr (std::is_same<T, double>::value || PMODE == 0) {
        return slot_mul<G, T>(A, B, L);
    } else if constexpr (PMODE == 1) {
        return slot_mul_3m<G, float>(A, B, L);
    } else {
        return slot_mul_bf16s<G>(A, B, L);
    }
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
// polynomial, split as C(Y) - i G S'(Y).  With EXCESS the identity term is
// left out (the result is exp(-i G) - I, accurate relative to ||G||).  Uses
// slots s0, s1.
template <class G, typename T, int PMODE = 0, bool EXCESS = false>
__device__ Tile<T> taylor_exp(const Tile<T>& Gt, int m, const Lane& L, double* s0, double* s1) {
    Tile<T> C;
    if constexpr (EXCESS) {
#pragma unroll
        for (int r = 0; r < 4; ++r) C.re[r] = C.im[r] = T(0);
    } else {
        C = ident<T>(L);
    }
    Tile<T> S;
    if (m <= 1) {
        S = Gt;
    } else {
        const int qc = m / 2;        // highest power of Y in C
        const int qs = (m - 1) / 2;  // highest power of Y in S'
        team_sync<G>();
        slot_store<G, T>(s0, Gt, L);
        team_sync<G>();
        Tile<T> P = mulT<G, T, PMODE>(s0, s0, L);   // Y = G G
        Tile<T> Sp = ident<T>(L);
        axpy(C, cos_coef(1), P);
        if (qs >= 1) axpy(Sp, sin_coef(1), P);
        if (qc >= 2) {
            team_sync<G>();
            slot_store<G, T>(s1, P, L);   // Y stays in s1
            team_sync<G>();
            for (int k = 2; k <= qc; ++k) {
                if (k == 2) {
                    P = mulT<G, T, PMODE>(s1, s1, L);
                } else {
                    team_sync<G>();
                    slot_store<G, T>(s0, P, L);
                    team_sync<G>();
                    P = mulT<G, T, PMODE>(s0, s1, L);
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
            S = mulT<G, T, PMODE>(s0, s1, L);
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

// exp(-i G) for a (pre-scaled) Hermitian tile set by the degree-m Chebyshev
// series on the interval [-theta, theta] that holds its spectrum
// (eq. chebychev_series with alpha = -theta, beta = theta, so the phase
// factor is 1): X = G / theta, a_k = (-i)^k J_k(theta) (row `jk` of the
// coefficient table), and the Clenshaw recurrence of Algorithm 1,
// D_k = a_k I + 2 X D_{k+1} - D_{k+2}, result D_0 - D_2.  m products.  FP64.
template <class G>
__device__ Tile<double> cheb_exp(const Tile<double>& Gt, int m, double theta, const double* jk, const Lane& L,
                                 double* s0, double* s1) {
    const double inv = 1.0 / theta;
    Tile<double> X, D1, D2, keep;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        X.re[r] = Gt.re[r] * inv;
        X.im[r] = Gt.im[r] * inv;
        D1.re[r] = D1.im[r] = D2.re[r] = D2.im[r] = keep.re[r] = keep.im[r] = 0.0;
    }
    if constexpr (G::TW != 1) {
        team_sync<G>();
        slot_store<G, double>(s0, X, L);   // X stays in s0
    }
    for (int k = m; k >= 0; --k) {
        Tile<double> P;
        if (k < m) {
            if constexpr (G::TW == 1) {
                // one-wave team: X is Hermitian, so X D1 comes from registers
                P = reg_mul_herm<double>(X, D1);
            } else {
                team_sync<G>();
                slot_store<G, double>(s1, D1, L);
                team_sync<G>();
                P = slot_mul<G, double>(s0, s1, L);
            }
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) P.re[r] = P.im[r] = 0.0;
        }
        // a_k = (-i)^k J_k: real for even k (sign + - + -), imaginary for odd
        const double jv = jk[k];
        const int q = k & 3;
        const double are = q == 0 ? jv : (q == 2 ? -jv : 0.0);
        const double aim = q == 1 ? -jv : (q == 3 ? jv : 0.0);
        Tile<double> Dk;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const bool diag = 16 * L.TI + crow<double>(L.g, r) == 16 * L.TJ + L.j;
            Dk.re[r] = fma(2.0, P.re[r], -D2.re[r]) + (diag ? are : 0.0);
            Dk.im[r] = fma(2.0, P.im[r], -D2.im[r]) + (diag ? aim : 0.0);
        }
        if (k == 0) keep = D2;
        D2 = D1;
        D1 = Dk;
    }
    Tile<double> U;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        U.re[r] = D1.re[r] - keep.re[r];
        U.im[r] = D1.im[r] - keep.im[r];
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

// E <- (I + E)^2 - I = 2E + E E, s times (FP64).
template <class G>
__device__ __forceinline__ Tile<double> square_excess_n(Tile<double> E, int s, const Lane& L, double* s0) {
    for (int i = 0; i < s; ++i) {
        team_sync<G>();
        slot_store<G, double>(s0, E, L);
        team_sync<G>();
        const Tile<double> P = slot_mul<G, double>(s0, s0, L);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            E.re[r] = fma(2.0, E.re[r], P.re[r]);
            E.im[r] = fma(2.0, E.im[r], P.im[r]);
        }
    }
    return E;
}

// Chain step of the reduced-precision kernels: Q <- (I + E) Q = Q + E Q,
// the product E Q in the working precision T (MFMA, product mode PMODE) and
// the accumulation in FP64 (Q: FP64 values in the T register layout).
template <class G, typename T, int PMODE>
__device__ __forceinline__ void chain_acc(Tile<double>& Q, const Tile<T>& E, const Lane& L, double* s0,
                                          double* s1) {
    Tile<T> Qt;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        Qt.re[r] = (T)Q.re[r];
        Qt.im[r] = (T)Q.im[r];
    }
    team_sync<G>();
    slot_store<G, T>(s0, E, L);
    slot_store<G, T>(s1, Qt, L);
    team_sync<G>();
    const Tile<T> P = mulT<G, T, PMODE>(s0, s1, L);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        Q.re[r] += (double)P.re[r];
        Q.im[r] += (double)P.im[r];
    }
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

// Per-slice output of a slice pair (one-wave 16-wide tile, d <= 8): the
// upper-left block holds slice ja, the lower-right one slice jb (none when
// jb < 0).
template <class G, typename T>
__device__ __forceinline__ void store_slice_pair(const PropParams& p, int64_t ja, int64_t jb, const Tile<T>& U,
                                                 const Lane& L) {
    const int du = p.du;
    const bool second = L.j >= 8;
    const int64_t js = second ? jb : ja;
    const int col = second ? L.j - 8 : L.j;
    if (js < 0 || col >= du) return;
    T* out = reinterpret_cast<T*>(p.slices_out) + js * (int64_t)du * du * 2;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = crow<T>(L.g, r);
        const int rb = second ? row - 8 : row;
        if ((second ? row >= 8 : row < 8) && rb < du) {
            out[(rb * du + col) * 2 + 0] = U.re[r];
            out[(rb * du + col) * 2 + 1] = U.im[r];
        }
    }
}

// The chain product of a slice-pair team: from Q = Q_A (+) Q_B (the two
// halves' products in the diagonal blocks), Q_B Q_A in the upper-left block
// with the identity elsewhere, the layout of an unpaired chain product.
template <class G>
__device__ __forceinline__ Tile<double> pair_product(const Tile<double>& Q, const Lane& L, double* s0, double* s1) {
    static_assert(G::D == 16 && G::TW == 1, "slice pairs live in one-wave 16-wide tiles");
    team_sync<G>();
    slot_store<G, double>(s0, Q, L);
    team_sync<G>();
    const double* re = s0;
    const double* im = s0 + G::PLANE;
    Tile<double> X, Y;
    const int col = L.j;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = crow<double>(L.g, r);
        const bool in = row < 8 && col < 8;
        const double id = row == col ? 1.0 : 0.0;
        X.re[r] = in ? re[(row + 8) * G::LD + col + 8] : id;
        X.im[r] = in ? im[(row + 8) * G::LD + col + 8] : 0.0;
        Y.re[r] = in ? re[row * G::LD + col] : id;
        Y.im[r] = in ? im[row * G::LD + col] : 0.0;
    }
    team_sync<G>();
    slot_store<G, double>(s0, X, L);
    slot_store<G, double>(s1, Y, L);
    team_sync<G>();
    return slot_mul<G, double>(s0, s1, L);
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

// Z - Z^H for a tile set Z (FP64): the adjoint is read back transposed from
// an LDS slot.  For Hermitian X and Y, (XY)^H = YX, so the commutator
// [X, Y] is XY - (XY)^H: one product instead of two.
template <class G>
__device__ __forceinline__ Tile<double> minus_adjoint(const Tile<double>& Z, const Lane& L, double* slot) {
    team_sync<G>();
    slot_store<G, double>(slot, Z, L);
    team_sync<G>();
    const double* re = slot;
    const double* im = slot + G::PLANE;
    const int col = 16 * L.TJ + L.j;
    Tile<double> o;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 16 * L.TI + crow<double>(L.g, r);
        o.re[r] = Z.re[r] - re[col * G::LD + row];
        o.im[r] = Z.im[r] + im[col * G::LD + row];
    }
    return o;
}

// X Y for a Hermitian X (FP64): from registers on one-wave teams, staged
// through slots s0, s1 otherwise.
template <class G>
__device__ __forceinline__ Tile<double> herm_mul(const Tile<double>& X, const Tile<double>& Y, const Lane& L,
                                                 double* s0, double* s1) {
    if constexpr (G::TW == 1) {
        return reg_mul_herm<double>(X, Y);
    } else {
        team_sync<G>();
        slot_store<G, double>(s0, X, L);
        slot_store<G, double>(s1, Y, L);
        team_sync<G>();
        return slot_mul<G, double>(s0, s1, L);
    }
}

// The sixth-order Magnus exponent of a slice (three-node scheme of Blanes,
// Casas and Ros) from its Hermitian moments P1, P2, P3 (the weights of
// m6_weight).  With a_q = -i P_q, the scheme's
//   C1 = [a1, a2],  C2 = -(1/60) [a1, 2 a3 + C1],
//   Omega = a1 + a3 / 12 + (1/240) [-20 a1 - a3 + C1, a2 + C2]
// reads, on Hermitian R1 = i C1 and R2 = i C2 and G = i Omega,
//   R1 = -i [P1, P2],  R2 = (i/60) [P1, 2 P3 + R1],
//   G = P1 + P3 / 12 - (i/240) [-20 P1 - P3 + R1, P2 + R2],
// three commutators of Hermitian matrices, each one product and an adjoint.
// Uses slots s0, s1.
template <class G>
__device__ Tile<double> magnus6_exponent(const Tile<double>& P1, const Tile<double>& P2, const Tile<double>& P3,
                                         const Lane& L, double* s0, double* s1) {
    Tile<double> K = minus_adjoint<G>(herm_mul<G>(P1, P2, L, s0, s1), L, s0);
    Tile<double> R1, W;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        R1.re[r] = K.im[r];
        R1.im[r] = -K.re[r];
        W.re[r] = 2.0 * P3.re[r] + R1.re[r];
        W.im[r] = 2.0 * P3.im[r] + R1.im[r];
    }
    K = minus_adjoint<G>(herm_mul<G>(P1, W, L, s0, s1), L, s0);
    Tile<double> X, Y;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        X.re[r] = (-20.0 * P1.re[r] - P3.re[r]) + R1.re[r];
        X.im[r] = (-20.0 * P1.im[r] - P3.im[r]) + R1.im[r];
        Y.re[r] = P2.re[r] - K.im[r] * (1.0 / 60.0);
        Y.im[r] = P2.im[r] + K.re[r] * (1.0 / 60.0);
    }
    K = minus_adjoint<G>(herm_mul<G>(X, Y, L, s0, s1), L, s0);
    Tile<double> Gt;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        Gt.re[r] = (P1.re[r] + P3.re[r] * (1.0 / 12.0)) + K.im[r] * (1.0 / 240.0);
        Gt.im[r] = (P1.im[r] + P3.im[r] * (1.0 / 12.0)) - K.re[r] * (1.0 / 240.0);
    }
    return Gt;
}

}  // namespace
}  // namespace pm
