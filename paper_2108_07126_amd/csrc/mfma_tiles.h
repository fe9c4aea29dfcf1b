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

// Per-wave coordinates.  ks: the staged FP64 products sum over k < 4 ks
// only (set from an embedded dimension whose matrices vanish outside their
// leading block; default all of D).
struct Lane {
    int lane, g, j, TI, TJ, wt;
    int ks = 1 << 30;
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
#pragma unroll 4
    for (int kb = 0; kb < G::D / 4; ++kb) {
        if (kb >= L.ks) break;   // rows k >= 4 L.ks vanish (embedded dimension)
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
#pragma unroll 4
    for (int kb = 0; kb < G::D / 4; ++kb) {
        if (kb >= L.ks) break;   // rows k >= 4 L.ks vanish (embedded dimension)
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

// ---- BF16 split products (the BF16-split mode) ------------------------------
// Every operand entry x is carried as x = hi + lo, hi = bf16(x), lo =
// bf16(x - hi) (round to nearest even), and each real product as
// hi*hi + hi*lo + lo*hi (lo*lo lies below the FP32 rounding of the result's
// scale), accumulated in FP32 on gfx950's 16x16x32 BF16 MFMA.  That
// instruction takes eight BF16 values of A and of B per lane and sums, over
// every lane group and slot, the products of the A and B values in the same
// slot: C[i][j] += sum_{g,s} A(g,s)[i] B(g,s)[j] with i (A) and j (B) the
// lane's index within its group of 16.  The eight slots of a lane may hold
// any pairs whose products belong to the same sum: eight values of k of one
// term, or four values of k of two terms.  The complex product is taken as
// four real products (no operand sums to split).
typedef __bf16 bf4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

struct Split4 {
    bf4_t hi, lo;
};

__device__ __forceinline__ Split4 split4(const float (&x)[4]) {
    Split4 s;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const __bf16 h = (__bf16)x[q];
        s.hi[q] = h;
        s.lo[q] = (__bf16)(x[q] - (float)h);
    }
    return s;
}

__device__ __forceinline__ bf8_t cat8(bf4_t a, bf4_t b) {
    return __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7);
}

__device__ __forceinline__ f4_t mfma_bf16x32(bf8_t a, bf8_t b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Register product of one-wave tiles (FP32 accumulator layout: a lane holds
// k = 4g + r, r = 0..3, of its column), the A-slices given as
// (a_r - i a_i)[r] as in reg_mul: Re = sum a_r Br + a_i Bi,
// Im = sum a_r Bi - a_i Br.  Each x32 MFMA carries two four-k terms (the
// tile's whole K = 16 twice), so a complex product takes six.
__device__ __forceinline__ Tile<float> reg_mul_bf16x(const Split4& ar, const Split4& ai, const Split4& br,
                                                     const Split4& bi) {
    const bf4_t nah = -ai.hi, nal = -ai.lo;
    f4_t re = {0, 0, 0, 0}, im = {0, 0, 0, 0};
    re = mfma_bf16x32(cat8(ar.hi, ar.hi), cat8(br.hi, br.lo), re);
    im = mfma_bf16x32(cat8(ar.hi, ar.hi), cat8(bi.hi, bi.lo), im);
    re = mfma_bf16x32(cat8(ar.lo, ai.hi), cat8(br.hi, bi.hi), re);
    im = mfma_bf16x32(cat8(ar.lo, nah), cat8(bi.hi, br.hi), im);
    re = mfma_bf16x32(cat8(ai.hi, ai.lo), cat8(bi.lo, bi.hi), re);
    im = mfma_bf16x32(cat8(nah, nal), cat8(br.lo, br.hi), im);
    Tile<float> out;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        out.re[r] = re[r];
        out.im[r] = im[r];
    }
    return out;
}

__device__ __forceinline__ Tile<float> reg_mul_bf16s(const float (&ar)[4], const float (&ai)[4],
                                                     const Tile<float>& B) {
    return reg_mul_bf16x(split4(ar), split4(ai), split4(B.re), split4(B.im));
}

// BF16 slots: a D x D complex matrix staged as four bf16 planes (hi and lo of
// the real and of the imaginary part), row stride D + 8 (16-byte aligned
// rows; sixteen lanes reading sixteen rows at one offset hit distinct
// banks).  A slot holds either the rows of X (operand A, or a Hermitian B,
// whose column j is the conjugate of its row j) or the rows of X^T (a
// general operand B).  Each entry is split once, when it is staged.
template <class G>
struct BfSlot {
    static constexpr int LDB = G::D + 8;
    static constexpr int PL = G::D * LDB;   // bf16 per plane
    static_assert(4 * PL * 2 <= G::SLOT * 8, "four bf16 planes fit a slot");
};

template <class G>
__device__ __forceinline__ void slot_store_bf16(double* slot, const Tile<float>& t, const Lane& L, bool trans) {
    using S = BfSlot<G>;
    __bf16* pl = reinterpret_cast<__bf16*>(slot);
    const Split4 sr = split4(t.re), si = split4(t.im);
    const int col = 16 * L.TJ + L.j;
    const int row0 = 16 * L.TI + 4 * L.g;   // rows row0 .. row0 + 3 (FP32 layout)
    if (trans) {
        // rows of X^T: the lane's four rows are four consecutive entries
        const int at = col * S::LDB + row0;
        *reinterpret_cast<bf4_t*>(pl + at) = sr.hi;
        *reinterpret_cast<bf4_t*>(pl + S::PL + at) = sr.lo;
        *reinterpret_cast<bf4_t*>(pl + 2 * S::PL + at) = si.hi;
        *reinterpret_cast<bf4_t*>(pl + 3 * S::PL + at) = si.lo;
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int at = (row0 + r) * S::LDB + col;
            pl[at] = sr.hi[r];
            pl[S::PL + at] = sr.lo[r];
            pl[2 * S::PL + at] = si.hi[r];
            pl[3 * S::PL + at] = si.lo[r];
        }
    }
}

// Tile (TI, TJ) of A B from BF16 slots: A holds the rows of A; B holds the
// rows of B^T, or with bherm the rows of a Hermitian B (B[k][j] =
// conj(B[j][k])).  Four real products, each three split terms, eight k per
// lane and K = 32 per step; the four sums are combined with the signs of
// the complex product at the end.
template <class G>
__device__ __forceinline__ Tile<float> slot_mul_bf16x(const double* A, const double* B, const Lane& L, bool bherm) {
    using S = BfSlot<G>;
    if constexpr (G::D == 16) {
        // K = 16: four k per lane group (k = 4 g + q), two terms per
        // instruction as in reg_mul_bf16x, whose A-slices a_r - i a_i take
        // a_i = -Im A here; a Hermitian B's stored rows give Im B = -(stored)
        const __bf16* pa = reinterpret_cast<const __bf16*>(A) + L.j * S::LDB + 4 * L.g;
        const __bf16* pb = reinterpret_cast<const __bf16*>(B) + L.j * S::LDB + 4 * L.g;
        Split4 ar, ai, br, bi;
        ar.hi = *reinterpret_cast<const bf4_t*>(pa);
        ar.lo = *reinterpret_cast<const bf4_t*>(pa + S::PL);
        ai.hi = -*reinterpret_cast<const bf4_t*>(pa + 2 * S::PL);
        ai.lo = -*reinterpret_cast<const bf4_t*>(pa + 3 * S::PL);
        br.hi = *reinterpret_cast<const bf4_t*>(pb);
        br.lo = *reinterpret_cast<const bf4_t*>(pb + S::PL);
        bi.hi = *reinterpret_cast<const bf4_t*>(pb + 2 * S::PL);
        bi.lo = *reinterpret_cast<const bf4_t*>(pb + 3 * S::PL);
        if (bherm) {
            bi.hi = -bi.hi;
            bi.lo = -bi.lo;
        }
        return reg_mul_bf16x(ar, ai, br, bi);
    }
    const __bf16* pa = reinterpret_cast<const __bf16*>(A) + (16 * L.TI + L.j) * S::LDB + 8 * L.g;
    const __bf16* pb = reinterpret_cast<const __bf16*>(B) + (16 * L.TJ + L.j) * S::LDB + 8 * L.g;
    f4_t rr = {0, 0, 0, 0}, ii = {0, 0, 0, 0}, ri = {0, 0, 0, 0}, ir = {0, 0, 0, 0};
#pragma unroll
    for (int kb = 0; kb < G::D / 32; ++kb) {
        const int o = 32 * kb;
        const bf8_t arh = *reinterpret_cast<const bf8_t*>(pa + o);
        const bf8_t arl = *reinterpret_cast<const bf8_t*>(pa + S::PL + o);
        const bf8_t aih = *reinterpret_cast<const bf8_t*>(pa + 2 * S::PL + o);
        const bf8_t ail = *reinterpret_cast<const bf8_t*>(pa + 3 * S::PL + o);
        const bf8_t brh = *reinterpret_cast<const bf8_t*>(pb + o);
        const bf8_t brl = *reinterpret_cast<const bf8_t*>(pb + S::PL + o);
        const bf8_t bih = *reinterpret_cast<const bf8_t*>(pb + 2 * S::PL + o);
        const bf8_t bil = *reinterpret_cast<const bf8_t*>(pb + 3 * S::PL + o);
        rr = mfma_bf16x32(arh, brh, rr);
        ii = mfma_bf16x32(aih, bih, ii);
        ri = mfma_bf16x32(arh, bih, ri);
        ir = mfma_bf16x32(aih, brh, ir);
        rr = mfma_bf16x32(arh, brl, rr);
        ii = mfma_bf16x32(aih, bil, ii);
        ri = mfma_bf16x32(arh, bil, ri);
        ir = mfma_bf16x32(aih, brl, ir);
        rr = mfma_bf16x32(arl, brh, rr);
        ii = mfma_bf16x32(ail, bih, ii);
        ri = mfma_bf16x32(arl, bih, ri);
        ir = mfma_bf16x32(ail, brh, ir);
    }
    // the stored imaginary part of B is Im B (rows of B^T) or -Im B (rows of
    // a Hermitian B)
    const float sg = bherm ? -1.0f : 1.0f;
    Tile<float> out;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        out.re[r] = rr[r] - sg * ii[r];
        out.im[r] = sg * ri[r] + ir[r];
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
// KS < 4 (FP64 layout only): only the first KS k-slices, rows k < 4 KS --
// the whole product for matrices that vanish outside their leading 4 KS
// rows and columns' block (an embedded dimension of at most 4 KS).
template <typename T, int KS = 4>
__device__ __forceinline__ Tile<T> reg_mul(const T (&ar)[4], const T (&ai)[4], const Tile<T>& B) {
    static_assert(KS == 4 || std::is_same<T, double>::value, "k-slices of rows g + 4r: FP64 layout");
    using V = typename V4<T>::type;
    V t1 = {0, 0, 0, 0}, t2 = {0, 0, 0, 0}, t3 = {0, 0, 0, 0};
#pragma unroll
    for (int r = 0; r < KS; ++r) {
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

// Slice pairs (FP64): one-wave tiles whose two 8 x 8 diagonal blocks hold
// two independent slices are multiplied as the stacked product
// [A_a; A_b] [B_a, B_b] -- K = 8 instead of 16, two k-slices instead of
// four, half the MFMA work of the embedded product.  For k-slice s the lane
// (g, j) supplies its register s (its column in the first block: row
// g + 4s) or s + 2 (second block: row 8 + g + 4s), for the A-slices as for
// the B operand.  The result's diagonal blocks are A_a B_a and A_b B_b in
// place; its off-diagonal blocks hold cross products of the two slices,
// which no later product reads (pair_mask clears them where a full product
// follows).
__device__ __forceinline__ Tile<double> reg_mul_stk(const double (&ar)[4], const double (&ai)[4],
                                                    const Tile<double>& B) {
    const bool hi = (__lane_id() & 8) != 0;
    d4_t t1 = {0, 0, 0, 0}, t2 = {0, 0, 0, 0}, t3 = {0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const double a_r = hi ? ar[q + 2] : ar[q], a_i = hi ? ai[q + 2] : ai[q];
        const double b_r = hi ? B.re[q + 2] : B.re[q], b_i = hi ? B.im[q + 2] : B.im[q];
        t1 = mfma16(a_r, b_r, t1);
        t2 = mfma16(a_i, b_i, t2);
        t3 = mfma16(a_r - a_i, b_r + b_i, t3);
    }
    Tile<double> out;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        out.re[r] = t1[r] + t2[r];
        out.im[r] = t3[r] - t1[r] + t2[r];
    }
    return out;
}

// Zero the off-diagonal 8 x 8 blocks of a slice-pair tile (FP64 layout:
// register r holds row g + 4r, in the second block for r >= 2).
__device__ __forceinline__ void pair_mask(Tile<double>& t, const Lane& L) {
    // unconditional selects: conditional stores into the tile's registers can
    // be merged into a store through a chosen address, which keeps the tile
    // in scratch memory
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const bool cross = (r >= 2) != (L.j >= 8);
        t.re[r] = cross ? 0.0 : t.re[r];
        t.im[r] = cross ? 0.0 : t.im[r];
    }
}

// Register product in the engine's product mode: FP64 and FP32-3M as 3M,
// FP32 as four real products, BF16 split as four split real products; STK:
// the stacked slice-pair product (FP64).
template <typename T, int PMODE, bool STK = false, int KS = 4>
__device__ __forceinline__ Tile<T> reg_mulP(const T (&ar)[4], const T (&ai)[4], const Tile<T>& B) {
    if constexpr (STK) return reg_mul_stk(ar, ai, B);
    else if constexpr (std::is_same<T, double>::value || PMODE == 1) return reg_mul<T, KS>(ar, ai, B);
    else if constexpr (PMODE == 0) return reg_mul4(ar, ai, B);
    else return reg_mul_bf16s(ar, ai, B);
}

// A B for a Hermitian A (the A-slices are conj of the lane's own registers).
template <typename T, int PMODE = 0, bool STK = false, int KS = 4>
__device__ __forceinline__ Tile<T> reg_mul_herm(const Tile<T>& A, const Tile<T>& B) {
    return reg_mulP<T, PMODE, STK, KS>(A.re, A.im, B);
}

// (C - i P) B for Hermitian C and P: the A-slice of C - i P at (j, k) is
// conj(C[k][j]) - i conj(P[k][j]) = (C_re - P_im) - i (C_im + P_re) of the
// lane's own registers.
template <typename T, int PMODE = 0, bool STK = false, int KS = 4>
__device__ __forceinline__ Tile<T> reg_mul_cp(const Tile<T>& C, const Tile<T>& P, const Tile<T>& B) {
    T ar[4], ai[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        ar[r] = C.re[r] - P.im[r];
        ai[r] = C.im[r] + P.re[r];
    }
    return reg_mulP<T, PMODE, STK, KS>(ar, ai, B);
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
template <typename T, int PMODE = 0, bool EXCESS = false, bool STK = false, int KS = 4>
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
    if constexpr (!std::is_same<T, double>::value && PMODE == 2) {
        // BF16 split: a Hermitian tile's split serves as the A-slices and as
        // the B operand alike, so G and Y are split once for every product
        // they enter
        const Split4 gr = split4(Gt.re), gi = split4(Gt.im);
        const Tile<T> Y = reg_mul_bf16x(gr, gi, gr, gi);
        const Split4 yr = split4(Y.re), yi = split4(Y.im);
        Tile<T> Sp = ident<T>(L);
        axpy(C, cos_coef(1), Y);
        if (qs >= 1) axpy(Sp, sin_coef(1), Y);
        Tile<T> Yk = Y;
        for (int k = 2; k <= qc; ++k) {
            Yk = reg_mul_bf16x(yr, yi, split4(Yk.re), split4(Yk.im));
            axpy(C, cos_coef(k), Yk);
            if (k <= qs) axpy(Sp, sin_coef(k), Yk);
        }
        P = qs >= 1 ? reg_mul_bf16x(gr, gi, split4(Sp.re), split4(Sp.im)) : Gt;
    } else {
        const Tile<T> Y = reg_mul_herm<T, PMODE, STK, KS>(Gt, Gt);
        Tile<T> Sp = ident<T>(L);
        axpy(C, cos_coef(1), Y);
        if (qs >= 1) axpy(Sp, sin_coef(1), Y);
        Tile<T> Yk = Y;
        for (int k = 2; k <= qc; ++k) {
            Yk = reg_mul_herm<T, PMODE, STK, KS>(Y, Yk);
            axpy(C, cos_coef(k), Yk);
            if (k <= qs) axpy(Sp, sin_coef(k), Yk);
        }
        P = qs >= 1 ? reg_mul_herm<T, PMODE, STK, KS>(Gt, Sp) : Gt;
    }
}

// Product modes of the FP32 kernels: 0 four real products, 1 3M, 2 BF16
// split (four split real products).  Staging and products of one mode go
// together: stage() writes a slot in the mode's format (BF16 split: split
// once into bf16 planes, the rows of X, or with trans of X^T), mulT()
// multiplies two such slots (BF16 split: B staged as the rows of a
// Hermitian matrix unless bherm is false, then as the rows of B^T).
template <class G, typename T, int PMODE>
__device__ __forceinline__ void stage(double* slot, const Tile<T>& t, const Lane& L, bool trans = false) {
    if constexpr (!std::is_same<T, double>::value && PMODE == 2) slot_store_bf16<G>(slot, t, L, trans);
    else slot_store<G, T>(slot, t, L);
}

template <class G, typename T, int PMODE>
__device__ __forceinline__ Tile<T> mulT(const double* A, const double* B, const Lane& L, bool bherm = true) {
    if constexpr (std::is_same<T, double>::value || PMODE == 0) {
        return slot_mul<G, T>(A, B, L);
    } else if constexpr (PMODE == 1) {
        return slot_mul_3m<G, float>(A, B, L);
    } else {
        return slot_mul_bf16x<G>(A, B, L, bherm);
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
        stage<G, T, PMODE>(s0, Gt, L);
        team_sync<G>();
        Tile<T> P = mulT<G, T, PMODE>(s0, s0, L);   // Y = G G
        Tile<T> Sp = ident<T>(L);
        axpy(C, cos_coef(1), P);
        if (qs >= 1) axpy(Sp, sin_coef(1), P);
        if (qc >= 2) {
            team_sync<G>();
            stage<G, T, PMODE>(s1, P, L);   // Y stays in s1
            team_sync<G>();
            for (int k = 2; k <= qc; ++k) {
                if (k == 2) {
                    P = mulT<G, T, PMODE>(s1, s1, L);
                } else {
                    team_sync<G>();
                    stage<G, T, PMODE>(s0, P, L);
                    team_sync<G>();
                    P = mulT<G, T, PMODE>(s0, s1, L);
                }
                axpy(C, cos_coef(k), P);
                if (k <= qs) axpy(Sp, sin_coef(k), P);
            }
        }
        if (qs >= 1) {
            team_sync<G>();
            stage<G, T, PMODE>(s0, Gt, L);
            stage<G, T, PMODE>(s1, Sp, L);
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
    stage<G, T, PMODE>(s0, E, L);
    stage<G, T, PMODE>(s1, Qt, L, true);     // Q is no Hermitian matrix: B staged as Q^T
    team_sync<G>();
    const Tile<T> P = mulT<G, T, PMODE>(s0, s1, L, false);
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

// exp(-i theta X) for the (pre-scaled) Hermitian tile set X = G / theta,
// spectrum in [-1, 1], by the degree-m Chebyshev series
// J_0(theta) + 2 sum_{k>=1} (-i)^k J_k(theta) T_k(X) (eq. chebychev_series
// with alpha = -theta, beta = theta, so the phase factor is 1), split into
// its even and odd halves and returned in the Hermitian pair form C - i P of
// the Taylor path.  With Y = T_2(X) = 2 X^2 - I, T_2j(X) = T_j(Y) and
// T_{2j+1}(X) = X (2 sum_{i=1..j} (-1)^{j-i} T_i(Y) + (-1)^j I), so
//   C = sum_{i <= m/2} e_i T_i(Y),   P = X sum_{i <= (m-1)/2} b_i T_i(Y),
// e_0 = J_0, e_i = 2 (-1)^i J_2i, and b the alternating suffix sums of the
// odd coefficients (row `ec` of the host's table: e, then b, kChebHalf
// each).  The T_i(Y) follow from T_{i+1} = 2 Y T_i - T_{i-1}; every product
// has the Hermitian left factor X or Y (registers on one-wave teams).
// floor(m/2) + 1 products, where the Clenshaw recurrence in X takes m.  FP64.
template <class G>
__device__ void cheb_parts(const Tile<double>& Gt, int m, double theta, const double* ec, const Lane& L,
                           double* s0, double* s1, Tile<double>& C, Tile<double>& P) {
    const double inv = 1.0 / theta;
    const double* eb = ec + kChebHalf;
    const int qc = m / 2, qs = (m - 1) / 2;   // m >= 1
    Tile<double> X, Sp;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const bool diag = 16 * L.TI + crow<double>(L.g, r) == 16 * L.TJ + L.j;
        X.re[r] = Gt.re[r] * inv;
        X.im[r] = Gt.im[r] * inv;
        C.re[r] = diag ? ec[0] : 0.0;
        Sp.re[r] = diag ? eb[0] : 0.0;
        C.im[r] = Sp.im[r] = 0.0;
    }
    if (qc >= 1) {
        Tile<double> Y = herm_mul<G>(X, X, L, s0, s1);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const bool diag = 16 * L.TI + crow<double>(L.g, r) == 16 * L.TJ + L.j;
            Y.re[r] = fma(2.0, Y.re[r], diag ? -1.0 : 0.0);
            Y.im[r] *= 2.0;
        }
        axpy(C, ec[1], Y);
        if (qs >= 1) axpy(Sp, eb[1], Y);
        if constexpr (G::TW > 1) {
            // multi-wave teams: Y, the same left factor of every step, is
            // staged once and read from its slot; the recurrence then holds
            // two terms of T and no copy of Y in registers
            team_sync<G>();
            slot_store<G, double>(s0, Y, L);
        }
        Tile<double> Tm = ident<double>(L), Tc = Y;
        for (int i = 2; i <= qc; ++i) {
            Tile<double> Tn;
            if constexpr (G::TW > 1) {
                team_sync<G>();
                slot_store<G, double>(s1, Tc, L);
                team_sync<G>();
                Tn = slot_mul<G, double>(s0, s1, L);
            } else {
                Tn = herm_mul<G>(Y, Tc, L, s0, s1);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                Tn.re[r] = fma(2.0, Tn.re[r], -Tm.re[r]);
                Tn.im[r] = fma(2.0, Tn.im[r], -Tm.im[r]);
            }
            axpy(C, ec[i], Tn);
            if (i <= qs) axpy(Sp, eb[i], Tn);
            Tm = Tc;
            Tc = Tn;
        }
    }
    if (qs >= 1) {
        P = herm_mul<G>(X, Sp, L, s0, s1);
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            P.re[r] = eb[0] * X.re[r];
            P.im[r] = eb[0] * X.im[r];
        }
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
