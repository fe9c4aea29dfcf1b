// Adjoint gradient of a real loss L(U(T)) with respect to every control
// sample, on the MFMA tile engine in FP64.
//
// With W the loss gradient in the convention dL = Re Tr(W^H dU(T)),
// P_j = U_{j-1} ... U_0 and S_j = U_{N-1} ... U_{j+1}:
//     dL = Re sum_j Tr(W^H S_j dU_j P_j) = Re sum_j Tr(F_j dG_j),
//     F_j = L_f(G_j, Lambda_j),  Lambda_j = P_j W^H S_j,  f(G) = exp(-i G),
// (cyclic trace and Tr(A L_f(G, E)) = Tr(L_f(G, A) E)), so that
//     dL / dw_{j,m} = Re Tr(F_j B_m)
// for the expand step's weights; the chain rule through the weight formulas
// gives dL / d samples.  The prefix/suffix structure is carried by
//     Omega_j = P_j W^H (U_{N-1} ... U_j),  Lambda_j = Omega_j U_j^H,
//     Omega_{j+1} = U_j Omega_j U_j^H,
// started at each chain from its checkpoint P_{j0}: the forward pass (run
// just before, with every tree node kept) leaves the product of every aligned
// power-of-two range of blocks, and P_{j0} is assembled from at most
// log2(#blocks) of them plus the earlier chains of its own block; then
// Omega_{j0} = P Z P^H with Z = W^H U(T) (P unitary).  Inside a chain the
// slices are recomputed (a checkpoint every `chunk` slices, nothing else
// stored).  F_j is the upper-right block of exp(-i [[G, Lambda], [0, G]]),
// evaluated with the same cos/sin Taylor scheme and scaling-and-squaring as
// the forward pass on (value, derivative) pairs:
//     (A, dA)(B, dB) = (A B, A dB + dA B).
#include "mfma_tiles.h"

namespace pm {
namespace {

template <class G>
__device__ __forceinline__ Tile<double> load_user(const double* A, int du, double pad_diag,
                                                  const Lane& L) {
    Tile<double> t;
    const int col = 16 * L.TJ + L.j;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 16 * L.TI + crow<double>(L.g, r);
        if (row < du && col < du) {
            t.re[r] = A[(row * du + col) * 2 + 0];
            t.im[r] = A[(row * du + col) * 2 + 1];
        } else {
            t.re[r] = (row == col) ? pad_diag : 0.0;
            t.im[r] = 0.0;
        }
    }
    return t;
}

// The conjugate transpose of a tile set, stored into a slot.
template <class G>
__device__ __forceinline__ void slot_store_adj(double* slot, const Tile<double>& t, const Lane& L) {
    double* re = slot;
    double* im = slot + G::PLANE;
    const int col = 16 * L.TJ + L.j;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 16 * L.TI + crow<double>(L.g, r);
        re[col * G::LD + row] = t.re[r];
        im[col * G::LD + row] = -t.im[r];
    }
}

__device__ __forceinline__ Tile<double> tadd(const Tile<double>& a, const Tile<double>& b) {
    Tile<double> c;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        c.re[r] = a.re[r] + b.re[r];
        c.im[r] = a.im[r] + b.im[r];
    }
    return c;
}

__device__ __forceinline__ Tile<double> tzero() {
    Tile<double> c;
#pragma unroll
    for (int r = 0; r < 4; ++r) c.re[r] = c.im[r] = 0.0;
    return c;
}

__device__ __forceinline__ Tile<double> tscale(const Tile<double>& a, int e) {
    Tile<double> c;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        c.re[r] = ldexp(a.re[r], e);
        c.im[r] = ldexp(a.im[r], e);
    }
    return c;
}

// C - i S
__device__ __forceinline__ Tile<double> c_minus_is(const Tile<double>& C, const Tile<double>& S) {
    Tile<double> u;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        u.re[r] = C.re[r] + S.im[r];
        u.im[r] = C.im[r] - S.re[r];
    }
    return u;
}

template <class G>
__device__ __forceinline__ Tile<double> mul2(const Tile<double>& A, const Tile<double>& B,
                                             const Lane& L, double* s0, double* s1) {
    team_sync<G>();
    slot_store<G, double>(s0, A, L);
    slot_store<G, double>(s1, B, L);
    team_sync<G>();
    return slot_mul<G, double>(s0, s1, L);
}

// A B^H
template <class G>
__device__ __forceinline__ Tile<double> mul_adjB(const Tile<double>& A, const Tile<double>& B,
                                                 const Lane& L, double* s0, double* s1) {
    team_sync<G>();
    slot_store<G, double>(s0, A, L);
    slot_store_adj<G>(s1, B, L);
    team_sync<G>();
    return slot_mul<G, double>(s0, s1, L);
}

// A^H B
template <class G>
__device__ __forceinline__ Tile<double> mul_adjA(const Tile<double>& A, const Tile<double>& B,
                                                 const Lane& L, double* s0, double* s1) {
    team_sync<G>();
    slot_store_adj<G>(s0, A, L);
    slot_store<G, double>(s1, B, L);
    team_sync<G>();
    return slot_mul<G, double>(s0, s1, L);
}

// (exp(-i G), L_f(G, E)) by the degree-m cos/sin Taylor scheme on
// (value, derivative) pairs; G and E pre-scaled by 2^-s.
template <class G>
__device__ void pair_taylor(const Tile<double>& Gt, const Tile<double>& Et, int m, const Lane& L,
                            double* s0, double* s1, Tile<double>& U, Tile<double>& dU) {
    Tile<double> C = ident<double>(L), dC = tzero(), S, dS;
    if (m <= 1) {
        S = Gt;
        dS = Et;
    } else {
        const int qc = m / 2, qs = (m - 1) / 2;
        team_sync<G>();
        slot_store<G, double>(s0, Gt, L);
        slot_store<G, double>(s1, Et, L);
        team_sync<G>();
        const Tile<double> Y = slot_mul<G, double>(s0, s0, L);
        const Tile<double> dY = tadd(slot_mul<G, double>(s0, s1, L), slot_mul<G, double>(s1, s0, L));
        Tile<double> Sp = ident<double>(L), dSp = tzero();
        axpy(C, cos_coef(1), Y);
        axpy(dC, cos_coef(1), dY);
        if (qs >= 1) {
            axpy(Sp, sin_coef(1), Y);
            axpy(dSp, sin_coef(1), dY);
        }
        Tile<double> P = Y, dP = dY;
        for (int k = 2; k <= qc; ++k) {
            team_sync<G>();
            slot_store<G, double>(s0, P, L);
            slot_store<G, double>(s1, Y, L);
            team_sync<G>();
            const Tile<double> Pn = slot_mul<G, double>(s0, s1, L);
            team_sync<G>();
            slot_store<G, double>(s1, dY, L);
            team_sync<G>();
            const Tile<double> t1 = slot_mul<G, double>(s0, s1, L);   // P dY
            team_sync<G>();
            slot_store<G, double>(s0, dP, L);
            slot_store<G, double>(s1, Y, L);
            team_sync<G>();
            const Tile<double> t2 = slot_mul<G, double>(s0, s1, L);   // dP Y
            P = Pn;
            dP = tadd(t1, t2);
            axpy(C, cos_coef(k), P);
            axpy(dC, cos_coef(k), dP);
            if (k <= qs) {
                axpy(Sp, sin_coef(k), P);
                axpy(dSp, sin_coef(k), dP);
            }
        }
        if (qs >= 1) {
            team_sync<G>();
            slot_store<G, double>(s0, Gt, L);
            slot_store<G, double>(s1, Sp, L);
            team_sync<G>();
            S = slot_mul<G, double>(s0, s1, L);
            team_sync<G>();
            slot_store<G, double>(s1, dSp, L);
            team_sync<G>();
            const Tile<double> t1 = slot_mul<G, double>(s0, s1, L);   // G dS'
            team_sync<G>();
            slot_store<G, double>(s0, Et, L);
            slot_store<G, double>(s1, Sp, L);
            team_sync<G>();
            const Tile<double> t2 = slot_mul<G, double>(s0, s1, L);   // E S'
            dS = tadd(t1, t2);
        } else {
            S = Gt;
            dS = Et;
        }
    }
    U = c_minus_is(C, S);
    dU = c_minus_is(dC, dS);
}

// pair_taylor for one-wave teams: the products whose left factor is
// Hermitian (G, and the powers of Y = G^2) are taken straight from registers
// (reg_mul_herm); the three with a general left factor (E G, dP Y, E S') are
// staged as before.  Same series, same products.
template <class G, int KS = 4>
__device__ void pair_taylor_reg(const Tile<double>& Gt, const Tile<double>& Et, int m, const Lane& L,
                                double* s0, double* s1, Tile<double>& U, Tile<double>& dU) {
    Tile<double> C = ident<double>(L), dC = tzero(), S, dS;
    if (m <= 1) {
        S = Gt;
        dS = Et;
    } else {
        const int qc = m / 2, qs = (m - 1) / 2;
        const Tile<double> Y = reg_mul_herm<double, 0, false, KS>(Gt, Gt);
        const Tile<double> dY = tadd(reg_mul_herm<double, 0, false, KS>(Gt, Et), mul2<G>(Et, Gt, L, s0, s1));
        Tile<double> Sp = ident<double>(L), dSp = tzero();
        axpy(C, cos_coef(1), Y);
        axpy(dC, cos_coef(1), dY);
        if (qs >= 1) {
            axpy(Sp, sin_coef(1), Y);
            axpy(dSp, sin_coef(1), dY);
        }
        Tile<double> P = Y, dP = dY;
        for (int k = 2; k <= qc; ++k) {
            const Tile<double> Pn = reg_mul_herm<double, 0, false, KS>(P, Y);
            const Tile<double> t1 = reg_mul_herm<double, 0, false, KS>(P, dY);   // P dY
            const Tile<double> t2 = mul2<G>(dP, Y, L, s0, s1);     // dP Y
            P = Pn;
            dP = tadd(t1, t2);
            axpy(C, cos_coef(k), P);
            axpy(dC, cos_coef(k), dP);
            if (k <= qs) {
                axpy(Sp, sin_coef(k), P);
                axpy(dSp, sin_coef(k), dP);
            }
        }
        if (qs >= 1) {
            S = reg_mul_herm<double, 0, false, KS>(Gt, Sp);
            dS = tadd(reg_mul_herm<double, 0, false, KS>(Gt, dSp), mul2<G>(Et, Sp, L, s0, s1));   // G dS' + E S'
        } else {
            S = Gt;
            dS = Et;
        }
    }
    U = c_minus_is(C, S);
    dU = c_minus_is(dC, dS);
}

// U_j = exp(-i G) from the scaled exponent Gt by the series and s squarings
// (one-wave teams: the series in registers).
template <class G, int KS = 4>
__device__ __forceinline__ Tile<double> slice_exp(const Tile<double>& Gt, int m, int s, const Lane& L, double* s0,
                                                  double* s1) {
    if constexpr (G::TW == 1) {
        Tile<double> C, P;
        taylor_parts_reg<double, 0, false, false, KS>(Gt, m, L, C, P);
        return square_n<G, double>(combine_cp<double>(C, P), s, L, s0);
    } else {
        return square_n<G, double>(taylor_exp<G, double>(Gt, m, L, s0, s1), s, L, s0);
    }
}

// Sum over the team of a per-lane value; uniform result.  red: LDS, TW doubles.
template <class G>
__device__ __forceinline__ double team_sum(double x, const Lane& L, double* red) {
    x = row16_sum(x);
    x = readlane_d(x, 0) + readlane_d(x, 16) + readlane_d(x, 32) + readlane_d(x, 48);
    if constexpr (G::TW == 1) {
        return x;
    } else {
        __syncthreads();
        if (L.lane == 0) red[L.wt] = x;
        __syncthreads();
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < G::TW; ++w) t += red[w];
        return t;
    }
}

// The product of every slice before `chain` (U_{j0-1} ... U_0) from a forward
// pass that kept its tree nodes and chain products: the aligned
// power-of-two node ranges over the blocks before this one (earliest range
// first), then this block's earlier chains.
template <class G>
__device__ Tile<double> chain_checkpoint(const PropParams& p, int64_t chain, const Lane& L, double* s0,
                                         double* s1) {
    const int64_t NN = (int64_t)G::D * G::D * 2;
    Tile<double> P = ident<double>(L);
    // leaves [0, b) as aligned tree nodes, earliest first: at level l the
    // first d_l nodes of b's group, d_l the base-kFanIn digit l of b
    const int64_t b = chain / G::NT;
    int nlev = 0;
    for (int64_t cnt = p.n_leaves; cnt > 1; cnt = (cnt + kFanIn - 1) / kFanIn) ++nlev;
    for (int l = nlev; l >= 0; --l) {
        const int64_t d = (b >> (kFanInLog2 * l)) & (kFanIn - 1);
        if (d == 0) continue;
        int64_t off = 0, cnt = p.n_leaves;
        for (int q = 0; q < l; ++q) {
            off += cnt;
            cnt = (cnt + kFanIn - 1) / kFanIn;
        }
        const int64_t first = (b >> (kFanInLog2 * (l + 1))) << kFanInLog2;
        if constexpr (G::TW == 1) {
            // one-wave team: the level's nodes are loaded together
            Tile<double> X[kFanIn - 1];
#pragma unroll
            for (int q = 0; q < kFanIn - 1; ++q)
                if (q < d) X[q] = node_load<G>(p.nodes + (off + first + q) * NN, L);
#pragma unroll
            for (int q = 0; q < kFanIn - 1; ++q)
                if (q < d) P = mul2<G>(X[q], P, L, s0, s1);
        } else {
            for (int64_t k = 0; k < d; ++k)
                P = mul2<G>(node_load<G>(p.nodes + (off + first + k) * NN, L), P, L, s0, s1);
        }
    }
    for (int64_t c = b * G::NT; c < chain; ++c)
        P = mul2<G>(node_load<G>(p.chain_out + c * NN, L), P, L, s0, s1);
    return P;
}

template <int D, int NT, bool BL>
__global__ void __launch_bounds__(64 * (D / 16) * (D / 16) * NT)
__attribute__((amdgpu_waves_per_eu(D == 64 ? 4 : 2, 8)))
backward_mfma(GradParams gp) {
    using G = Geo<D, NT>;
    const PropParams& p = gp.p;
    extern __shared__ double dsm[];
    double* slots = dsm;
    double* red = slots + NT * 2 * G::SLOT;
    double* lbasis = red + G::TD * D + 2;

    Lane L;
    L.lane = threadIdx.x & 63;
    L.g = L.lane >> 4;
    L.j = L.lane & 15;
    const int wave = wave_uniform((int)(threadIdx.x >> 6));
    const int team = wave / G::TW;
    L.wt = wave % G::TW;
    L.TI = L.wt / G::TD;
    L.TJ = L.wt % G::TD;
    L.ks = (p.du + 3) / 4;   // the tiles vanish outside the leading du x du block
    double* s0 = slots + team * 2 * G::SLOT;
    double* s1 = s0 + G::SLOT;
    if constexpr (BL) {
        const int n = p.M * G::TW * 512;
        block_copy_to_lds(lbasis, p.basis, n);
        __syncthreads();
    }
    const double* bas = BL ? lbasis : p.basis;
    // backward unit: part `part` of chain `chain` (split parts of equal length)
    const int64_t unit = (int64_t)blockIdx.x * NT + team;
    const int64_t chain = unit / gp.split;
    const int64_t part = unit % gp.split;
    if (chain >= p.n_chains) return;   // no block-wide barrier follows
    const int64_t c0 = chain * p.chunk, c1 = min(p.n_slices, c0 + p.chunk);
    const int64_t sub = (p.chunk + gp.split - 1) / gp.split;
    const int64_t j0 = min(c1, c0 + part * sub);
    const int64_t j1 = min(c1, j0 + sub);
    if (j0 >= j1) return;

    const WeightRecipe wr = weight_recipe(p, L.lane);
    const double lth = lane_theta_of(p, L.lane);
    const int64_t bofs = mfma_basis_index(D, 0, L.TI, L.TJ, 0, 0, L.lane);
    // slice j's exponent, scaled by 2^-s for its plan (m, s)
    auto slice_exponent = [&](const SliceSamples& smp, Tile<double>& Gt, int& m, int& s) {
        const double wl = combine_weight(p, wr, smp);
        double gre[4] = {0, 0, 0, 0}, gim[4] = {0, 0, 0, 0};
#pragma unroll 4
        for (int mm = 0; mm < p.M; ++mm) {
            const double w = readlane_d(wl, mm);
            const double* bb = bas + bofs + (int64_t)mm * G::TW * 512;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                gre[r] = fma(w, bb[r * 64], gre[r]);
                gim[r] = fma(w, bb[256 + r * 64], gim[r]);
            }
        }
        const double nu = wave_uniform(team_norm1<G, double>(gre, gim, L, red));
        plan_expm_lanes(p, nu, L.lane, lth, m, s);
        m = wave_uniform(m);
        s = wave_uniform(s);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            Gt.re[r] = ldexp(gre[r], -s);
            Gt.im[r] = ldexp(gim[r], -s);
        }
    };

    // checkpoint P = U_{j0-1} ... U_0: the chain's, then the unit's
    // predecessors in the chain recomputed
    Tile<double> P = chain_checkpoint<G>(p, chain, L, s0, s1);
    for (int64_t j = c0; j < j0; ++j) {
        Tile<double> Gt;
        int m, s;
        slice_exponent(gather_samples(p, wr, j), Gt, m, s);
        const Tile<double> U = slice_exp<G>(Gt, m, s, L, s0, s1);
        P = mul2<G>(U, P, L, s0, s1);
    }
    // Omega_{j0} = P Z P^H, Z = W^H U(T)
    const Tile<double> Wt = load_user<G>(gp.W, p.du, 0.0, L);
    const Tile<double> UTt = load_user<G>(gp.UT, p.du, 1.0, L);
    const Tile<double> Z = mul_adjA<G>(Wt, UTt, L, s0, s1);
    Tile<double> Om = mul_adjB<G>(mul2<G>(P, Z, L, s0, s1), P, L, s0, s1);

    SliceSamples smp = gather_samples(p, wr, j0);
    for (int64_t j = j0; j < j1; ++j) {
        const SliceSamples cur = smp;
        if (j + 1 < j1) smp = gather_samples(p, wr, j + 1);
        Tile<double> Gt;
        int m, s;
        slice_exponent(cur, Gt, m, s);
        // U_j, Lambda_j = Omega_j U_j^H and Omega_{j+1} = U_j Omega_j U_j^H =
        // U_j Lambda_j (one-wave teams without squarings: U_j Lambda_j from the
        // series' Hermitian pair C - i P in registers)
        Tile<double> Lam;
        if constexpr (G::TW == 1) {
            Tile<double> Cr, Pr;
            taylor_parts_reg<double>(Gt, m, L, Cr, Pr);
            const Tile<double> U = square_n<G, double>(combine_cp<double>(Cr, Pr), s, L, s0);
            Lam = mul_adjB<G>(Om, U, L, s0, s1);
            Om = s == 0 ? reg_mul_cp<double>(Cr, Pr, Lam) : mul2<G>(U, Lam, L, s0, s1);
        } else {
            const Tile<double> U = slice_exp<G>(Gt, m, s, L, s0, s1);
            Lam = mul_adjB<G>(Om, U, L, s0, s1);
            Om = mul2<G>(U, Lam, L, s0, s1);
        }
        // F_j = L_f(G_j, Lambda_j)
        Tile<double> Up, F;
        if constexpr (G::TW == 1) pair_taylor_reg<G>(Gt, tscale(Lam, -s), m, L, s0, s1, Up, F);
        else pair_taylor<G>(Gt, tscale(Lam, -s), m, L, s0, s1, Up, F);
        for (int q = 0; q < s; ++q) {
            team_sync<G>();
            slot_store<G, double>(s0, Up, L);
            slot_store<G, double>(s1, F, L);
            team_sync<G>();
            const Tile<double> Un = slot_mul<G, double>(s0, s0, L);
            F = tadd(slot_mul<G, double>(s0, s1, L), slot_mul<G, double>(s1, s0, L));
            Up = Un;
        }
        // dL/dw_{j,m} = Re Tr(F B_m) = sum over entries of Re(F) Re(B) + Im(F) Im(B) (B Hermitian)
        for (int mm = 0; mm < p.M; ++mm) {
            const double* bb = bas + bofs + (int64_t)mm * G::TW * 512;
            double part = 0.0;
#pragma unroll
            for (int r = 0; r < 4; ++r) part = fma(F.re[r], bb[r * 64], fma(F.im[r], bb[256 + r * 64], part));
            const double g = team_sum<G>(part, L, red);
            if (L.lane == 0 && L.wt == 0) gp.gw[j * p.M + mm] = g;
        }
    }
}

// The backward of one-wave teams (D = 16) as a two-stage pipeline: each
// unit (a chain, or a part of one) runs on two waves of the block.  The
// first (role 0) carries the recursion: slice j's exponent and plan,
// U_j, Lambda_j = Omega_j U_j^H and Omega_{j+1} = U_j Lambda_j, and hands
// (G_j scaled, Lambda_j, m, s) to the second through LDS.  The second
// (role 1) takes F_j = L_f(G_j, Lambda_j) by the (value, derivative) series
// and its contractions with the basis, for slice j while the first is at
// slice j + 1: per slice the longer of the two instead of their sum.  Before
// the slices, role 0 multiplies the checkpoint's tree nodes while role 1
// multiplies the block's earlier chains and forms Z = W^H U(T).  Same
// products as backward_mfma; the block's waves meet at two barriers per
// slice, all the same number of times (units past the end idle through them).
// A block holds UPB units: waves 0 .. UPB-1 take role 0 of units 0 .. UPB-1
// and waves UPB .. 2 UPB-1 role 1.  A CU places a block's waves on its four
// SIMDs in turn, so with UPB = 4 every SIMD runs one wave of each role (the
// lighter recursion beside the heavier derivative) instead of two of one.
template <int NT, bool BL, int KS, int UPB>
__global__ void __launch_bounds__(128 * UPB) __attribute__((amdgpu_waves_per_eu(2, 8)))
backward_pipe(GradParams gp) {
    using G = Geo<16, NT>;   // G::NT: chains per leaf of the forward's tree
    const PropParams& p = gp.p;
    extern __shared__ double dsm[];
    double* slots = dsm;
    double* red = slots + 2 * UPB * 2 * G::SLOT;
    double* lbasis = red + G::TD * 16 + 2;
    double* hand = lbasis + (BL ? p.M * 512 : 0);    // per unit: 2 tiles of 512 doubles, then m, s

    Lane L;
    L.lane = threadIdx.x & 63;
    L.g = L.lane >> 4;
    L.j = L.lane & 15;
    L.wt = 0;
    L.TI = L.TJ = 0;
    L.ks = (p.du + 3) / 4;   // the tiles vanish outside the leading du x du block
    const int wave = wave_uniform((int)(threadIdx.x >> 6));
    const int role = wave / UPB;
    const int ub = wave % UPB;   // the unit within the block
    // the derivative side is the longer of the two per slice: its waves go
    // first in their SIMD's issue (78 -> 75 us per evaluation at N = 4096)
    if (role == 1) __builtin_amdgcn_s_setprio(2);
    double* s0 = slots + wave * 2 * G::SLOT;
    double* s1 = s0 + G::SLOT;
    if constexpr (BL) {
        const int n = p.M * 512;
        block_copy_to_lds(lbasis, p.basis, n);
    }
    __syncthreads();
    const double* bas = BL ? lbasis : p.basis;
    double* hb = hand + ub * 1040;
    int* hms = reinterpret_cast<int*>(hb + 1024);
    // lane-private handoff layout: tile t, register r of lane l at t * 512 + r * 64 + l (re), + 256 (im)
    auto put = [&](int t, const Tile<double>& x) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            hb[t * 512 + r * 64 + L.lane] = x.re[r];
            hb[t * 512 + 256 + r * 64 + L.lane] = x.im[r];
        }
    };
    auto get = [&](int t) {
        Tile<double> x;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            x.re[r] = hb[t * 512 + r * 64 + L.lane];
            x.im[r] = hb[t * 512 + 256 + r * 64 + L.lane];
        }
        return x;
    };

    const int64_t unit = (int64_t)blockIdx.x * UPB + ub;
    const int64_t chain = unit / gp.split;
    const int64_t part = unit % gp.split;
    const bool live = chain < p.n_chains;
    const int64_t c0 = live ? chain * p.chunk : 0, c1 = live ? min(p.n_slices, c0 + p.chunk) : 0;
    const int64_t sub = (p.chunk + gp.split - 1) / gp.split;   // slices per unit (block-uniform bound)
    const int64_t j0 = min(c1, c0 + part * sub);
    const int64_t j1 = live ? min(c1, j0 + sub) : j0;

    const WeightRecipe wr = weight_recipe(p, L.lane);
    const double lth = lane_theta_of(p, L.lane);
    const int64_t bofs = mfma_basis_index(16, 0, 0, 0, 0, 0, L.lane);
    auto slice_exponent = [&](const SliceSamples& smp, Tile<double>& Gt, int& m, int& s) {
        const double wl = combine_weight(p, wr, smp);
        double gre[4] = {0, 0, 0, 0}, gim[4] = {0, 0, 0, 0};
#pragma unroll 4
        for (int mm = 0; mm < p.M; ++mm) {
            const double w = readlane_d(wl, mm);
            const double* bb = bas + bofs + (int64_t)mm * 512;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                gre[r] = fma(w, bb[r * 64], gre[r]);
                gim[r] = fma(w, bb[256 + r * 64], gim[r]);
            }
        }
        const double nu = wave_uniform(team_norm1<G, double>(gre, gim, L, red));
        plan_expm_lanes(p, nu, L.lane, lth, m, s);
        m = wave_uniform(m);
        s = wave_uniform(s);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            Gt.re[r] = ldexp(gre[r], -s);
            Gt.im[r] = ldexp(gim[r], -s);
        }
    };

    // checkpoint P = U_{j0-1} ... U_0 (chain_checkpoint's product, in two
    // halves) and Omega_{j0} = P Z P^H
    Tile<double> Om, P;
    const int64_t NN = 512;
    const int64_t b = chain / G::NT;   // the chain's leaf
    if (role == 0) {
        if (live) {
            // the aligned tree nodes above level 0 before the leaf's group
            P = ident<double>(L);
            int nlev = 0;
            for (int64_t cnt = p.n_leaves; cnt > 1; cnt = (cnt + kFanIn - 1) / kFanIn) ++nlev;
            for (int l = nlev; l >= 1; --l) {
                const int64_t d = (b >> (kFanInLog2 * l)) & (kFanIn - 1);
                if (d == 0) continue;
                int64_t off = 0, cnt = p.n_leaves;
                for (int q = 0; q < l; ++q) {
                    off += cnt;
                    cnt = (cnt + kFanIn - 1) / kFanIn;
                }
                const int64_t first = (b >> (kFanInLog2 * (l + 1))) << kFanInLog2;
                // four nodes in flight at a time
#pragma unroll
                for (int h = 0; h < kFanIn; h += kFanIn / 2) {
                    Tile<double> X[kFanIn / 2];
#pragma unroll
                    for (int q = 0; q < kFanIn / 2; ++q)
                        if (h + q < d) X[q] = node_load<G>(p.nodes + (off + first + h + q) * NN, L);
#pragma unroll
                    for (int q = 0; q < kFanIn / 2; ++q)
                        if (h + q < d) P = mul2<G>(X[q], P, L, s0, s1);
                }
            }
        }
    } else if (live) {
        // the level-0 nodes before the leaf in its group, then the leaf's
        // earlier chains (later on the left), and Z = W^H U(T)
        Tile<double> Pc = ident<double>(L);
        const int64_t d0 = b & (kFanIn - 1), first0 = b - d0;
        for (int64_t q = 0; q < d0; ++q) Pc = mul2<G>(node_load<G>(p.nodes + (first0 + q) * NN, L), Pc, L, s0, s1);
        for (int64_t c = b * G::NT; c < chain; ++c)
            Pc = mul2<G>(node_load<G>(p.chain_out + c * NN, L), Pc, L, s0, s1);
        const Tile<double> Wt = load_user<G>(gp.W, p.du, 0.0, L);
        const Tile<double> UTt = load_user<G>(gp.UT, p.du, 1.0, L);
        put(0, Pc);
        put(1, mul_adjA<G>(Wt, UTt, L, s0, s1));
    }
    __syncthreads();
    SliceSamples smp;
    if (role == 0 && live) {
        P = mul2<G>(get(0), P, L, s0, s1);
        const Tile<double> Z = get(1);
        // the unit's predecessors in the chain, recomputed
        for (int64_t j = c0; j < j0; ++j) {
            Tile<double> Gt;
            int m, s;
            slice_exponent(gather_samples(p, wr, j), Gt, m, s);
            P = mul2<G>(slice_exp<G, KS>(Gt, m, s, L, s0, s1), P, L, s0, s1);
        }
        Om = mul_adjB<G>(mul2<G>(P, Z, L, s0, s1), P, L, s0, s1);
        smp = gather_samples(p, wr, j0 < j1 ? j0 : 0);
    }
    __syncthreads();   // role 1 has read nothing yet; role 0 is done with the handoff area

    // the pipeline: step k, role 0 on slice j0 + k, role 1 on slice j0 + k - 1.
    // One loop per role (the other role's loop-carried state stays out of
    // its registers); both take sub + 1 steps of two barriers each.
    if (role == 0) {
        for (int64_t k = 0; k <= sub; ++k) {
            const int64_t j = j0 + k;
            const bool act = j < j1 && k < sub;
            Tile<double> Gt, Lam;
            int m = 0, s = 0;
            if (act) {
                const SliceSamples cur = smp;
                if (j + 1 < j1) smp = gather_samples(p, wr, j + 1);
                slice_exponent(cur, Gt, m, s);
                Tile<double> Cr, Pr;
                taylor_parts_reg<double, 0, false, false, KS>(Gt, m, L, Cr, Pr);
                const Tile<double> U = square_n<G, double>(combine_cp<double>(Cr, Pr), s, L, s0);
                Lam = mul_adjB<G>(Om, U, L, s0, s1);
                Om = s == 0 ? reg_mul_cp<double, 0, false, KS>(Cr, Pr, Lam) : mul2<G>(U, Lam, L, s0, s1);
            }
            __syncthreads();
            if (act) {
                put(0, Gt);
                put(1, Lam);
                if (L.lane == 0) {
                    hms[0] = m;
                    hms[1] = s;
                }
            }
            __syncthreads();
        }
    } else {
        Tile<double> Gt, Lam;
        int m = 0, s = 0;
        for (int64_t k = 0; k <= sub; ++k) {
            const int64_t j = j0 + k - 1;
            if (k >= 1 && j < j1) {
                // F_j = L_f(G_j, Lambda_j) and dL/dw_{j,m} = Re Tr(F_j B_m)
                Tile<double> Up, F;
                pair_taylor_reg<G, KS>(Gt, tscale(Lam, -s), m, L, s0, s1, Up, F);
                for (int q = 0; q < s; ++q) {
                    team_sync<G>();
                    slot_store<G, double>(s0, Up, L);
                    slot_store<G, double>(s1, F, L);
                    team_sync<G>();
                    const Tile<double> Un = slot_mul<G, double>(s0, s0, L);
                    F = tadd(slot_mul<G, double>(s0, s1, L), slot_mul<G, double>(s1, s0, L));
                    Up = Un;
                }
                for (int mm = 0; mm < p.M; ++mm) {
                    const double* bb = bas + bofs + (int64_t)mm * 512;
                    double acc = 0.0;
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc = fma(F.re[r], bb[r * 64], fma(F.im[r], bb[256 + r * 64], acc));
                    const double g = team_sum<G>(acc, L, red);
                    if (L.lane == 0) {
                        gp.gw[j * p.M + mm] = g;
                        if (gp.grad_direct && mm >= 1) gp.grad_direct[(int64_t)(mm - 1) * p.n_samples + j] = p.h * g;
                    }
                }
            }
            __syncthreads();
            __syncthreads();
            Gt = get(0);
            Lam = get(1);
            m = hms[0];
            s = hms[1];
        }
    }
}

// Rows < rows and columns < cols of a tile set from a row-major complex
// block with leading dimension ld (zero elsewhere).
template <class G>
__device__ __forceinline__ Tile<double> load_block(const double* A, int rows, int cols, int ld, const Lane& L) {
    Tile<double> t;
    const int col = 16 * L.TJ + L.j;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 16 * L.TI + crow<double>(L.g, r);
        const bool in = row < rows && col < cols;
        t.re[r] = in ? A[(row * ld + col) * 2 + 0] : 0.0;
        t.im[r] = in ? A[(row * ld + col) * 2 + 1] : 0.0;
    }
    return t;
}

template <class G>
__device__ __forceinline__ void store_block(double* A, const Tile<double>& t, int rows, int cols, int ld,
                                            const Lane& L) {
    const int col = 16 * L.TJ + L.j;
    if (col >= cols) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 16 * L.TI + crow<double>(L.g, r);
        if (row < rows) {
            A[(row * ld + col) * 2 + 0] = t.re[r];
            A[(row * ld + col) * 2 + 1] = t.im[r];
        }
    }
}

// Trajectory: every prefix P_j = U_{j-1} ... U_0, j = 0..N (applied to a
// block of states, or to a density matrix), from the same checkpoints as the
// gradient: each chain starts from its checkpoint and multiplies its
// recomputed slices in, writing its rows of the output before each slice;
// the last chain also writes j = N.
template <int D, int NT, bool BL>
__global__ void __launch_bounds__(64 * (D / 16) * (D / 16) * NT)
__attribute__((amdgpu_waves_per_eu(D == 64 ? 4 : 2, 8)))
trajectory_mfma(TrajParams tp) {
    using G = Geo<D, NT>;
    const PropParams& p = tp.p;
    extern __shared__ double dsm[];
    double* slots = dsm;
    double* red = slots + NT * 2 * G::SLOT;
    double* lbasis = red + G::TD * D + 2;

    Lane L;
    L.lane = threadIdx.x & 63;
    L.g = L.lane >> 4;
    L.j = L.lane & 15;
    const int wave = wave_uniform((int)(threadIdx.x >> 6));
    const int team = wave / G::TW;
    L.wt = wave % G::TW;
    L.TI = L.wt / G::TD;
    L.TJ = L.wt % G::TD;
    L.ks = (tp.p.du + 3) / 4;   // the tiles vanish outside the leading du x du block
    double* s0 = slots + team * 2 * G::SLOT;
    double* s1 = s0 + G::SLOT;
    if constexpr (BL) {
        const int n = p.M * G::TW * 512;
        block_copy_to_lds(lbasis, p.basis, n);
        __syncthreads();
    }
    const double* bas = BL ? lbasis : p.basis;
    const int64_t chain = (int64_t)blockIdx.x * NT + team;
    if (chain >= p.n_chains) return;   // no block-wide barrier follows
    const int64_t j0 = chain * p.chunk;
    const int64_t j1 = min(p.n_slices, j0 + p.chunk);
    const int du = p.du;
    const int cols = tp.kind == PM_TRAJ_STATES ? tp.n_vec : du;
    const int64_t stride = (int64_t)du * cols * 2;

    // S_j: P_j, P_j Psi_0 or P_j rho_0 P_j^H at the chain's first slice
    Tile<double> S = chain_checkpoint<G>(p, chain, L, s0, s1);
    if (tp.kind == PM_TRAJ_STATES) {
        S = mul2<G>(S, load_block<G>(tp.x0, du, cols, cols, L), L, s0, s1);
    } else if (tp.kind == PM_TRAJ_DENSITY) {
        S = mul_adjB<G>(mul2<G>(S, load_block<G>(tp.x0, du, du, du, L), L, s0, s1), S, L, s0, s1);
    }
    const WeightRecipe wr = weight_recipe(p, L.lane);
    const double lth = lane_theta_of(p, L.lane);
    SliceSamples smp = gather_samples(p, wr, j0);
    const int64_t bofs = mfma_basis_index(D, 0, L.TI, L.TJ, 0, 0, L.lane);
    // the commutator-free scheme has two exponentials per slice: a slice
    // boundary is every second one
    const int vs = p.order == kOrderCF4 ? 1 : 0;
    for (int64_t j = j0; j < j1; ++j) {
        if ((j & vs) == 0) store_block<G>(tp.out + (j >> vs) * stride, S, du, cols, cols, L);
        const double wl = combine_weight(p, wr, smp);
        if (j + 1 < j1) smp = gather_samples(p, wr, j + 1);
        double gre[4] = {0, 0, 0, 0}, gim[4] = {0, 0, 0, 0};
#pragma unroll 4
        for (int m = 0; m < p.M; ++m) {
            const double w = readlane_d(wl, m);
            const double* bb = bas + bofs + (int64_t)m * G::TW * 512;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                gre[r] = fma(w, bb[r * 64], gre[r]);
                gim[r] = fma(w, bb[256 + r * 64], gim[r]);
            }
        }
        const double nu = wave_uniform(team_norm1<G, double>(gre, gim, L, red));
        int m, s;
        plan_expm_lanes(p, nu, L.lane, lth, m, s);
        m = wave_uniform(m);
        s = wave_uniform(s);
        Tile<double> Gt;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            Gt.re[r] = ldexp(gre[r], -s);
            Gt.im[r] = ldexp(gim[r], -s);
        }
        if constexpr (G::TW == 1) {
            // one-wave team: the series as the Hermitian pair C - i P in
            // registers; without squarings U S straight from it (the density
            // kind's S U^H has a non-Hermitian left factor and is staged)
            Tile<double> C, P;
            taylor_parts_reg<double>(Gt, m, L, C, P);
            if (s == 0 && tp.kind != PM_TRAJ_DENSITY) {
                S = reg_mul_cp<double>(C, P, S);
                continue;
            }
            const Tile<double> U = square_n<G, double>(combine_cp<double>(C, P), s, L, s0);
            S = mul2<G>(U, S, L, s0, s1);
            if (tp.kind == PM_TRAJ_DENSITY) S = mul_adjB<G>(S, U, L, s0, s1);
        } else {
            const Tile<double> U = square_n<G, double>(taylor_exp<G, double>(Gt, m, L, s0, s1), s, L, s0);
            S = mul2<G>(U, S, L, s0, s1);
            if (tp.kind == PM_TRAJ_DENSITY) S = mul_adjB<G>(S, U, L, s0, s1);
        }
    }
    if (j1 == p.n_slices) store_block<G>(tp.out + (p.n_slices >> vs) * stride, S, du, cols, cols, L);
}

// dL/d samples from dL/dw by the weight formulas of the expand step; one
// thread per (control, sample).
__global__ void __launch_bounds__(256) samples_grad(GradParams gp, double* grad) {
    const PropParams& p = gp.p;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int K = p.K, M = p.M;
    const int64_t S = p.n_samples, N = p.n_slices;
    if (idx >= (int64_t)K * S) return;
    const int k = (int)(idx / S);
    const int64_t q = idx % S;
    const double h = p.h, h2 = h * h * (1.0 / 12.0);
    const double* g = gp.gw;
    const double* c = p.samples;
    if (p.order == 2) {
        grad[idx] = h * g[q * M + 1 + k];
        return;
    }
    if (p.order == kOrderCF4) {
        // exponents 2j and 2j+1 weigh the samples of slice j by
        // (h/12)(3, 4, -1) and (h/12)(-1, 4, 3)
        const double h12 = h * (1.0 / 12.0);
        const int64_t NS = N >> 1;
        double a = 0.0;
        if (q & 1) {
            const int64_t j = (q - 1) / 2;
            a = 4.0 * (g[(2 * j) * M + 1 + k] + g[(2 * j + 1) * M + 1 + k]);
        } else {
            const int64_t jf = q / 2, jl = q / 2 - 1;   // first sample of jf, last of jl
            if (jf < NS) a += 3.0 * g[(2 * jf) * M + 1 + k] - g[(2 * jf + 1) * M + 1 + k];
            if (jl >= 0) a += 3.0 * g[(2 * jl + 1) * M + 1 + k] - g[(2 * jl) * M + 1 + k];
        }
        grad[idx] = h12 * a;
        return;
    }
    double acc = 0.0;
    // role 1 (middle sample of slice (q-1)/2)
    if (q & 1) {
        const int64_t j = (q - 1) / 2;
        acc += (4.0 * h / 6.0) * g[j * M + 1 + k];
    } else {
        // role 0 of slice q/2 and role 2 of slice q/2 - 1
        for (int role = 0; role < 2; ++role) {
            const int64_t j = role == 0 ? q / 2 : q / 2 - 1;
            if (j < 0 || j >= N) continue;
            const double* gj = g + j * M;
            const double sg = role == 0 ? -1.0 : 1.0;   // d(s2 - s0)
            acc += (h / 6.0) * gj[1 + k] + sg * h2 * gj[1 + K + k];
            int mq = 1 + 2 * K;
            for (int a = 0; a < K; ++a)
                for (int b = a + 1; b < K; ++b, ++mq) {
                    // w = h2 (s0_a s2_b - s2_a s0_b)
                    const double* ca = c + (int64_t)a * S + 2 * j;
                    const double* cb = c + (int64_t)b * S + 2 * j;
                    if (a == k) acc += gj[mq] * h2 * (role == 0 ? cb[2] : -cb[0]);
                    if (b == k) acc += gj[mq] * h2 * (role == 0 ? -ca[2] : ca[0]);
                }
        }
    }
    grad[idx] = acc;
}

template <int D, int NT, bool BL>
hipError_t launch_bwd(const GradParams& gp, size_t lds, hipStream_t stream) {
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)backward_mfma<D, NT, BL>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const int64_t blocks = (gp.p.n_chains * gp.split + NT - 1) / NT;
    hipLaunchKernelGGL((backward_mfma<D, NT, BL>), dim3((unsigned)blocks), dim3(64 * (D / 16) * (D / 16) * NT),
                       lds, stream, gp);
    return hipGetLastError();
}

// LDS of backward_pipe with UPB units per block: two staging slots per wave,
// the reduction row, the basis when BL, and a handoff area per unit.
constexpr size_t kPipeUPB = 4;
size_t pipe_lds_bytes(int M, bool bl) {
    using G = Geo<16, 4>;
    return sizeof(double) * (2 * kPipeUPB * 2 * G::SLOT + G::TD * 16 + 2 + (bl ? (size_t)M * 512 : 0) +
                             kPipeUPB * 1040);
}

// KS: register products over the k-slices that the embedded dimension
// reaches (1 for du <= 4, 2 for du <= 8, else all 4).
template <bool BL, int KS>
hipError_t launch_bwd_pipe(const GradParams& gp, hipStream_t stream) {
    constexpr int NT = 4;   // the forward's chains per leaf
    constexpr int UPB = (int)kPipeUPB;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)backward_pipe<NT, BL, KS, UPB>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const int64_t units = gp.p.n_chains * gp.split;
    const int64_t blocks = (units + UPB - 1) / UPB;
    hipLaunchKernelGGL((backward_pipe<NT, BL, KS, UPB>), dim3((unsigned)blocks), dim3(128 * UPB),
                       pipe_lds_bytes(gp.p.M, BL), stream, gp);
    return hipGetLastError();
}

// The basis stays in LDS only while the block's LDS fits in 160 KiB.
template <int KS>
hipError_t launch_bwd_pipe_bl(const GradParams& gp, hipStream_t stream) {
    const bool bl = gp.p.basis_lds != 0 && pipe_lds_bytes(gp.p.M, true) <= 160 * 1024;
    return bl ? launch_bwd_pipe<true, KS>(gp, stream) : launch_bwd_pipe<false, KS>(gp, stream);
}

hipError_t launch_bwd_pipe_ks(const GradParams& gp, hipStream_t stream) {
    if (gp.p.du <= 4) return launch_bwd_pipe_bl<1>(gp, stream);
    return gp.p.du <= 8 ? launch_bwd_pipe_bl<2>(gp, stream) : launch_bwd_pipe_bl<4>(gp, stream);
}

template <int D, int NT, bool BL>
hipError_t launch_traj(const TrajParams& tp, size_t lds, hipStream_t stream) {
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)trajectory_mfma<D, NT, BL>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const int64_t blocks = (tp.p.n_chains + NT - 1) / NT;
    hipLaunchKernelGGL((trajectory_mfma<D, NT, BL>), dim3((unsigned)blocks), dim3(64 * (D / 16) * (D / 16) * NT),
                       lds, stream, tp);
    return hipGetLastError();
}

}  // namespace

int mfma_chains_per_block(int D);

hipError_t launch_trajectory(int D, const TrajParams& tp, hipStream_t stream) {
    const int NT = mfma_chains_per_block(D);
    const int TD = D / 16;
    size_t lds = sizeof(double) * ((size_t)NT * 2 * 2 * D * (D + 1) + (size_t)TD * D + 2);
    const bool bl = tp.p.basis_lds != 0;
    if (bl) lds += sizeof(double) * (size_t)tp.p.M * TD * TD * 512;
    switch (D) {
        case 16: return bl ? launch_traj<16, 4, true>(tp, lds, stream) : launch_traj<16, 4, false>(tp, lds, stream);
        case 32: return launch_traj<32, 1, false>(tp, lds, stream);
        case 64: return launch_traj<64, 1, false>(tp, lds, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_backward(int D, const GradParams& gp, double* grad_samples, hipStream_t stream) {
    const int NT = mfma_chains_per_block(D);
    const int TD = D / 16;
    size_t lds = sizeof(double) * ((size_t)NT * 2 * 2 * D * (D + 1) + (size_t)TD * D + 2);
    const bool bl = gp.p.basis_lds != 0;
    if (bl) lds += sizeof(double) * (size_t)gp.p.M * TD * TD * 512;
    hipError_t e;
    // D = 16: the two-wave pipeline; at order 2 it also writes dL/d samples
    // itself
    GradParams gq = gp;
    gq.grad_direct = (D == 16 && gp.p.order == 2) ? grad_samples : nullptr;
    switch (D) {
        case 16: e = launch_bwd_pipe_ks(gq, stream); break;
        case 32: e = launch_bwd<32, 1, false>(gp, lds, stream); break;
        case 64: e = launch_bwd<64, 1, false>(gp, lds, stream); break;
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    const int64_t n = (int64_t)gp.p.K * gp.p.n_samples;
    if (n == 0 || gq.grad_direct) return hipSuccess;
    hipLaunchKernelGGL(samples_grad, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, gq,
                       grad_samples);
    return hipGetLastError();
}

}  // namespace pm
