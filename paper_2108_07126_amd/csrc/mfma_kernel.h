#pragma once
// MFMA propagation kernel for dimensions 16, 32 and 64 (and smaller ones
// embedded in 16), shared by the translation units that instantiate it.
//
// One *team* of (D/16)^2 wavefronts runs a chain of consecutive slices; each
// wave owns one 16x16 output tile of every D x D matrix, held in registers in
// the accumulator layout of v_mfma_*_16x16x4 (lane 16 g + j holds four rows
// of column j, see crow()).  Per slice the team
//   1. expands G_j = sum_m w_m B_m in FP64 (lane m gathers the samples of
//      weight m one slice ahead; basis tiles from LDS or L2 in that layout),
//   2. bounds ||G_j||_1 and plans the Taylor degree m and squarings s,
//   3. evaluates exp(-i G) = C(Y) - i G S'(Y), Y = G^2 (cos / sin Taylor
//      series split by parity: every product is of commuting Hermitian
//      matrices), then squares s times,
//   4. optionally stores U_j, and multiplies it into the team's chain
//      product Q <- U_j Q (later slices on the left, eq. slices).
// One-wave teams (D = 16) multiply straight from registers: register r of
// a lane is the B operand of k-slice r, and the A operand of a Hermitian
// left factor (or of U = C - i P) is formed from the lane's own registers.
// Larger teams stage both operands in LDS (row stride D+1, split re/im
// planes, conflict-free fragment reads; in BF16-split mode bf16 hi/lo planes
// split once at staging).  Complex products run as three real MFMA products
// (3M) in FP64 and FP32-3M, four in plain FP32 and in BF16 split, each of
// the latter's real products three split terms (v_mfma_f64_16x16x4f64,
// v_mfma_f32_16x16x4f32, v_mfma_f32_16x16x32_bf16).
// Finally the blocks' chain products enter the ticketed FP64 product tree of
// mfma_tree.h (fan-in 8: the last of eight consecutive nodes to arrive
// multiplies them, a group of one moves up unchanged) -- the reduction of the
// Reduction by matrix multiplication section, in the same launch.
#include "mfma_tree.h"

namespace pm {
namespace {

// Waves per SIMD the register allocation must allow.  D = 16 keeps its
// whole series in registers; its launch (about two chains per SIMD) never
// asks for more than two waves per SIMD.
template <typename T, int D>
constexpr int min_waves_per_eu() {
    return D == 16 ? 2 : (D == 64 ? 4 : (std::is_same<T, double>::value ? 3 : 4));
}

// PAIR (D = 16, d <= 8, at most 32 basis matrices, the basis given in both
// diagonal 8 x 8 blocks): the team's chain is split into two halves that
// advance in lockstep, the first half's slice in the upper-left block and
// the second half's in the lower-right one.  Block-diagonal matrices stay
// block-diagonal through every product of the series, the squarings and the
// chain, so one tile carries two slices; lanes 0-31 gather the first
// slice's weights and lanes 32-63 the second's, and a lane expands with the
// weights of the block its column lies in.  At the end the halves' products
// are multiplied (second on the left) into the usual embedded chain product.
//
// M6 (FP64, PM_ORDER_MAGNUS6): the expand step forms the slice's three
// Hermitian moments P1, P2, P3 on the basis {H0, H_k} (three weights per
// basis matrix, gathered by lanes 16 q + m), and the exponent is the
// sixth-order Magnus combination of magnus6_exponent (three commutators by
// product and adjoint); the plan, the series and the chain are unchanged.
template <typename T, int D, int NT, bool BL, int PMODE, bool CH, bool PAIR, bool M6>
__global__ void __launch_bounds__(64 * (D / 16) * (D / 16) * NT)
__attribute__((amdgpu_waves_per_eu(min_waves_per_eu<T, D>(), 8)))
propagate_mfma(PropParams p) {
    using G = Geo<D, NT>;
    extern __shared__ double dsm[];
    double* slots = dsm;
    double* red = slots + NT * 2 * G::SLOT;
    int* tick = reinterpret_cast<int*>(red + G::TD * D);
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
    // staged products over the rows that the embedded dimension reaches
    // (slice pairs use both diagonal blocks)
    if constexpr (!PAIR) L.ks = (p.du + 3) / 4;
    double* s0 = slots + team * 2 * G::SLOT;
    double* s1 = s0 + G::SLOT;

    // the block's copy of the basis (same for every slice)
    if constexpr (BL) {
        const int n = p.M * G::TW * 512;
        block_copy_to_lds(lbasis, p.basis, n);
        __syncthreads();
    }
    const double* bas = BL ? lbasis : p.basis;

    // this team's chain of consecutive slices (empty past the end)
    const int64_t chain = (int64_t)blockIdx.x * NT + team;
    const int64_t j0 = min(p.n_slices, chain_first(p, chain));
    const int64_t j1 = min(p.n_slices, chain_first(p, chain + 1));
    static_assert(!PAIR || D == 16, "slice pairs live in the 16-wide tile");
    static_assert(!M6 || (std::is_same<T, double>::value && !PAIR), "sixth order: FP64, one slice per tile");
    // PAIR: halves [j0, jm) and [jm, j1); otherwise one run [j0, j1)
    const int64_t jm = PAIR ? j0 + (j1 - j0 + 1) / 2 : j1;
    const int64_t steps = jm - j0;
    const bool wsecond = PAIR && L.lane >= 32;   // this lane gathers the second half's weight
    const bool bsecond = PAIR && L.j >= 8;       // this lane's column lies in the second block
    const int64_t wbase = wsecond ? jm : j0, wend = wsecond ? j1 : jm;
    const int64_t jlast = p.n_slices > 0 ? p.n_slices - 1 : 0;
    constexpr bool kF64 = std::is_same<T, double>::value;
    // FP64: the chain product in registers.  Reduced modes: slices as I + E
    // (E accurate relative to ||G||) and the chain as Q <- Q + E Q with Q in
    // FP64, so the rounding of the working precision never touches the
    // identity part.
    Tile<T> Q = ident<T>(L);
    Tile<double> Qx = ident_as<T>(L);
    // lane m < M gathers and combines the weight of basis matrix m; the next
    // slice's samples are loaded while this slice is exponentiated
    WeightRecipe wr;
    if constexpr (M6) wr = m6_recipe(p, L.lane);
    else wr = weight_recipe(p, PAIR ? (L.lane & 31) : L.lane);
    auto gather = [&](int64_t j) {
        if constexpr (M6) return m6_gather(p, wr, j);
        else return gather_samples(p, wr, j);
    };
    const double lth = lane_theta_of(p, L.lane);
    const double lcth = lane_ctheta_of(p, L.lane);
    SliceSamples smp = gather(min(wbase, jlast));
    // output of the step's slice(s); the second block's slice in PAIR mode
    auto store_out = [&](int64_t t, const Tile<T>& U) {
        if constexpr (PAIR) store_slice_pair<G, T>(p, j0 + t, jm + t < j1 ? jm + t : -1, U, L);
        else store_slice<G, T>(p, j0 + t, U, L);
    };
    for (int64_t t = 0; t < steps; ++t) {
        double wl;
        if constexpr (M6) wl = wbase + t < wend ? m6_weight(p, wr, smp) : 0.0;
        else wl = wbase + t < wend ? combine_weight(p, wr, smp) : 0.0;
        if (t + 1 < steps) smp = gather(min(wbase + t + 1, jlast));
        // expand (FP64)
        double gre[4] = {0, 0, 0, 0}, gim[4] = {0, 0, 0, 0};
        const int64_t bofs = mfma_basis_index(D, 0, L.TI, L.TJ, 0, 0, L.lane);
        if constexpr (M6) {
            // the three moments from one pass over the basis, then the
            // sixth-order exponent
            Tile<double> P1, P2, P3;
#pragma unroll
            for (int r = 0; r < 4; ++r) P1.re[r] = P1.im[r] = P2.re[r] = P2.im[r] = P3.re[r] = P3.im[r] = 0.0;
            const double* bb = bas + bofs;
            constexpr int64_t STR = G::TW * 512;
            for (int m = 0; m < p.M; ++m) {
                const double w1 = readlane_d(wl, m), w2 = readlane_d(wl, 16 + m), w3 = readlane_d(wl, 32 + m);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const double xr = bb[m * STR + r * 64], xi = bb[m * STR + 256 + r * 64];
                    P1.re[r] = fma(w1, xr, P1.re[r]);
                    P1.im[r] = fma(w1, xi, P1.im[r]);
                    P2.re[r] = fma(w2, xr, P2.re[r]);
                    P2.im[r] = fma(w2, xi, P2.im[r]);
                    P3.re[r] = fma(w3, xr, P3.re[r]);
                    P3.im[r] = fma(w3, xi, P3.im[r]);
                }
            }
            const Tile<double> Gm = magnus6_exponent<G>(P1, P2, P3, L, s0, s1);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                gre[r] = Gm.re[r];
                gim[r] = Gm.im[r];
            }
        } else {
            // four basis matrices' entries are loaded before their FMAs, so
            // the load latencies overlap; the sum still runs in order of m
            const double* bb = bas + bofs;
            constexpr int64_t STR = G::TW * 512;
            int m = 0;
            // (one-wave teams only: a 16-wave team's 128 registers per lane
            // would spill the four matrices' entries)
            for (; G::TW == 1 && m + 4 <= p.M; m += 4) {
                double x[4][8];
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        x[q][r] = bb[(m + q) * STR + r * 64];
                        x[q][4 + r] = bb[(m + q) * STR + 256 + r * 64];
                    }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    double w = readlane_d(wl, m + q);
                    if constexpr (PAIR) {
                        const double w2 = readlane_d(wl, 32 + m + q);
                        w = bsecond ? w2 : w;
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        gre[r] = fma(w, x[q][r], gre[r]);
                        gim[r] = fma(w, x[q][4 + r], gim[r]);
                    }
                }
            }
            for (; m < p.M; ++m) {
                double w = readlane_d(wl, m);
                if constexpr (PAIR) {
                    const double w2 = readlane_d(wl, 32 + m);
                    w = bsecond ? w2 : w;
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    gre[r] = fma(w, bb[m * STR + r * 64], gre[r]);
                    gim[r] = fma(w, bb[m * STR + 256 + r * 64], gim[r]);
                }
            }
        }
        // plan (FP64)
        const double nu = wave_uniform(team_norm1<G, T>(gre, gim, L, red));
        int m, s;
        if constexpr (CH) plan_cheb_lanes(p, nu, L.lane, lcth, m, s);
        else plan_expm_lanes(p, nu, L.lane, lth, m, s);
        m = wave_uniform(m);
        s = wave_uniform(s);
        Tile<T> Gt;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            Gt.re[r] = (T)ldexp(gre[r], -s);
            Gt.im[r] = (T)ldexp(gim[r], -s);
        }
        if constexpr (kF64) {
            // exponentiate, square, store, chain product Q <- U Q
            Tile<T> U;
            if constexpr (G::TW == 1) {
                // one-wave team: the series as the Hermitian pair C - i P and,
                // without squarings, the chain product straight from it, all
                // in registers
                Tile<double> C, P;
                if constexpr (CH)
                    cheb_parts<G>(Gt, m, p.ctheta[m], p.cheb_j + kChebSplitOffset + m * 2 * kChebHalf, L, s0,
                                  s1, C, P);
                else
                    // slice pairs: the stacked block products (half the MFMA work)
                    taylor_parts_reg<double, 0, false, PAIR>(Gt, m, L, C, P);
                if (s == 0) {
                    if (p.slices_out) store_out(t, combine_cp<double>(C, P));
                    Q = reg_mul_cp<double, 0, PAIR>(C, P, Q);
                    continue;
                }
                U = combine_cp<double>(C, P);
            } else if constexpr (CH) {
                Tile<double> C, P;
                cheb_parts<G>(Gt, m, p.ctheta[m], p.cheb_j + kChebSplitOffset + m * 2 * kChebHalf, L, s0, s1, C,
                              P);
                U = combine_cp<double>(C, P);
            } else {
                U = taylor_exp<G, T, PMODE>(Gt, m, L, s0, s1);
            }
            if constexpr (PAIR) {
                // full 16-wide products follow: clear the cross blocks
                pair_mask(U, L);
                pair_mask(Q, L);
            }
            if (s > 0) U = square_n<G, double>(U, s, L, s0);
            if (p.slices_out) store_out(t, U);
            team_sync<G>();
            slot_store<G, T>(s0, U, L);
            slot_store<G, T>(s1, Q, L);
            team_sync<G>();
            Q = mulT<G, T, PMODE>(s0, s1, L);
        } else {
            Tile<T> E;
            if constexpr (G::TW == 1) {
                // one-wave team: E = C - i P in registers and, without
                // squarings, Q <- Q + E Q with E Q in registers too
                Tile<T> C, P;
                taylor_parts_reg<T, PMODE, true>(Gt, m, L, C, P);
                if (s == 0) {
                    if (p.slices_out) store_out(t, plus_ident<T>(combine_cp<T>(C, P), L));
                    Tile<T> Qt;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        Qt.re[r] = (T)Qx.re[r];
                        Qt.im[r] = (T)Qx.im[r];
                    }
                    const Tile<T> EQ = reg_mul_cp<T, PMODE>(C, P, Qt);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        Qx.re[r] += (double)EQ.re[r];
                        Qx.im[r] += (double)EQ.im[r];
                    }
                    continue;
                }
                E = combine_cp<T>(C, P);
            } else {
                E = taylor_exp<G, T, PMODE, true>(Gt, m, L, s0, s1);
            }
            if (s > 0)
                E = relayout<G, T>(square_excess_n<G>(relayout<G, double>(E, s0, L), s, L, s0), s0, L);
            if (p.slices_out) store_out(t, plus_ident<T>(E, L));
            chain_acc<G, T, PMODE>(Qx, E, L, s0, s1);
        }
    }
    Tile<double> Qd;
    if constexpr (kF64) Qd = Q;
    else Qd = relayout_rows<G, T, double>(Qx, s0, L);
    if constexpr (PAIR) Qd = pair_product<G>(Qd, L, s0, s1);
    if (p.chain_out && chain < p.n_chains)
        node_store<G>(p.chain_out + chain * (int64_t)G::D * G::D * 2, Qd, L);
    // one-wave teams of a block: combine their chains in LDS (later team on
    // the left), so the block enters the global tree as a single leaf
    if constexpr (NT > 1) {
        for (int st = 1; st < NT; st <<= 1) {
            __syncthreads();
            slot_store<G, double>(s1, Qd, L);
            __syncthreads();
            if ((team & (2 * st - 1)) == 0) {
                const double* later = slots + (team + st) * 2 * G::SLOT + G::SLOT;
                Qd = slot_mul<G, double>(later, s1, L);
            }
        }
        if constexpr (G::TW == 1 && 2 * NT == kFanIn) {
            // the block's teams stay together into the tree
            tree_reduce_teams<G, NT>(p, blockIdx.x, Qd, L, team, slots, tick);
            return;
        }
        if (team != 0) return;
    }
    tree_reduce<G>(p, blockIdx.x, Qd, L, s0, s1, tick);
}

template <int D, int NT>
constexpr size_t lds_fixed_bytes() {
    using G = Geo<D, NT>;
    return sizeof(double) * ((size_t)NT * 2 * G::SLOT + (size_t)G::TD * D + 2);
}

template <typename T, int D, int NT, bool BL, int PMODE, bool CH, bool PAIR, bool M6>
hipError_t launch_one(const PropParams& p, hipStream_t stream) {
    using G = Geo<D, NT>;
    const size_t lds = lds_fixed_bytes<D, NT>() + (BL ? sizeof(double) * (size_t)p.M * G::TW * 512 : 0);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)propagate_mfma<T, D, NT, BL, PMODE, CH, PAIR, M6>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL((propagate_mfma<T, D, NT, BL, PMODE, CH, PAIR, M6>), dim3((unsigned)p.n_leaves),
                       dim3(G::THREADS), lds, stream, p);
    return hipGetLastError();
}

template <typename T, int D, int NT, int PMODE, bool CH, bool PAIR = false, bool M6 = false>
hipError_t launch_bl(const PropParams& p, hipStream_t stream) {
    if constexpr (D == 16) {
        if (p.basis_lds) return launch_one<T, D, NT, true, PMODE, CH, PAIR, M6>(p, stream);
    }
    return launch_one<T, D, NT, false, PMODE, CH, PAIR, M6>(p, stream);
}

// The Chebyshev series is an FP64 method.
template <typename T, int D, int NT, int PMODE>
hipError_t launch_method(const PropParams& p, hipStream_t stream) {
    if constexpr (std::is_same<T, double>::value) {
        if (p.method == PM_EXPM_CHEBYSHEV) return launch_bl<T, D, NT, PMODE, true, false>(p, stream);
    }
    return launch_bl<T, D, NT, PMODE, false, false>(p, stream);
}

}  // namespace

// Teams per block for the one-wave teams of D = 16.
constexpr int kNT16 = 4;

}  // namespace pm
