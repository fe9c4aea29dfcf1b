// Batched uneven instances in one persistent launch.
//
// One block of 16 waves per CU pulls packets from a shared counter until the
// queue is empty (every block reaches its exit).  A packet holds up to
// teams(D) consecutive chains of one instance (D = 16: 16 one-wave teams;
// D = 32: 4 teams of 4 waves; D = 64: one team of 16 waves; dimensions below
// 16 are embedded in 16).  The teams step through their chains in lockstep:
// each step expands every team's slice, takes the largest ||G||_1 over the
// teams for one shared (degree, squarings) plan, exponentiates and multiplies
// into the team's chain product; a team past the end of its chain uses G = 0,
// whose exponential is exactly I.  The team products are then multiplied in
// LDS (later chains on the left) and the packet's product enters its
// instance's ticketed FP64 tree, whose root writes that instance's U(T).
// Per-instance parameters live in device memory as PropParams records, so the
// single-propagation helpers (weights, norms, planner, Taylor) serve as is.
#include "mfma_tree.h"

namespace pm {
namespace {

template <typename T, int PMODE, int D>
__device__ void run_packet(const BatchParams& bp, const BatchPacket& P, double* dsm) {
    constexpr int TEAMS = batch_teams(D);
    using G = Geo<D, TEAMS>;
    const PropParams& p = bp.inst[P.inst];
    double* slots = dsm;
    double* red = slots + TEAMS * 2 * G::SLOT;
    double* nush = red + TEAMS * G::TD * D;
    int* tick = reinterpret_cast<int*>(nush + TEAMS);

    Lane L;
    L.lane = threadIdx.x & 63;
    L.g = L.lane >> 4;
    L.j = L.lane & 15;
    const int wave = wave_uniform((int)(threadIdx.x >> 6));
    const int team = wave / G::TW;
    L.wt = wave % G::TW;
    L.TI = L.wt / G::TD;
    L.TJ = L.wt % G::TD;
    L.ks = (p.du + 3) / 4;   // the tiles vanish outside the instance's du x du block
    double* s0 = slots + team * 2 * G::SLOT;
    double* s1 = s0 + G::SLOT;
    double* tred = red + team * G::TD * D;

    const bool active = team < P.nchains;
    const int64_t chain = P.chain0 + team;
    const int64_t j0 = active ? chain * p.chunk : 0;
    const int64_t j1 = active ? min(p.n_slices, j0 + p.chunk) : 0;
    constexpr bool kF64 = std::is_same<T, double>::value;
    Tile<T> Q = ident<T>(L);
    Tile<double> Qx = ident_as<T>(L);
    const WeightRecipe wr = weight_recipe(p, L.lane);
    const double lth = lane_theta_of(p, L.lane);
    SliceSamples smp = gather_samples(p, wr, j0);
    const int64_t bofs = mfma_basis_index(D, 0, L.TI, L.TJ, 0, 0, L.lane);
    for (int64_t t = 0; t < P.steps; ++t) {
        const int64_t j = j0 + t;
        const bool valid = j < j1;
        const double wl = valid ? combine_weight(p, wr, smp) : 0.0;
        if (j + 1 < j1) smp = gather_samples(p, wr, j + 1);
        double gre[4] = {0, 0, 0, 0}, gim[4] = {0, 0, 0, 0};
#pragma unroll 4
        for (int m = 0; m < p.M; ++m) {
            const double w = readlane_d(wl, m);
            const double* b = p.basis + bofs + (int64_t)m * G::TW * 512;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                gre[r] = fma(w, b[r * 64], gre[r]);
                gim[r] = fma(w, b[256 + r * 64], gim[r]);
            }
        }
        // one plan for the whole block: the largest norm over the teams
        const double nu_team = wave_uniform(team_norm1<G, T>(gre, gim, L, tred));
        __syncthreads();
        if (L.lane == 0 && L.wt == 0) nush[team] = nu_team;
        __syncthreads();
        double nu = 0.0;
#pragma unroll
        for (int q = 0; q < TEAMS; ++q) nu = fmax(nu, nush[q]);
        nu = wave_uniform(nu);
        int m, s;
        plan_expm_lanes(p, nu, L.lane, lth, m, s);
        m = wave_uniform(m);
        s = wave_uniform(s);
        Tile<T> Gt;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            Gt.re[r] = (T)ldexp(gre[r], -s);
            Gt.im[r] = (T)ldexp(gim[r], -s);
        }
        if constexpr (kF64) {
            Tile<T> U = taylor_exp<G, T, PMODE>(Gt, m, L, s0, s1);
            if (s > 0) U = square_n<G, double>(U, s, L, s0);
            team_sync<G>();
            slot_store<G, T>(s0, U, L);
            slot_store<G, T>(s1, Q, L);
            team_sync<G>();
            Q = mulT<G, T, PMODE>(s0, s1, L);
        } else {
            // reduced modes: I + E slices, Q <- Q + E Q with Q in FP64
            Tile<T> E = taylor_exp<G, T, PMODE, true>(Gt, m, L, s0, s1);
            if (s > 0)
                E = relayout<G, T>(square_excess_n<G>(relayout<G, double>(E, s0, L), s, L, s0), s0, L);
            chain_acc<G, T, PMODE>(Qx, E, L, s0, s1);
        }
    }
    Tile<double> Qd;
    if constexpr (kF64) Qd = Q;
    else Qd = relayout_rows<G, T, double>(Qx, s0, L);
    if constexpr (TEAMS > 1) {
        for (int st = 1; st < TEAMS; st <<= 1) {
            __syncthreads();
            slot_store<G, double>(s1, Qd, L);
            __syncthreads();
            if ((team & (2 * st - 1)) == 0) {
                const double* later = slots + (team + st) * 2 * G::SLOT + G::SLOT;
                Qd = slot_mul<G, double>(later, s1, L);
            }
        }
    }
    if constexpr (G::TW == 1) {
        if (team == 0) tree_reduce<G>(p, P.leaf, Qd, L, s0, s1, tick, true);
    } else {
        tree_reduce<G>(p, P.leaf, Qd, L, s0, s1, tick, team == 0);
    }
}

template <typename T, int PMODE>
__global__ void __launch_bounds__(1024) batch_kernel(BatchParams bp) {
    extern __shared__ double dsm[];
    __shared__ int pk_sh;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) pk_sh = (int)atomicAdd(bp.queue, 1u);
        __syncthreads();
        const int pk = pk_sh;
        if (pk >= bp.n_packets) break;
        const BatchPacket P = bp.packets[pk];
        if (P.D == 16) run_packet<T, PMODE, 16>(bp, P, dsm);
        else if (P.D == 32) run_packet<T, PMODE, 32>(bp, P, dsm);
        else run_packet<T, PMODE, 64>(bp, P, dsm);
    }
}

__global__ void batch_reset(unsigned* queue) { *queue = 0u; }

template <int D>
constexpr size_t batch_lds_for() {
    constexpr int TEAMS = batch_teams(D);
    using G = Geo<D, TEAMS>;
    return sizeof(double) * ((size_t)TEAMS * 2 * G::SLOT + (size_t)TEAMS * G::TD * D + TEAMS + 2);
}

constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }
constexpr size_t kBatchLds = cmax(batch_lds_for<16>(), cmax(batch_lds_for<32>(), batch_lds_for<64>()));

template <typename T, int PMODE>
hipError_t launch_batch_t(const BatchParams& bp, int blocks, hipStream_t stream) {
    hipLaunchKernelGGL((batch_kernel<T, PMODE>), dim3(blocks), dim3(1024), kBatchLds, stream, bp);
    return hipGetLastError();
}

template <typename T, int PMODE>
hipError_t allow_lds() {
    return hipFuncSetAttribute((const void*)batch_kernel<T, PMODE>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kBatchLds);
}

}  // namespace

// Let the batch kernels use their LDS (call before any launch or capture).
hipError_t batch_setup(int precision) {
    switch (precision) {
        case PM_FP64: return allow_lds<double, 0>();
        case PM_FP32: return allow_lds<float, 0>();
        case PM_FP32_3M: return allow_lds<float, 1>();
        case PM_BF16_SPLIT: return allow_lds<float, 2>();
        default: return hipErrorInvalidValue;
    }
}

// Reset the queue and launch the persistent kernel (both capturable).
hipError_t launch_batch(int precision, const BatchParams& bp, int blocks, hipStream_t stream) {
    hipLaunchKernelGGL(batch_reset, dim3(1), dim3(1), 0, stream, bp.queue);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (precision) {
        case PM_FP64: return launch_batch_t<double, 0>(bp, blocks, stream);
        case PM_FP32: return launch_batch_t<float, 0>(bp, blocks, stream);
        case PM_FP32_3M: return launch_batch_t<float, 1>(bp, blocks, stream);
        case PM_BF16_SPLIT: return launch_batch_t<float, 2>(bp, blocks, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace pm
