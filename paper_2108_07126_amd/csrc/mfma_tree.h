// The product tree of the MFMA engines (propagation, batch, gradient).
#pragma once

#include "mfma_tiles.h"

namespace pm {
namespace {

// Pairwise product tree over the chain products (FP64).  Level l holds
// cnt_l nodes; node i pairs with i^1 (odd index = later slices = left
// factor); an unpaired last node moves up unchanged.  The first team to reach
// a pair leaves its product in `nodes` and exits; the second multiplies.
// With p.store_nodes every node of every level (carried ones and the root
// included) is left in `nodes`, so node (l, i) holds the product over leaves
// [i 2^l, (i+1) 2^l) for the gradient's checkpoints.
// With active == false (a multi-wave team that only keeps another team's
// barriers) the wave follows the same barriers and tickets but touches no
// memory and writes nothing.
template <class G>
__device__ void tree_reduce(const PropParams& p, int64_t leaf, Tile<double> Q, const Lane& L,
                            double* s0, double* s1, int* tick, bool active = true) {
    const int64_t NN = (int64_t)G::D * G::D * 2;
    int64_t idx = leaf, cnt = p.n_leaves, off = 0;
    while (cnt > 1) {
        const int64_t pcnt = (cnt + 1) >> 1, poff = off + cnt, par = idx >> 1;
        const bool carry = (idx == cnt - 1) && (cnt & 1);
        if (carry && p.store_nodes && active) node_store<G>(p.nodes + (off + idx) * NN, Q, L);
        if (!carry) {
            if (active) node_store<G>(p.nodes + (off + idx) * NN, Q, L);
            // publish the node with one agent-scope release before the
            // ticket, and acquire only as the second arriver of a pair:
            // these fences write back / invalidate the XCD's L2, so each is
            // issued once per team where it is needed
            unsigned t;
            if constexpr (G::TW == 1) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                unsigned v = 0;
                if (L.lane == 0) v = atomicAdd(&p.counters[poff + par], 1u);
                t = (unsigned)__builtin_amdgcn_readfirstlane((int)__shfl(v, 0));
                if (t == 0) return;
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            } else {
                __syncthreads();   // every wave's tile of the node is stored
                if (active && L.wt == 0 && L.lane == 0) {
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                    const unsigned v = atomicAdd(&p.counters[poff + par], 1u);
                    if (v != 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    *tick = (int)v;
                }
                __syncthreads();
                t = (unsigned)*tick;
                __syncthreads();
                if (t == 0) return;
            }
            if (active && L.lane == 0 && L.wt == 0) atomicExch(&p.counters[poff + par], 0u);
            const Tile<double> other = active ? node_load<G>(p.nodes + (off + (idx ^ 1)) * NN, L) : Q;
            team_sync<G>();
            slot_store<G, double>(s0, (idx & 1) ? Q : other, L);   // left factor: later slices
            slot_store<G, double>(s1, (idx & 1) ? other : Q, L);
            team_sync<G>();
            Q = slot_mul<G, double>(s0, s1, L);
        }
        idx = par;
        off = poff;
        cnt = pcnt;
    }
    if (!active) return;
    if (p.store_nodes) node_store<G>(p.nodes + off * NN, Q, L);
    const int col = 16 * L.TJ + L.j;
    if (col < p.du) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * L.TI + crow<double>(L.g, r);
            if (row < p.du) {
                p.U_out[(row * p.du + col) * 2 + 0] = Q.re[r];
                p.U_out[(row * p.du + col) * 2 + 1] = Q.im[r];
            }
        }
    }
}

}  // namespace
}  // namespace pm
