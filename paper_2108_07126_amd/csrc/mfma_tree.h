// The product tree of the MFMA engines (propagation, batch, gradient).
#pragma once

#include "mfma_tiles.h"

namespace pm {
namespace {

// Product trees over the chain (or block) products, in FP64.  With
// active == false (a multi-wave team that only keeps another team's
// barriers) a wave follows the same barriers and tickets but touches no
// memory and writes nothing.

// Publish this team's node (stored by the caller) and take a ticket on
// counter c: one agent-scope release before the ticket, and an acquire only
// for the team that goes on (ticket `proceed`).  These fences write back /
// invalidate the XCD's L2, so each is issued once per team where needed.
// Returns the ticket (the same value in every wave of the team).
template <class G>
__device__ __forceinline__ unsigned publish_ticket(const PropParams& p, int64_t c, unsigned proceed, const Lane& L,
                                                   int* tick, bool active) {
    unsigned t;
    if constexpr (G::TW == 1) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        unsigned v = 0;
        if (L.lane == 0) v = atomicAdd(&p.counters[c], 1u);
        t = (unsigned)__builtin_amdgcn_readfirstlane((int)__shfl(v, 0));
        if (t == proceed) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    } else {
        __syncthreads();   // every wave's tile of the node is stored
        if (active && L.wt == 0 && L.lane == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const unsigned v = atomicAdd(&p.counters[c], 1u);
            if (v == proceed) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            *tick = (int)v;
        }
        __syncthreads();
        t = (unsigned)*tick;
        __syncthreads();
    }
    return t;
}

// The root's product into U_out (the d x d corner of the D x D tile set).
template <class G>
__device__ __forceinline__ void store_root(const PropParams& p, const Tile<double>& Q, const Lane& L) {
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

// Product tree with fan-in kFanIn: the last of up to kFanIn consecutive
// nodes of a level to arrive multiplies them (later nodes on the left) and
// goes on; a group of one moves up unchanged.  Against a pairwise tree this
// publishes each node once and acquires once per group (for 8 leaves 8
// releases and 1 acquire instead of 14 and 7) in a third of the levels.
// With p.store_nodes every node of every level (carried ones and the root
// included) is left in `nodes`: node (l, i) holds the product over leaves
// [i 8^l, (i+1) 8^l), the aligned blocks the gradient's and the
// trajectory's checkpoints are assembled from.

template <class G>
__device__ void tree_reduce_groups(const PropParams& p, int64_t leaf, Tile<double> Q, const Lane& L,
                                   double* s0, double* s1, int* tick, bool active) {
    const int64_t NN = (int64_t)G::D * G::D * 2;
    int64_t idx = leaf, cnt = p.n_leaves, off = 0;
    while (cnt > 1) {
        const int64_t pcnt = (cnt + kFanIn - 1) / kFanIn, poff = off + cnt, grp = idx / kFanIn;
        const int64_t first = grp * kFanIn;
        const int64_t members = min(cnt, first + kFanIn) - first;
        if (members == 1 && p.store_nodes && active) node_store<G>(p.nodes + (off + idx) * NN, Q, L);
        if (members > 1) {
            if (active) node_store<G>(p.nodes + (off + idx) * NN, Q, L);
            const unsigned t = publish_ticket<G>(p, poff + grp, (unsigned)(members - 1), L, tick, active);
            if (t != (unsigned)(members - 1)) return;
            if (active && L.lane == 0 && L.wt == 0) atomicExch(&p.counters[poff + grp], 0u);
            const int64_t last = first + members - 1;
            if constexpr (G::TW == 1) {
                // one-wave team (its chain registers are free by now): the
                // group's nodes are loaded together, so their latencies
                // after the acquire overlap instead of adding up
                Tile<double> X[kFanIn];
#pragma unroll
                for (int q = 0; q < kFanIn; ++q)
                    X[q] = (q < members && first + q != idx) ? node_load<G>(p.nodes + (off + first + q) * NN, L) : Q;
                Tile<double> P = Q;
#pragma unroll
                for (int q = 0; q < kFanIn; ++q)
                    if (q == members - 1) P = X[q];
#pragma unroll
                for (int q = kFanIn - 2; q >= 0; --q)
                    if (q <= members - 2) {
                        team_sync<G>();
                        slot_store<G, double>(s0, P, L);   // left factor: later slices
                        slot_store<G, double>(s1, X[q], L);
                        team_sync<G>();
                        P = slot_mul<G, double>(s0, s1, L);
                    }
                Q = P;
            } else {
                Tile<double> P = (last == idx || !active) ? Q : node_load<G>(p.nodes + (off + last) * NN, L);
                for (int64_t k = last - 1; k >= first; --k) {
                    const Tile<double> X = (k == idx || !active) ? Q : node_load<G>(p.nodes + (off + k) * NN, L);
                    team_sync<G>();
                    slot_store<G, double>(s0, P, L);   // left factor: later slices
                    slot_store<G, double>(s1, X, L);
                    team_sync<G>();
                    P = slot_mul<G, double>(s0, s1, L);
                }
                Q = P;
            }
        }
        idx = grp;
        off = poff;
        cnt = pcnt;
    }
    if (!active) return;
    if (p.store_nodes) node_store<G>(p.nodes + off * NN, Q, L);
    store_root<G>(p, Q, L);
}

// A node published to the other XCDs inside one launch, written and read as
// agent-scope atomic accesses.  Those bypass the per-XCD L2s' private state
// (the stores write through to the device's coherence point and the loads
// read from it), so a node is visible to every XCD once its stores have
// completed: the publisher waits for that completion before it takes the
// ticket, and the ticket's last taker reads the nodes after the ticket.  A
// release/acquire fence pair would add an L2 writeback and an invalidate
// (for ordinary cached stores and loads) per node, which none of these
// accesses needs.
template <class G>
__device__ __forceinline__ void node_store_coherent(double* node, const Tile<double>& t, const Lane& L) {
    const int col = 16 * L.TJ + L.j;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 16 * L.TI + crow<double>(L.g, r);
        __hip_atomic_store(&node[(row * G::D + col) * 2 + 0], t.re[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&node[(row * G::D + col) * 2 + 1], t.im[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // the stores complete before anything after this point is issued (and
    // the compiler keeps them before it)
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

template <class G>
__device__ __forceinline__ Tile<double> node_load_coherent(double* node, const Lane& L) {
    Tile<double> t;
    const int col = 16 * L.TJ + L.j;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 16 * L.TI + crow<double>(L.g, r);
        t.re[r] = __hip_atomic_load(&node[(row * G::D + col) * 2 + 0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        t.im[r] = __hip_atomic_load(&node[(row * G::D + col) * 2 + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return t;
}

// The same tree for a block of NT one-wave teams (16-wide tiles) that all
// stay into it: team 0 publishes the block's node (coherent stores, above)
// and takes the group's ticket, and the outcome goes to every team through
// LDS.  When the block is its group's last arrival, the teams load the
// group's nodes (two each, all at once) and stage node q in LDS slot q; the
// group's product is then formed pairwise, slot q + w times slot q into slot
// q for w = 1, 2, 4 (later nodes on the left), four products at once in the
// first round: three dependent products per level instead of seven.  Same
// nodes and root as tree_reduce_groups up to the association inside each
// group.
template <class G, int NT>
__device__ void tree_reduce_teams(const PropParams& p, int64_t leaf, Tile<double> Q, const Lane& L, int team,
                                  double* slots, int* tick) {
    static_assert(G::TW == 1 && 2 * NT == kFanIn, "one slot per group member");
    constexpr int64_t NN = (int64_t)G::D * G::D * 2;
    int64_t idx = leaf, cnt = p.n_leaves, off = 0;
    while (cnt > 1) {
        const int64_t pcnt = (cnt + kFanIn - 1) / kFanIn, poff = off + cnt, grp = idx / kFanIn;
        const int64_t first = grp * kFanIn;
        const int members = (int)(min(cnt, first + kFanIn) - first);
        if (members == 1) {
            if (p.store_nodes && team == 0) node_store<G>(p.nodes + (off + idx) * NN, Q, L);
        } else {
            if (team == 0) {
                node_store_coherent<G>(p.nodes + (off + idx) * NN, Q, L);
                unsigned v = 0;
                if (L.lane == 0) v = atomicAdd(&p.counters[poff + grp], 1u);
                const unsigned t = (unsigned)__builtin_amdgcn_readfirstlane((int)__shfl(v, 0));
                if (t == (unsigned)(members - 1) && L.lane == 0) atomicExch(&p.counters[poff + grp], 0u);
                if (L.lane == 0) *tick = (int)t;
            }
            __syncthreads();
            const int t = *tick;
            __syncthreads();
            if (t != members - 1) return;   // the whole block leaves
            // node q of the group into slot q: the block's own node from
            // team 0's registers, the others loaded two per team, every load
            // in flight at once
            if (team == 0) slot_store<G, double>(slots + (idx - first) * G::SLOT, Q, L);
            Tile<double> X[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int q = team + h * NT;
                if (q < members && first + q != idx) X[h] = node_load_coherent<G>(p.nodes + (off + first + q) * NN, L);
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int q = team + h * NT;
                if (q < members && first + q != idx) slot_store<G, double>(slots + q * G::SLOT, X[h], L);
            }
            __syncthreads();
#pragma unroll
            for (int w = 1; w < kFanIn; w <<= 1) {
                const int q = 2 * w * team;
                const bool act = q + w < members;
                Tile<double> P;
                if (act) P = slot_mul<G, double>(slots + (q + w) * G::SLOT, slots + q * G::SLOT, L);
                __syncthreads();
                if (act) slot_store<G, double>(slots + q * G::SLOT, P, L);
                __syncthreads();
            }
            if (team == 0) {
                const int col = L.j;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = crow<double>(L.g, r);
                    Q.re[r] = slots[row * G::LD + col];
                    Q.im[r] = slots[G::PLANE + row * G::LD + col];
                }
            }
        }
        idx = grp;
        off = poff;
        cnt = pcnt;
    }
    if (team != 0) return;
    if (p.store_nodes) node_store<G>(p.nodes + off * NN, Q, L);
    store_root<G>(p, Q, L);
}

// The product tree over the chain (or block) products.
template <class G>
__device__ void tree_reduce(const PropParams& p, int64_t leaf, Tile<double> Q, const Lane& L,
                            double* s0, double* s1, int* tick, bool active = true) {
    tree_reduce_groups<G>(p, leaf, Q, L, s0, s1, tick, active);
}

}  // namespace
}  // namespace pm
