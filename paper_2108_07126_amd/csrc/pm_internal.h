// Internal interface between the host runtime (parament.cpp) and the HIP
// engines.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/parament.h"

namespace pm {

constexpr int kMaxCtrl = 8;
constexpr int kMaxBasis = 1 + 2 * kMaxCtrl + kMaxCtrl * (kMaxCtrl - 1) / 2;  // 45
constexpr int kMaxDeg = PM_MAX_TAYLOR_DEGREE;
constexpr int kMaxCheb = PM_MAX_CHEBYSHEV_DEGREE;
// Chebyshev table: rows [m][k] = J_k(theta_m), k <= kMaxCheb, then for the
// even/odd split rows [m][2][kChebHalf] of the even and odd coefficients.
constexpr int kChebHalf = kMaxCheb / 2 + 1;
constexpr int kChebSplitOffset = (kMaxCheb + 1) * (kMaxCheb + 1);
constexpr int kOrderCF4 = PM_ORDER_CF4;   // two exponentials per slice, in product order
constexpr int kOrderM6 = PM_ORDER_MAGNUS6; // sixth-order Magnus, three samples per slice
constexpr int kFanIn = 8;                  // fan-in of the MFMA engines' product tree
constexpr int kFanInLog2 = 3;

// Everything one propagation launch needs, passed by value as the kernel
// argument.  Pointers are device pointers.
struct PropParams {
    const double* basis;      // Hermitian basis in the engine's layout, FP64
    const double* samples;    // [K][n_samples]
    int64_t n_samples;
    int64_t n_slices;         // N
    int64_t chunk;            // consecutive slices per chain (after the first n_long chains)
    int64_t n_long;           // the first n_long chains hold chunk_long slices each (0: none)
    int64_t chunk_long;
    int64_t n_chains;         // chains covering the N slices
    int64_t n_leaves;         // leaves of the product tree (blocks or waves)
    void* slices_out;         // nullptr or [N][du][du] complex (c128 / c64)
    double* nodes;            // tree nodes, [2 * n_leaves][D][D] complex128
    unsigned* counters;       // [2 * n_leaves] pair tickets, zero between launches
    double* U_out;            // [du][du] complex128
    double* chain_out;        // nullptr or [n_chains][D][D] complex128 chain products
    int store_nodes;          // keep every tree node (gradient checkpoints)
    double h;
    double theta[kMaxDeg + 1];   // Taylor thresholds for the working precision
    int K, M, order, du;
    int max_degree, force_s;
    int basis_lds;               // MFMA engine: block keeps a copy of the basis in LDS
    int pair;                    // MFMA engine, D = 16: two slices of dimension <= 8 per tile
    int method;                  // PM_EXPM_TAYLOR or PM_EXPM_CHEBYSHEV
    const double* cheb_j;        // Chebyshev: [m][k] = J_k(ctheta[m]), k <= m <= kMaxCheb; then the split rows
    double ctheta[kMaxCheb + 1]; // Chebyshev: half-width of the spectral interval for degree m
    uint8_t pair_a[kMaxBasis];   // order 4: control indices of i[H_a, H_b]
    uint8_t pair_b[kMaxBasis];
};

// The gradient kernels' arguments.
struct GradParams {
    PropParams p;       // forward parameters; p.nodes and p.chain_out filled by the forward
    const double* W;    // [du][du] complex128, dL = Re Tr(W^H dU(T))
    const double* UT;   // [du][du] complex128, U(T) of that forward
    double* gw;         // [N][M] dL / d w_{j,m}
    int split;          // backward units per chain (>= 1): unit u covers part u % split of chain u / split
    double* grad_direct;  // order 2 on the pipelined backward: dL/d samples written there directly
                          // (dL/dc_k(j) = h dL/dw_{j,1+k}), no separate chain-rule kernel; else null
};

// Trajectory kernel arguments (PM_TRAJ_* kinds of the public header).
struct TrajParams {
    PropParams p;       // forward parameters; p.nodes and p.chain_out filled by the forward
    int kind;           // propagators, states or density
    const double* x0;   // [du][n_vec] states or [du][du] density, complex128; unused for propagators
    int n_vec;          // state columns
    double* out;        // [N+1][du][cols] complex128
};

hipError_t launch_trajectory(int D, const TrajParams& tp, hipStream_t stream);

// Propagation with the tree workspace in a caller-provided device region
// (parament.cpp; used by the entry point that allocates nothing).
pm_status equiprop_fixed_workspace(pm_ctx* ctx, const double* samples_dev, int64_t n_samples, double dt,
                                   double* U_out_dev, void* slices_out_dev, void* stream, void* base,
                                   size_t bytes);
int context_device(const pm_ctx* ctx);
pm_status context_device_fail(pm_ctx* ctx, hipError_t e, const char* where);

// Control optimisation helpers (engine_grape.hip).
hipError_t launch_fidelity(const double* U, const double* V, int du, double* W, double* loss, hipStream_t st);
hipError_t launch_update(double* c, const double* g, double* m, double* v, int64_t n, double step, int optimizer,
                         int it, double b1, double b2, double eps, hipStream_t st);
hipError_t launch_zero(double* a, int64_t n, hipStream_t st);

// Batched instances: a packet is up to teams(D) consecutive chains of one
// instance, run in lockstep by one block of the persistent batch kernel.
struct BatchPacket {
    int inst;          // instance index
    int D;             // 16, 32 or 64
    int nchains;       // chains in the packet (the rest of the block's teams idle)
    int leaf;          // packet index within its instance = leaf of the instance's tree
    int64_t chain0;    // first chain; team t runs chain chain0 + t
    int64_t steps;     // slices of the packet's longest chain
};

struct BatchParams {
    const PropParams* inst;      // device array, one record per instance
    const BatchPacket* packets;  // in execution order
    int n_packets;
    unsigned* queue;             // next packet; zeroed before every launch
};

constexpr int batch_teams(int D) { return D == 16 ? 16 : (D == 32 ? 4 : 1); }

// Engines.  D is the (padded) engine dimension.
//   MFMA engine: D in {16, 32, 64}; one team of (D/16)^2 waves per slice
//   chain, every wave owning one 16x16 output tile.
//   VALU engine: D in {2, 4}; one slice per lane.
enum EngineKind { ENGINE_VALU = 0, ENGINE_MFMA = 1 };

struct EngineInfo {
    int kind;
    int D;                 // engine dimension
    int chunk_unit;        // a chain's length is a multiple of this
    int chains_per_leaf;   // chains combined before the global tree
    int resident_chains;   // chains the whole GPU runs at once (rough)
    int f64_rows;          // MFMA: accumulator rows interleaved as in FP64 (g + 4r)
};

// Engine choice for a user dimension; false if unsupported.
bool pick_engine(int du, int precision, EngineInfo* out);

// Basis layout of the engine, filled from the FP64 basis [M][du][du]
// (interleaved complex, row-major) into `dst` (host memory, size from
// basis_layout_doubles).
int64_t basis_layout_doubles(const EngineInfo& e, int M);
void basis_to_layout(const EngineInfo& e, int M, int du, const double* basis, double* dst);

hipError_t launch_propagate(const EngineInfo& e, int precision, const PropParams& p,
                            hipStream_t stream);

// MFMA basis layout: [m][tile][plane][r][lane] with tile = TI*(D/16)+TJ,
// lane = 16 g + j holding element (16 TI + row(g, r), 16 TJ + j), where
// row(g, r) = g + 4 r for FP64 kernels and 4 g + r for FP32 kernels (the
// accumulator layouts of the two 16x16x4 MFMA instructions).
__host__ __device__ inline int64_t mfma_basis_index(int D, int m, int TI, int TJ, int plane,
                                                    int r, int lane) {
    const int TD = D / 16;
    return ((((int64_t)m * TD * TD + TI * TD + TJ) * 2 + plane) * 4 + r) * 64 + lane;
}

}  // namespace pm
