// Host runtime of the C ABI declared in include/parament.h: contexts, input
// validation, the Hermitian basis (drift, controls and the effective
// commutator controls of eq. magnus_coeffs), Taylor thresholds and
// planning, engine choice, workspace, and the launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "pm_internal.h"

namespace pm {
hipError_t launch_mfma(int D, int precision, const PropParams& p, hipStream_t stream);
hipError_t launch_valu(int D, bool fp64, const PropParams& p, hipStream_t stream);
int mfma_chains_per_block(int D);
hipError_t launch_backward(int D, const GradParams& gp, double* grad_samples, hipStream_t stream);
hipError_t launch_batch(int precision, const BatchParams& bp, int blocks, hipStream_t stream);
hipError_t batch_setup(int precision);
}  // namespace pm

using cplx = std::complex<double>;

struct pm_ctx {
    int device = 0;
    int precision = PM_FP64;
    bool ready = false;
    bool broken = false;
    int64_t dim = 0;
    int64_t n_ctrl = 0;
    int order = 2;
    int M = 0;
    pm::EngineInfo eng{};
    std::vector<double> basis;   // FP64 [M][dim][dim] interleaved
    std::vector<double> norms;   // [M]
    uint8_t pair_a[pm::kMaxBasis] = {};
    uint8_t pair_b[pm::kMaxBasis] = {};
    double theta[pm::kMaxDeg + 1] = {};
    int64_t theta_n = -1;        // slice count the theta table was made for
    int max_degree = PM_MAX_TAYLOR_DEGREE;
    int force_s = -1;
    int64_t chunk_override = 0;
    int chain_skew = -1;         // pm_set_chain_skew: percent, -1 automatic
    int n_cu = 256;              // compute units of the device
    int64_t call_chunk = 0;      // chain length planned for the current call (0: none)
    int64_t ws_limit = 0;        // device workspace limit in bytes (0: none)
    int method = PM_EXPM_TAYLOR;
    double* d_cheb = nullptr;    // Chebyshev coefficient table on the device
    // device buffers
    double* d_basis = nullptr;
    double* d_nodes = nullptr;
    size_t nodes_bytes = 0;
    unsigned* d_counters = nullptr;
    size_t counters_bytes = 0;
    double* d_basis_pair = nullptr;   // D = 16, d <= 8: the basis in both diagonal blocks
    double* d_samples = nullptr;
    size_t samples_bytes = 0;
    double* d_U = nullptr;
    size_t u_bytes = 0;
    void* d_slices = nullptr;
    size_t slices_bytes = 0;
    // gradient: FP64 MFMA engine (d <= 4 embedded in 16) and its workspace
    pm::EngineInfo geng{};
    double* d_basis_grad = nullptr;   // null: d_basis already has the gradient engine's layout
    double* d_chain = nullptr;
    size_t chain_bytes = 0;
    double* d_gw = nullptr;
    size_t gw_bytes = 0;
    double* d_UT = nullptr;
    size_t ut_bytes = 0;
    double* d_W = nullptr;
    size_t w_bytes = 0;
    double* d_grad = nullptr;
    size_t grad_bytes = 0;
    double* d_mom = nullptr;      // optimiser moments [2][K * n_samples]
    size_t mom_bytes = 0;
    std::string err;
};

namespace {

pm_status fail(pm_ctx* ctx, pm_status s, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return s;
}

pm_status hip_fail(pm_ctx* ctx, hipError_t e, const char* where) {
    if (ctx) {
        ctx->broken = true;
        ctx->err = std::string(where) + ": " + hipGetErrorString(e);
    }
    return PM_E_DEVICE;
}

struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Why the last pm_create / pm_batch_create on this thread failed (no
// handle exists to carry the message).
thread_local std::string g_create_err;

pm_status create_fail(pm_status s, const std::string& what, hipError_t e = hipSuccess) {
    g_create_err = e == hipSuccess ? what : what + ": " + hipGetErrorString(e);
    (void)hipGetLastError();
    return s;
}

double unit_roundoff(int precision) {
    switch (precision) {
        case PM_FP64: return std::ldexp(1.0, -53);
        case PM_FP32:
        case PM_FP32_3M: return std::ldexp(1.0, -24);
        case PM_BF16_SPLIT: return std::ldexp(1.0, -16);
        default: return -1.0;
    }
}

// Largest theta with theta^(m+1)/(m+1)! / (1 - theta/(m+2)) <= u, or, with
// `relative`, the same bound divided by theta (the remainder relative to
// ||X|| = theta) <= u.  Both bounds increase on [0, m+2).
double taylor_theta(int m, double u, bool relative) {
    auto bound = [m, relative](double th) {
        double t = 1.0;
        for (int k = 1; k <= m + 1; ++k) t *= th / k;
        t /= (1.0 - th / (m + 2));
        return relative ? (th > 0.0 ? t / th : 0.0) : t;
    };
    double lo = 0.0, hi = m + 1.0;   // bound is increasing on [0, m+2)
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (bound(mid) <= u) lo = mid; else hi = mid;
    }
    return lo;
}

int taylor_products_host(int m) {
    if (m <= 1) return 0;
    if (m == 2) return 1;
    return m / 2 + 1;
}

void plan_host(const double* theta, int md, int force_s, double nu, int* m_out, int* s_out) {
    auto next = [](int c) { return c < 3 ? c + 1 : c + 2; };
    if (force_s >= 0) {
        const double x = std::ldexp(nu, -force_s);
        int m = md;
        for (int c = 1; c <= md; c = next(c))
            if (theta[c] >= x) { m = c; break; }
        *m_out = m;
        *s_out = force_s;
        return;
    }
    int bm = md, bs = 0, bc = 1 << 30;
    for (int s = 0; s < 64; ++s) {
        if (s >= bc) break;
        const double x = std::ldexp(nu, -s);
        for (int c = 1; c <= md; c = next(c)) {
            if (theta[c] >= x) {
                const int cost = taylor_products_host(c) + s;
                if (cost < bc) { bc = cost; bm = c; bs = s; }
                break;
            }
        }
    }
    if (bc == (1 << 30)) { bm = md; bs = 0; }
    *m_out = bm;
    *s_out = bs;
}

// Truncation target for a propagation of n slices (see pm_taylor_theta).
double truncation_target(int precision, int64_t n) {
    const double u = unit_roundoff(precision);
    return std::max(std::ldexp(1.0, -53), u / std::sqrt((double)std::max<int64_t>(n, 1)));
}

// Reduced-precision modes carry each slice as I + E and accumulate the
// chains as Q + E Q, so their rounding error scales with ||E|| ~ ||G||; the
// truncation criterion is relative to ||G|| to match.
bool relative_truncation(int precision) { return precision != PM_FP64; }

void fill_theta(double* theta, int precision, int64_t n) {
    const double u = truncation_target(precision, n);
    theta[0] = 0.0;
    for (int m = 1; m <= pm::kMaxDeg; ++m) theta[m] = taylor_theta(m, u, relative_truncation(precision));
}

// Lubich's estimate of the Chebyshev truncation error (eq. error_chebychev)
// for degree m and spectral width w = beta - alpha.
double lubich_error(int m, double w) {
    const double rho = w / (4.0 * m + 4.0);
    return 4.0 * std::pow(std::exp(1.0 - rho * rho) * rho, m + 1);
}

// Largest ||G|| with lubich_error(m, 2 ||G||) <= u; the estimate increases in
// rho up to rho = 1/sqrt(2), which brackets the root.
double chebyshev_theta(int m, double u) {
    double lo = 0.0, hi = 1.0 / std::sqrt(2.0);
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (lubich_error(m, mid * (4.0 * m + 4.0)) <= u) lo = mid; else hi = mid;
    }
    return lo * (4.0 * m + 4.0) / 2.0;
}

void plan_chebyshev_host(const double* ctheta, int md, int force_s, double nu, int* m_out, int* s_out) {
    if (force_s >= 0) {
        const double x = std::ldexp(nu, -force_s);
        int m = md;
        for (int c = 1; c <= md; ++c)
            if (ctheta[c] >= x) { m = c; break; }
        *m_out = m;
        *s_out = force_s;
        return;
    }
    // cost: the even/odd split's products plus the squarings; the smallest
    // feasible degree of each s is its cheapest
    int bm = md, bs = 0, bc = 1 << 30;
    for (int s = 0; s < 64 && s < bc; ++s) {
        const double x = std::ldexp(nu, -s);
        for (int c = 1; c <= md; ++c)
            if (ctheta[c] >= x) {
                const int cost = taylor_products_host(c) + s;
                if (cost < bc) { bc = cost; bm = c; bs = s; }
                break;
            }
    }
    *m_out = bm;
    *s_out = bs;
}

using Mat = std::vector<cplx>;

Mat load_mat(const double* p, int64_t d) {
    Mat m(d * d);
    for (int64_t i = 0; i < d * d; ++i) m[i] = cplx(p[2 * i], p[2 * i + 1]);
    return m;
}

Mat matmul(const Mat& a, const Mat& b, int64_t d) {
    Mat c(d * d, cplx(0, 0));
    for (int64_t i = 0; i < d; ++i)
        for (int64_t k = 0; k < d; ++k) {
            const cplx aik = a[i * d + k];
            for (int64_t j = 0; j < d; ++j) c[i * d + j] += aik * b[k * d + j];
        }
    return c;
}

// i [A, B] = i (A B - B A): Hermitian when A and B are.
Mat icomm(const Mat& a, const Mat& b, int64_t d) {
    Mat ab = matmul(a, b, d), ba = matmul(b, a, d);
    Mat c(d * d);
    for (int64_t i = 0; i < d * d; ++i) c[i] = cplx(0, 1) * (ab[i] - ba[i]);
    return c;
}

bool hermitian_ok(const Mat& a, int64_t d, bool finite_only = false) {
    double mx = 0.0, dev = 0.0;
    for (int64_t i = 0; i < d; ++i)
        for (int64_t j = 0; j < d; ++j) {
            const cplx x = a[i * d + j];
            if (!std::isfinite(x.real()) || !std::isfinite(x.imag())) return false;
            mx = std::max(mx, std::abs(x));
            dev = std::max(dev, std::abs(x - std::conj(a[j * d + i])));
        }
    return finite_only || dev <= 1e-12 * std::max(1.0, mx);
}

void symmetrize(Mat& a, int64_t d) {
    for (int64_t i = 0; i < d; ++i) {
        a[i * d + i] = cplx(a[i * d + i].real(), 0.0);
        for (int64_t j = i + 1; j < d; ++j) {
            const cplx v = 0.5 * (a[i * d + j] + std::conj(a[j * d + i]));
            a[i * d + j] = v;
            a[j * d + i] = std::conj(v);
        }
    }
}

double norm1(const Mat& a, int64_t d) {
    double best = 0.0;
    for (int64_t j = 0; j < d; ++j) {
        double s = 0.0;
        for (int64_t i = 0; i < d; ++i) s += std::abs(a[i * d + j]);
        best = std::max(best, s);
    }
    return best;
}

// The ordered basis: H0, H_1..H_K [, i[H0,H_k] (k=1..K), i[H_k,H_k'] (k<k')].
pm_status build_basis(int64_t d, const double* H0, int64_t K, const double* Hk, int order,
                      std::vector<Mat>* out, std::vector<std::pair<int, int>>* pairs,
                      std::string* err) {
    std::vector<Mat> base;
    base.push_back(load_mat(H0, d));
    for (int64_t k = 0; k < K; ++k) base.push_back(load_mat(Hk + 2 * k * d * d, d));
    for (size_t i = 0; i < base.size(); ++i) {
        if (!hermitian_ok(base[i], d)) {
            *err = (i == 0 ? std::string("H0") : "H_" + std::to_string(i)) +
                   " is not Hermitian (or not finite)";
            return PM_E_NOT_HERMITIAN;
        }
        symmetrize(base[i], d);
    }
    *out = base;
    pairs->clear();
    if (order == 4) {
        for (int64_t k = 1; k <= K; ++k) {
            Mat c = icomm(base[0], base[k], d);
            symmetrize(c, d);
            out->push_back(c);
        }
        for (int64_t a = 1; a <= K; ++a)
            for (int64_t b = a + 1; b <= K; ++b) {
                Mat c = icomm(base[a], base[b], d);
                symmetrize(c, d);
                out->push_back(c);
                pairs->push_back({(int)a - 1, (int)b - 1});
            }
    }
    return PM_OK;
}

template <typename P>
void dfree(P*& p) {
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

pm_status ensure(pm_ctx* ctx, void** ptr, size_t* have, size_t need, const char* what,
                 bool zero = false) {
    if (need <= *have && *ptr) return PM_OK;
    if (*ptr) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(ctx, e, "hipDeviceSynchronize");
        (void)hipFree(*ptr);
        *ptr = nullptr;
        *have = 0;
    }
    need = std::max<size_t>(need, 256);
    hipError_t e = hipMalloc(ptr, need);
    if (e != hipSuccess) {
        *ptr = nullptr;
        (void)hipGetLastError();
        return fail(ctx, PM_E_OOM, std::string("hipMalloc failed for ") + what);
    }
    if (zero) {
        e = hipMemset(*ptr, 0, need);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipMemset");
        e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(ctx, e, "hipDeviceSynchronize");
    }
    *have = need;
    return PM_OK;
}

bool order_ok(int order) {
    return order == PM_ORDER_MIDPOINT || order == PM_ORDER_MAGNUS4 || order == PM_ORDER_CF4 ||
           order == PM_ORDER_MAGNUS6;
}

// Slices covered by n_samples samples (one per slice for the midpoint rule,
// three per slice for sixth order, 2N + 1 otherwise).
int64_t n_slices_of(int order, int64_t n_samples) {
    if (order == 2) return n_samples;
    if (order == PM_ORDER_MAGNUS6) return n_samples / 3;
    return (n_samples - 1) / 2;
}

// Exponentials the kernels evaluate: one per slice, two for CF4 (the
// factors of each slice in product order).
int64_t n_exps_of(int order, int64_t n_samples) {
    const int64_t N = n_slices_of(order, n_samples);
    return order == PM_ORDER_CF4 ? 2 * N : N;
}

// Sample counts the integrator accepts: N >= 1 (order 2), 2N + 1 (orders 4
// and CF4), 3N (order 6).
bool samples_ok(int order, int64_t n_samples) {
    if (order == 2) return n_samples >= 1;
    if (order == PM_ORDER_MAGNUS6) return n_samples >= 3 && n_samples % 3 == 0;
    return n_samples >= 3 && n_samples % 2 == 1;
}

pm_status check_prop_args(pm_ctx* ctx, int64_t n_samples, double dt) {
    if (!ctx) return PM_E_INVALID_ARG;
    if (ctx->broken) return fail(ctx, PM_E_DEVICE, "context unusable after a device error");
    if (!ctx->ready) return fail(ctx, PM_E_NOT_READY, "pm_set_hamiltonian has not been called");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ctx, PM_E_INVALID_ARG, "dt must be finite and > 0");
    if (!samples_ok(ctx->order, n_samples))
        return fail(ctx, PM_E_INVALID_ARG, ctx->order == 2 ? "order 2 needs n_samples >= 1" :
                    ctx->order == PM_ORDER_MAGNUS6 ? "order 6 needs n_samples = 3N, N >= 1" :
                    "orders 4 and CF4 need an odd n_samples >= 3");
    if (n_samples > (int64_t(1) << 40)) return fail(ctx, PM_E_INVALID_ARG, "n_samples too large");
    return PM_OK;
}

// Process-wide tuning table (pm_tuning_set): target chain counts of the
// automatic chunking per engine class and precision, and batch chain lengths.
int64_t g_tune_chains[5][4] = {};
int64_t g_tune_batch_chunk[3][4] = {};

int tune_class(int D) {
    switch (D) {
        case 2: return 0;
        case 4: return 1;
        case 16: return 2;
        case 32: return 3;
        case 64: return 4;
        default: return -1;
    }
}

// Chain length: about one chain per resident wave team (or the tuned count),
// in whole units.  The tuned counts are measured on propagations that return
// U(T) only; with per-slice output the two-dimensional VALU kernel keeps one
// chain per resident wave (two per SIMD): in FP32 at 2^26 slices 1.14 ms
// against 1.38 ms with the tuned 1024 chains (FP64 is tuned to the same count;
// for d=4 the tuned counts measured as fast or faster).
int64_t auto_chunk(const pm::EngineInfo& e, int64_t N, int precision, bool per_slice) {
    int64_t target = (int64_t)e.resident_chains;
    const int tc = tune_class(e.D);
    const bool tuned = !(per_slice && e.kind == pm::ENGINE_VALU && e.D == 2);
    if (tuned && tc >= 0 && precision >= 0 && precision < 4 && g_tune_chains[tc][precision] > 0)
        target = g_tune_chains[tc][precision];
    int64_t c = (N + target - 1) / target;
    if (c < 1) c = 1;
    // Short MFMA chains: below four slices the product tree's extra leaves
    // cost more than the parallelism gains.  Measured on the d=16 workload
    // (graph replay): N = 8192, chains of 4 (512 blocks, uneven chains) 52.7
    // us, of 8 53.9 us, of 2 75.1 us; N = 4096 gradient, chains of 4 beat 2
    // by 13 % and 8 by 30 %.
    const int64_t cmin = 4;
    if (e.kind == pm::ENGINE_MFMA && c < cmin) c = cmin;
    const int64_t u = e.chunk_unit;
    return ((c + u - 1) / u) * u;
}

// Chain length of a propagation: the user's, else the automatic one; whole
// units, and for the VALU engine at most 2^20 slices (its per-slice output
// addresses a chain's slices with 32-bit offsets).
int64_t effective_chunk(const pm_ctx* ctx, const pm::EngineInfo& e, int64_t N, bool per_slice = false) {
    if (ctx->call_chunk > 0) return ctx->call_chunk;
    int64_t c = ctx->chunk_override > 0 ? ctx->chunk_override
                                        : auto_chunk(e, N, ctx->precision, per_slice);
    c = ((c + e.chunk_unit - 1) / e.chunk_unit) * e.chunk_unit;
    if (e.kind == pm::ENGINE_VALU && c > (int64_t(1) << 20)) c = int64_t(1) << 20;
    // CF4: a chain starts at a slice boundary (an even exponential index)
    if (ctx->order == PM_ORDER_CF4 && (c & 1)) ++c;
    return c;
}

// Uneven chains for a D = 16 launch of exactly two blocks per CU.  A CU
// places the two blocks' waves two to a SIMD, and the SIMD's issue favours
// the older wave: the blocks dispatched first (one per CU, the lower block
// indices) finish their chains well before the second ones, which then run
// their last slices one wave per SIMD, too few to keep the MFMA pipe busy.
// Giving the first-dispatched blocks' chains `pct` percent more slices (the
// others correspondingly fewer) lets both finish together.  Measured on the
// d = 16 workload (graph replay, one box): N = 2^17 FP64 334 -> 321 us at 20 %
// and 317 us at 25 %; FP32-3M 249 -> 234 us at 20 %; N = 32768 FP64 117 ->
// 111 us at 25 %.  The product over the chains is unchanged (the tree still
// multiplies consecutive chains in order); only its association differs.
// The small-dimension engine's blocks of four one-chain waves meet the same
// arbitration at two blocks per CU; its chains stay in whole units (and at
// most 2^20 slices).  Measured there (d = 2, N = 2^26, FP64): 567 -> 546 us
// without and 1251 -> 1188 us with per-slice output at 25 %; in FP32 20 %
// gained nothing and 40 % lost 12 %, so its reduced modes keep equal chains.
void skew_chains(const pm_ctx* ctx, const pm::EngineInfo& e, pm::PropParams& p) {
    const bool valu = e.kind == pm::ENGINE_VALU;
    if (!valu && !(e.kind == pm::ENGINE_MFMA && e.D == 16)) return;
    const int pct = ctx->chain_skew >= 0 ? ctx->chain_skew : (ctx->precision == PM_FP64 ? 25 : (valu ? 0 : 20));
    if (pct <= 0 || p.n_leaves != 2 * (int64_t)ctx->n_cu) return;
    const bool even = ctx->order == PM_ORDER_CF4;   // chains start at a slice boundary
    const int64_t u = e.chunk_unit;
    auto whole = [&](int64_t c) {
        c = (c + u - 1) / u * u;
        return even && (c & 1) ? c + 1 : c;
    };
    const int64_t n_long = (int64_t)ctx->n_cu * e.chains_per_leaf;
    const int64_t cl = whole(p.chunk + (p.chunk * pct + 50) / 100);
    const int64_t rest = p.n_slices - n_long * cl, n_short = p.n_chains - n_long;
    if (cl <= p.chunk || n_short <= 0 || rest < n_short || (valu && cl > (int64_t(1) << 20))) return;
    const int64_t cs = whole((rest + n_short - 1) / n_short);
    if (cs >= p.chunk) return;
    p.n_long = n_long;
    p.chunk_long = cl;
    p.chunk = cs;
}

// ---- device workspace under the context's limit (pm_set_workspace_limit)

// Bytes ensure() allocates for a request.
size_t alloc_bytes(size_t need) { return std::max<size_t>(need, 256); }

// The context's device workspace for one call at chain length `chunk`:
// the product tree's nodes and tickets; for the checkpointed forward pass
// (gradient, trajectory) also U(T) and every chain product; for the
// gradient the weight gradients of every slice.
size_t call_bytes(const pm_ctx* ctx, const pm::EngineInfo& e, int64_t N, int64_t chunk, int kind) {
    const int64_t chains = (N + chunk - 1) / chunk;
    const int64_t leaves = (chains + e.chains_per_leaf - 1) / e.chains_per_leaf;
    const size_t node = (size_t)e.D * e.D * 16;
    size_t b = alloc_bytes(node * (size_t)(2 * leaves + 64)) + alloc_bytes(4 * (size_t)(2 * leaves + 64));
    if (kind != PM_WORK_PROPAGATE) b += 16 * PM_MAX_DIM * PM_MAX_DIM + alloc_bytes(node * (size_t)chains);
    if (kind == PM_WORK_GRADIENT) b += alloc_bytes(sizeof(double) * (size_t)N * ctx->M);
    return b;
}

// Chain length of a call of `kind` over N exponentials with `extra` bytes
// of other workspace: the automatic (or pm_set_chunk's) length, doubled
// while the call's workspace exceeds the limit -- longer chains mean fewer
// tree nodes and, for the gradient and the trajectory, checkpoints further
// apart with more recomputation between them.  PM_E_OOM when even one chain
// does not fit, or when the length fixed by pm_set_chunk does not.
pm_status plan_call(pm_ctx* ctx, const pm::EngineInfo& e, int64_t N, int kind, bool per_slice, size_t extra,
                    int64_t* chunk_out, size_t* bytes_out) {
    int64_t c = effective_chunk(ctx, e, N, per_slice);
    size_t b = call_bytes(ctx, e, N, c, kind) + extra;
    const size_t lim = (size_t)ctx->ws_limit;
    if (ctx->ws_limit > 0 && b > lim) {
        if (ctx->chunk_override > 0)
            return fail(ctx, PM_E_OOM, "the chain length set by pm_set_chunk needs " + std::to_string(b) +
                                           " bytes of device workspace, over the limit of " + std::to_string(lim));
        const int64_t u = e.chunk_unit;
        const int64_t cmax = e.kind == pm::ENGINE_VALU ? std::min<int64_t>(N, int64_t(1) << 20) : N;
        while (b > lim && c < cmax) {
            c = std::min<int64_t>(2 * c, ((cmax + u - 1) / u) * u);
            c = ((c + u - 1) / u) * u;
            if (e.kind == pm::ENGINE_VALU && c > (int64_t(1) << 20)) c = int64_t(1) << 20;
            if (ctx->order == PM_ORDER_CF4 && (c & 1)) ++c;
            b = call_bytes(ctx, e, N, c, kind) + extra;
        }
        if (b > lim)
            return fail(ctx, PM_E_OOM, "this call needs at least " + std::to_string(b) +
                                           " bytes of device workspace, over the limit of " + std::to_string(lim));
    }
    *chunk_out = c;
    if (bytes_out) *bytes_out = b;
    return PM_OK;
}

// Device workspace the context holds (every per-call buffer; not the basis
// or the Chebyshev table uploaded at set-up).
size_t held_workspace(const pm_ctx* c) {
    return c->nodes_bytes + c->counters_bytes + c->samples_bytes + c->u_bytes + c->slices_bytes + c->chain_bytes +
           c->gw_bytes + c->ut_bytes + c->w_bytes + c->grad_bytes + c->mom_bytes;
}

pm_status release_workspace(pm_ctx* c) {
    DeviceGuard g(c->device);
    const hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(c, e, "hipDeviceSynchronize");
    dfree(c->d_nodes);
    dfree(c->d_counters);
    dfree(c->d_samples);
    dfree(c->d_U);
    dfree(c->d_chain);
    dfree(c->d_gw);
    dfree(c->d_UT);
    dfree(c->d_W);
    dfree(c->d_grad);
    dfree(c->d_mom);
    if (c->d_slices) (void)hipFree(c->d_slices);
    c->d_slices = nullptr;
    c->nodes_bytes = c->counters_bytes = c->samples_bytes = c->u_bytes = c->slices_bytes = 0;
    c->chain_bytes = c->gw_bytes = c->ut_bytes = c->w_bytes = c->grad_bytes = c->mom_bytes = 0;
    return PM_OK;
}

// Before a call that needs `need` bytes: if what the context holds plus
// that could pass the limit, release the held buffers first, so the call
// allocates no more than its own need.
pm_status fit_workspace(pm_ctx* ctx, size_t need) {
    if (ctx->ws_limit <= 0 || held_workspace(ctx) + need <= (size_t)ctx->ws_limit) return PM_OK;
    return release_workspace(ctx);
}

// The planned chain length, in force for the duration of one entry point.
struct CallChunk {
    pm_ctx* c;
    CallChunk(pm_ctx* ctx, int64_t chunk) : c(ctx) { c->call_chunk = chunk; }
    ~CallChunk() { c->call_chunk = 0; }
};

// Plan, fit and fix the chain length of one call.
pm_status begin_call(pm_ctx* ctx, const pm::EngineInfo& e, int64_t n_samples, int kind, bool per_slice,
                     size_t extra, int64_t* chunk) {
    size_t need = 0;
    pm_status s = plan_call(ctx, e, n_exps_of(ctx->order, n_samples), kind, per_slice, extra, chunk, &need);
    if (s != PM_OK) return s;
    return fit_workspace(ctx, need);
}

// Workspace and kernel parameters of one propagation on engine e.
// A caller-provided device workspace for the tree's tickets and nodes
// (the entry point that allocates nothing): tickets first, 256-byte aligned,
// then the nodes.
struct FixedWorkspace {
    void* base;
    size_t bytes;
};

size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }

pm_status prepare(pm_ctx* ctx, const pm::EngineInfo& e, bool keep_nodes, const double* basis, const double* d_samples,
                  int64_t n_samples, double dt, double* d_U, void* d_slices, pm::PropParams* out,
                  const FixedWorkspace* fixed = nullptr) {
    const int64_t N = n_exps_of(ctx->order, n_samples);
    const int64_t chunk = effective_chunk(ctx, e, N, d_slices != nullptr);
    const int64_t chains = (N + chunk - 1) / chunk;
    const int64_t leaves = (chains + e.chains_per_leaf - 1) / e.chains_per_leaf;
    const size_t node_bytes = (size_t)e.D * e.D * 16;
    const size_t nodes_need = node_bytes * (size_t)(2 * leaves + 64);
    const size_t tickets_need = sizeof(unsigned) * (size_t)(2 * leaves + 64);
    double* nodes;
    unsigned* tickets;
    if (fixed) {
        const size_t need = round256(tickets_need) + nodes_need;
        if (need > fixed->bytes)
            return fail(ctx, PM_E_INVALID_ARG,
                        "this propagation needs " + std::to_string(need) + " bytes of tree workspace (" +
                            std::to_string(leaves) + " leaves); the fixed workspace holds " +
                            std::to_string(fixed->bytes) + " (use longer chains: pm_set_chunk)");
        tickets = static_cast<unsigned*>(fixed->base);
        nodes = reinterpret_cast<double*>(static_cast<char*>(fixed->base) + round256(tickets_need));
    } else {
        pm_status st = ensure(ctx, (void**)&ctx->d_nodes, &ctx->nodes_bytes, nodes_need, "tree nodes");
        if (st != PM_OK) return st;
        st = ensure(ctx, (void**)&ctx->d_counters, &ctx->counters_bytes, tickets_need, "tree tickets", true);
        if (st != PM_OK) return st;
        nodes = ctx->d_nodes;
        tickets = ctx->d_counters;
    }

    pm::PropParams& p = *out;
    std::memset(&p, 0, sizeof(p));
    p.basis = basis;
    p.samples = d_samples;
    p.n_samples = n_samples;
    p.n_slices = N;
    p.chunk = chunk;
    p.chunk_long = chunk;
    p.n_long = 0;
    p.n_chains = chains;
    p.n_leaves = leaves;
    if (!keep_nodes) skew_chains(ctx, e, p);
    p.slices_out = d_slices;
    p.nodes = nodes;
    p.counters = tickets;
    p.U_out = d_U;
    p.h = dt;
    if (ctx->theta_n != N) {
        fill_theta(ctx->theta, ctx->precision, N);
        ctx->theta_n = N;
    }
    std::memcpy(p.theta, ctx->theta, sizeof(p.theta));
    p.K = (int)ctx->n_ctrl;
    p.M = ctx->M;
    p.order = ctx->order;
    p.du = (int)ctx->dim;
    p.max_degree = ctx->max_degree;
    p.force_s = ctx->force_s;
    p.method = ctx->method;
    p.cheb_j = ctx->d_cheb;
    if (ctx->method == PM_EXPM_CHEBYSHEV) {
        const double u = unit_roundoff(ctx->precision);
        p.ctheta[0] = 0.0;
        for (int m = 1; m <= pm::kMaxCheb; ++m) p.ctheta[m] = chebyshev_theta(m, u);
    }
    // D = 16: the block keeps the basis in LDS when it is small (<= 64 KiB)
    p.basis_lds = (e.kind == pm::ENGINE_MFMA && e.D == 16 &&
                   (size_t)ctx->M * e.D * e.D * 16 <= 64 * 1024) ? 1 : 0;
    // two slices per tile for Taylor propagations of dimension <= 8 (also
    // the checkpointed forward pass: its chain products and tree nodes come
    // out in the unpaired layout)
    if (ctx->d_basis_pair && basis == ctx->d_basis && (ctx->method == PM_EXPM_TAYLOR || keep_nodes) &&
        e.kind == pm::ENGINE_MFMA && e.D == 16) {
        p.pair = 1;
        p.basis = ctx->d_basis_pair;
    }
    std::memcpy(p.pair_a, ctx->pair_a, sizeof(p.pair_a));
    std::memcpy(p.pair_b, ctx->pair_b, sizeof(p.pair_b));
    return PM_OK;
}

pm_status launch(pm_ctx* ctx, const double* d_samples, int64_t n_samples, double dt, double* d_U,
                 void* d_slices, hipStream_t stream) {
    pm::PropParams p;
    pm_status st = prepare(ctx, ctx->eng, false, ctx->d_basis, d_samples, n_samples, dt, d_U, d_slices, &p);
    if (st != PM_OK) return st;
    hipError_t he = pm::launch_propagate(ctx->eng, ctx->precision, p, stream);
    if (he != hipSuccess) return hip_fail(ctx, he, "kernel launch");
    return PM_OK;
}

// Gradient: forward on the FP64 MFMA engine keeping chain products and every
// tree node (U(T) into ctx->d_UT), then the backward kernels.
// Forward pass on the FP64 gradient engine that keeps every tree node and
// chain product (the checkpoints of the gradient and the trajectory).
// U(T) goes to d_U when given (the caller's device buffer, dim x dim), else
// to the context's buffer; p.U_out says where.
pm_status forward_keep(pm_ctx* ctx, const double* d_samples, int64_t n_samples, double dt, hipStream_t stream,
                       bool run_forward, pm::PropParams* out, double* d_U = nullptr) {
    const pm::EngineInfo& e = ctx->geng;
    const double* basis = ctx->d_basis_grad ? ctx->d_basis_grad : ctx->d_basis;
    pm::PropParams& p = *out;
    pm_status st = ensure(ctx, (void**)&ctx->d_UT, &ctx->ut_bytes, 16 * PM_MAX_DIM * PM_MAX_DIM, "U(T)");
    if (st != PM_OK) return st;
    st = prepare(ctx, e, true, basis, d_samples, n_samples, dt, d_U ? d_U : ctx->d_UT, nullptr, &p);
    if (st != PM_OK) return st;
    p.method = PM_EXPM_TAYLOR;   // the adjoint and the trajectory use the Taylor evaluation
    st = ensure(ctx, (void**)&ctx->d_chain, &ctx->chain_bytes, (size_t)p.n_chains * e.D * e.D * 16,
                "chain products");
    if (st != PM_OK) return st;
    p.chain_out = ctx->d_chain;
    p.store_nodes = 1;
    if (run_forward) {
        const hipError_t he = pm::launch_propagate(e, PM_FP64, p, stream);
        if (he != hipSuccess) return hip_fail(ctx, he, "forward launch");
    }
    // the backward and trajectory kernels recompute single slices
    p.pair = 0;
    p.basis = basis;
    return PM_OK;
}

pm_status launch_grad(pm_ctx* ctx, const double* d_samples, int64_t n_samples, double dt,
                      const double* d_W, double* d_grad, hipStream_t stream, bool run_forward,
                      bool run_backward, double* d_U = nullptr) {
    const pm::EngineInfo& e = ctx->geng;
    pm::PropParams p;
    pm_status st = forward_keep(ctx, d_samples, n_samples, dt, stream, run_forward, &p, d_U);
    if (st != PM_OK) return st;
    hipError_t he;
    if (!run_backward) return PM_OK;
    st = ensure(ctx, (void**)&ctx->d_gw, &ctx->gw_bytes, sizeof(double) * (size_t)p.n_slices * p.M,
                "weight gradients");
    if (st != PM_OK) return st;
    pm::GradParams gp;
    gp.p = p;
    gp.W = d_W;
    gp.UT = p.U_out;   // where the forward left U(T)
    gp.gw = ctx->d_gw;
    // few long chains: split each into parts of at least four slices (each
    // part recomputes its predecessors in the chain) until about 2048 waves
    // run (D = 16: two waves per unit); shorter parts lose more to the
    // recomputation than they gain
    gp.split = 1;
    gp.grad_direct = nullptr;
    const int64_t max_units = e.D == 16 ? 1024 : 2048;
    while (p.n_chains * gp.split * 2 <= max_units && p.chunk >= 8 * gp.split) gp.split *= 2;
    he = pm::launch_backward(e.D, gp, d_grad, stream);
    if (he != hipSuccess) return hip_fail(ctx, he, "backward launch");
    return PM_OK;
}

}  // namespace

namespace pm {

bool pick_engine(int du, int precision, EngineInfo* out) {
    if (du < 1 || du > PM_MAX_DIM) return false;
    if (unit_roundoff(precision) < 0) return false;
    EngineInfo e{};
    if (du <= 4) {
        e.kind = ENGINE_VALU;
        e.D = du <= 2 ? 2 : 4;
        e.chunk_unit = 1024;        // a run of a multiple of 16 slices per lane (two sample blocks)
        e.chains_per_leaf = 4;      // a block of four waves is a leaf
        e.resident_chains = 256 * 8;
    } else {
        e.kind = ENGINE_MFMA;
        e.D = du <= 16 ? 16 : (du <= 32 ? 32 : 64);
        e.chunk_unit = 1;
        e.chains_per_leaf = mfma_chains_per_block(e.D);   // a block is a leaf
        e.resident_chains = e.D == 16 ? 256 * 8 : (e.D == 32 ? 256 * 4 : 256);
        e.f64_rows = precision == PM_FP64 ? 1 : 0;
    }
    *out = e;
    return true;
}

int64_t basis_layout_doubles(const EngineInfo& e, int M) {
    return (int64_t)M * e.D * e.D * 2;
}

void basis_to_layout(const EngineInfo& e, int M, int du, const double* basis, double* dst) {
    const int D = e.D;
    std::memset(dst, 0, sizeof(double) * basis_layout_doubles(e, M));
    for (int m = 0; m < M; ++m) {
        const double* b = basis + (int64_t)m * du * du * 2;
        for (int r = 0; r < du; ++r)
            for (int c = 0; c < du; ++c) {
                const double re = b[(r * du + c) * 2], im = b[(r * du + c) * 2 + 1];
                if (e.kind == ENGINE_VALU) {
                    dst[((int64_t)m * D * D + r * D + c) * 2 + 0] = re;
                    dst[((int64_t)m * D * D + r * D + c) * 2 + 1] = im;
                } else {
                    const int TI = r / 16, TJ = c / 16, rr = r % 16, cc = c % 16;
                    const int g = e.f64_rows ? rr % 4 : rr / 4;
                    const int ri = e.f64_rows ? rr / 4 : rr % 4;
                    const int lane = 16 * g + cc;
                    dst[mfma_basis_index(D, m, TI, TJ, 0, ri, lane)] = re;
                    dst[mfma_basis_index(D, m, TI, TJ, 1, ri, lane)] = im;
                }
            }
    }
}

hipError_t launch_propagate(const EngineInfo& e, int precision, const PropParams& p,
                            hipStream_t stream) {
    if (e.kind == ENGINE_VALU) return launch_valu(e.D, precision == PM_FP64, p, stream);
    return launch_mfma(e.D, precision, p, stream);
}

}  // namespace pm

// ------------------------------------------------------------------ C ABI

extern "C" {

const char* pm_status_string(pm_status s) {
    switch (s) {
        case PM_OK: return "PM_OK";
        case PM_E_INVALID_ARG: return "PM_E_INVALID_ARG";
        case PM_E_NOT_READY: return "PM_E_NOT_READY";
        case PM_E_NOT_HERMITIAN: return "PM_E_NOT_HERMITIAN";
        case PM_E_OOM: return "PM_E_OOM";
        case PM_E_DEVICE: return "PM_E_DEVICE";
        case PM_E_UNSUPPORTED: return "PM_E_UNSUPPORTED";
    }
    return "PM_E_UNKNOWN";
}

const char* pm_last_error(const pm_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

int64_t pm_basis_count(int64_t n_ctrl, int order) {
    if (n_ctrl < 0 || n_ctrl > pm::kMaxCtrl) return -1;
    if (order == 2 || order == PM_ORDER_CF4 || order == PM_ORDER_MAGNUS6) return 1 + n_ctrl;
    if (order == 4) return 1 + 2 * n_ctrl + n_ctrl * (n_ctrl - 1) / 2;
    return -1;
}

pm_status pm_taylor_theta(int m, int precision, int64_t n_slices, double* theta_out) {
    if (m < 1 || m > PM_MAX_TAYLOR_DEGREE || !theta_out || n_slices < 1) return PM_E_INVALID_ARG;
    if (unit_roundoff(precision) < 0) return PM_E_INVALID_ARG;
    *theta_out = taylor_theta(m, truncation_target(precision, n_slices), relative_truncation(precision));
    return PM_OK;
}

pm_status pm_chebyshev_theta(int m, int precision, double* theta_out) {
    if (m < 1 || m > PM_MAX_CHEBYSHEV_DEGREE || !theta_out || unit_roundoff(precision) < 0)
        return PM_E_INVALID_ARG;
    *theta_out = chebyshev_theta(m, unit_roundoff(precision));
    return PM_OK;
}

pm_status pm_plan_chebyshev(double nu, int precision, int max_degree, int force_s, int* m_out, int* s_out) {
    if (!m_out || !s_out || !(nu >= 0.0) || max_degree < 1 || max_degree > PM_MAX_CHEBYSHEV_DEGREE ||
        force_s < -1 || force_s > 62 || unit_roundoff(precision) < 0)
        return PM_E_INVALID_ARG;
    double ct[pm::kMaxCheb + 1];
    ct[0] = 0.0;
    for (int m = 1; m <= pm::kMaxCheb; ++m) ct[m] = chebyshev_theta(m, unit_roundoff(precision));
    plan_chebyshev_host(ct, max_degree, force_s, nu, m_out, s_out);
    return PM_OK;
}

pm_status pm_plan_expm(double nu, int precision, int max_degree, int64_t n_slices, int* m_out,
                       int* s_out) {
    if (!m_out || !s_out || !(nu >= 0.0) || max_degree < 1 || max_degree > PM_MAX_TAYLOR_DEGREE ||
        n_slices < 1)
        return PM_E_INVALID_ARG;
    if (unit_roundoff(precision) < 0) return PM_E_INVALID_ARG;
    double th[pm::kMaxDeg + 1];
    fill_theta(th, precision, n_slices);
    plan_host(th, max_degree, -1, nu, m_out, s_out);
    return PM_OK;
}

pm_status pm_build_basis_host(int64_t dim, const double* H0, int64_t n_ctrl, const double* Hk,
                              int order, double* basis_out, double* norms_out) {
    if (dim < 1 || dim > PM_MAX_DIM || !H0 || n_ctrl < 0 || n_ctrl > pm::kMaxCtrl ||
        (n_ctrl > 0 && !Hk) || !order_ok(order))
        return PM_E_INVALID_ARG;
    std::vector<Mat> basis;
    std::vector<std::pair<int, int>> pairs;
    std::string err;
    pm_status s = build_basis(dim, H0, n_ctrl, Hk, order, &basis, &pairs, &err);
    if (s != PM_OK) return s;
    for (size_t m = 0; m < basis.size(); ++m) {
        if (basis_out)
            for (int64_t i = 0; i < dim * dim; ++i) {
                basis_out[(m * dim * dim + i) * 2 + 0] = basis[m][i].real();
                basis_out[(m * dim * dim + i) * 2 + 1] = basis[m][i].imag();
            }
        if (norms_out) norms_out[m] = norm1(basis[m], dim);
    }
    return PM_OK;
}

pm_status pm_slice_weights_host(int64_t n_ctrl, const double* samples, int64_t n_samples,
                                double dt, int order, int64_t slice, double* weights_out) {
    if (n_ctrl < 0 || n_ctrl > pm::kMaxCtrl || (n_ctrl > 0 && !samples) || !weights_out ||
        !order_ok(order))
        return PM_E_INVALID_ARG;
    if (!samples_ok(order, n_samples)) return PM_E_INVALID_ARG;
    const int64_t N = n_exps_of(order, n_samples);
    if (slice < 0 || slice >= N) return PM_E_INVALID_ARG;
    const int64_t K = n_ctrl, S = n_samples;
    const double h = dt;
    int64_t m = 0;
    if (order == PM_ORDER_MAGNUS6) {
        // the three moments P1, P2, P3 on {H0, H_k}
        const double r15 = std::sqrt(15.0);
        weights_out[m++] = h;
        for (int64_t k = 0; k < K; ++k) weights_out[m++] = h * samples[k * S + 3 * slice + 1];
        weights_out[m++] = 0.0;
        for (int64_t k = 0; k < K; ++k) {
            const double* c = samples + k * S + 3 * slice;
            weights_out[m++] = (r15 * h / 3.0) * (c[2] - c[0]);
        }
        weights_out[m++] = 0.0;
        for (int64_t k = 0; k < K; ++k) {
            const double* c = samples + k * S + 3 * slice;
            weights_out[m++] = (10.0 * h / 3.0) * ((c[2] - 2.0 * c[1]) + c[0]);
        }
        return PM_OK;
    }
    if (order == PM_ORDER_CF4) {
        // factor f of slice j: (h/12)(3 s0 + 4 s1 - s2), mirrored for f = 1
        const int64_t j = slice >> 1;
        const bool second = (slice & 1) != 0;
        weights_out[m++] = 0.5 * h;
        for (int64_t k = 0; k < K; ++k) {
            const double* c = samples + k * S + 2 * j;
            const double a = second ? c[2] : c[0], b = second ? c[0] : c[2];
            weights_out[m++] = (h / 12.0) * (3.0 * a + 4.0 * c[1] - b);
        }
        return PM_OK;
    }
    weights_out[m++] = h;
    if (order == 2) {
        for (int64_t k = 0; k < K; ++k) weights_out[m++] = h * samples[k * S + slice];
        return PM_OK;
    }
    auto s = [&](int64_t k, int i) { return samples[k * S + 2 * slice + i]; };
    for (int64_t k = 0; k < K; ++k) weights_out[m++] = (h / 6.0) * (s(k, 0) + 4.0 * s(k, 1) + s(k, 2));
    const double h2 = h * h / 12.0;
    for (int64_t k = 0; k < K; ++k) weights_out[m++] = h2 * (s(k, 2) - s(k, 0));
    for (int64_t a = 0; a < K; ++a)
        for (int64_t b = a + 1; b < K; ++b) weights_out[m++] = h2 * (s(a, 0) * s(b, 2) - s(a, 2) * s(b, 0));
    return PM_OK;
}

pm_status pm_create(pm_ctx** out, int device, int precision) {
    if (!out) return PM_E_INVALID_ARG;
    *out = nullptr;
    g_create_err.clear();
    if (unit_roundoff(precision) < 0) return create_fail(PM_E_INVALID_ARG, "unknown precision");
    int n = 0;
    const hipError_t de = hipGetDeviceCount(&n);
    if (de != hipSuccess || n <= 0) return create_fail(PM_E_DEVICE, "no HIP device", de);
    if (device < 0 || device >= n) return PM_E_INVALID_ARG;
    pm_ctx* ctx = new (std::nothrow) pm_ctx();
    if (!ctx) return PM_E_OOM;
    ctx->device = device;
    ctx->precision = precision;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        ctx->n_cu = cus;
    *out = ctx;
    return PM_OK;
}

pm_status pm_destroy(pm_ctx* ctx) {
    if (!ctx) return PM_OK;
    {
        DeviceGuard g(ctx->device);
        (void)hipDeviceSynchronize();
        dfree(ctx->d_basis);
        dfree(ctx->d_nodes);
        dfree(ctx->d_counters);
        dfree(ctx->d_samples);
        dfree(ctx->d_U);
        dfree(ctx->d_basis_grad);
        dfree(ctx->d_basis_pair);
        dfree(ctx->d_cheb);
        dfree(ctx->d_mom);
        dfree(ctx->d_chain);
        dfree(ctx->d_gw);
        dfree(ctx->d_UT);
        dfree(ctx->d_W);
        dfree(ctx->d_grad);
        if (ctx->d_slices) (void)hipFree(ctx->d_slices);
        ctx->d_slices = nullptr;
    }
    delete ctx;
    return PM_OK;
}

pm_status pm_set_expm_policy(pm_ctx* ctx, int max_taylor_degree, int force_s) {
    if (!ctx) return PM_E_INVALID_ARG;
    if (max_taylor_degree < 1 || max_taylor_degree > PM_MAX_TAYLOR_DEGREE || force_s < -1 || force_s > 62)
        return fail(ctx, PM_E_INVALID_ARG, "max_taylor_degree in [1, 21], force_s in [-1, 62]");
    ctx->max_degree = max_taylor_degree;
    ctx->force_s = force_s;
    return PM_OK;
}

pm_status pm_set_chain_skew(pm_ctx* ctx, int percent) {
    if (!ctx || percent < -1 || percent > 100)
        return ctx ? fail(ctx, PM_E_INVALID_ARG, "chain skew must be -1 (automatic) or 0..100") : PM_E_INVALID_ARG;
    ctx->chain_skew = percent;
    return PM_OK;
}

pm_status pm_set_chunk(pm_ctx* ctx, int64_t chunk) {
    if (!ctx || chunk < 0) return ctx ? fail(ctx, PM_E_INVALID_ARG, "chunk must be >= 0") : PM_E_INVALID_ARG;
    ctx->chunk_override = chunk;
    return PM_OK;
}

pm_status pm_set_workspace_limit(pm_ctx* ctx, int64_t bytes) {
    if (!ctx) return PM_E_INVALID_ARG;
    if (bytes < 0) return fail(ctx, PM_E_INVALID_ARG, "the workspace limit must be >= 0");
    ctx->ws_limit = bytes;
    if (bytes > 0 && held_workspace(ctx) > (size_t)bytes) return release_workspace(ctx);
    return PM_OK;
}

int64_t pm_workspace_held(const pm_ctx* ctx) { return ctx ? (int64_t)held_workspace(ctx) : -1; }

pm_status pm_workspace_plan(int64_t dim, int64_t n_ctrl, int order, int precision, int64_t n_samples, int kind,
                            int64_t limit, int64_t* chunk_out, int64_t* bytes_out) {
    if (dim < 1 || dim > PM_MAX_DIM || n_ctrl < 0 || n_ctrl > pm::kMaxCtrl || !order_ok(order) || limit < 0 ||
        !chunk_out || !samples_ok(order, n_samples) || unit_roundoff(precision) < 0 ||
        (kind != PM_WORK_PROPAGATE && kind != PM_WORK_GRADIENT && kind != PM_WORK_TRAJECTORY))
        return PM_E_INVALID_ARG;
    if ((order == PM_ORDER_MAGNUS6 || kind != PM_WORK_PROPAGATE) && precision != PM_FP64) return PM_E_UNSUPPORTED;
    if (order == PM_ORDER_MAGNUS6 && kind != PM_WORK_PROPAGATE) return PM_E_UNSUPPORTED;
    // a context as pm_set_hamiltonian would leave it, without the device
    pm_ctx c;
    c.precision = precision;
    c.dim = dim;
    c.n_ctrl = n_ctrl;
    c.order = order;
    c.M = (int)pm_basis_count(n_ctrl, order);
    c.ws_limit = limit;
    const int edim = order == PM_ORDER_MAGNUS6 && dim <= 4 ? 16 : (int)dim;
    if (!pm::pick_engine(edim, precision, &c.eng) || !pm::pick_engine(dim <= 16 ? 16 : (int)dim, PM_FP64, &c.geng))
        return PM_E_UNSUPPORTED;
    const pm::EngineInfo& e = kind == PM_WORK_PROPAGATE ? c.eng : c.geng;
    size_t b = 0;
    const pm_status s = plan_call(&c, e, n_exps_of(order, n_samples), kind, false, 0, chunk_out, &b);
    if (s != PM_OK) return s;
    if (bytes_out) *bytes_out = (int64_t)b;
    return PM_OK;
}

pm_status pm_set_expm_method(pm_ctx* ctx, int method) {
    if (!ctx) return PM_E_INVALID_ARG;
    if (method != PM_EXPM_TAYLOR && method != PM_EXPM_CHEBYSHEV)
        return fail(ctx, PM_E_INVALID_ARG, "unknown expm method");
    if (method == PM_EXPM_CHEBYSHEV && ctx->precision != PM_FP64)
        return fail(ctx, PM_E_UNSUPPORTED, "the Chebyshev series is built for PM_FP64 contexts only");
    if (method == PM_EXPM_CHEBYSHEV && !ctx->d_cheb) {
        // coefficient table J_k(theta_m), k <= m, for every degree m; then
        // the even/odd split of each degree's series (the tile engines):
        // even e_0 = J_0, e_i = 2 (-1)^i J_2i, i <= m/2; odd, with
        // o_j = 2 (-1)^j J_{2j+1} (j <= (m-1)/2) and the suffix sums
        // s_i = o_i - s_{i+1}: b_0 = s_0, b_i = 2 s_i
        const double u = unit_roundoff(ctx->precision);
        constexpr int H = pm::kChebHalf;
        std::vector<double> tab((size_t)pm::kChebSplitOffset + (size_t)(pm::kMaxCheb + 1) * 2 * H, 0.0);
        for (int m = 1; m <= pm::kMaxCheb; ++m) {
            const double th = chebyshev_theta(m, u);
            double J[pm::kMaxCheb + 1];
            for (int k = 0; k <= m; ++k) {
                J[k] = std::cyl_bessel_j((double)k, th);
                tab[(size_t)m * (pm::kMaxCheb + 1) + k] = J[k];
            }
            double* e = tab.data() + pm::kChebSplitOffset + (size_t)m * 2 * H;
            double* b = e + H;
            for (int i = 0; 2 * i <= m; ++i) e[i] = i == 0 ? J[0] : 2.0 * ((i & 1) ? -1.0 : 1.0) * J[2 * i];
            const int qs = (m - 1) / 2;
            double suf = 0.0;
            for (int i = qs; i >= 0; --i) {
                suf = 2.0 * ((i & 1) ? -1.0 : 1.0) * J[2 * i + 1] - suf;
                b[i] = i == 0 ? suf : 2.0 * suf;
            }
        }
        DeviceGuard g(ctx->device);
        void* ptr = nullptr;
        hipError_t e = hipMalloc(&ptr, tab.size() * sizeof(double));
        if (e != hipSuccess) return hip_fail(ctx, e, "Chebyshev table");
        e = hipMemcpy(ptr, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(ptr);
            return hip_fail(ctx, e, "Chebyshev table upload");
        }
        ctx->d_cheb = static_cast<double*>(ptr);
    }
    ctx->method = method;
    return PM_OK;
}

pm_status pm_launch_shape(pm_ctx* ctx, int64_t n_samples, int64_t* chunk, int64_t* chains,
                          int64_t* leaves) {
    if (!ctx || !chunk || !chains || !leaves) return ctx ? fail(ctx, PM_E_INVALID_ARG, "null output") : PM_E_INVALID_ARG;
    if (ctx->dim == 0) return fail(ctx, PM_E_NOT_READY, "pm_set_hamiltonian has not been called");
    const int64_t N = n_exps_of(ctx->order, n_samples);
    if (N < 1 || !samples_ok(ctx->order, n_samples))
        return fail(ctx, PM_E_INVALID_ARG, "bad n_samples for the integrator order");
    int64_t c = 0;
    const pm_status s = plan_call(ctx, ctx->eng, N, PM_WORK_PROPAGATE, false, 0, &c, nullptr);
    if (s != PM_OK) return s;
    *chunk = c;
    *chains = (N + c - 1) / c;
    *leaves = (*chains + ctx->eng.chains_per_leaf - 1) / ctx->eng.chains_per_leaf;
    return PM_OK;
}

pm_status pm_set_hamiltonian(pm_ctx* ctx, int64_t dim, const double* H0, int64_t n_ctrl,
                             const double* Hk, int order) {
    if (!ctx) return PM_E_INVALID_ARG;
    if (ctx->broken) return fail(ctx, PM_E_DEVICE, "context unusable after a device error");
    if (dim < 1 || dim > PM_MAX_DIM) return fail(ctx, PM_E_INVALID_ARG, "dim must be in [1, 64]");
    if (n_ctrl < 0 || n_ctrl > pm::kMaxCtrl) return fail(ctx, PM_E_INVALID_ARG, "n_ctrl must be in [0, 8]");
    if (!order_ok(order))
        return fail(ctx, PM_E_INVALID_ARG, "order must be 2, 4, PM_ORDER_CF4 or PM_ORDER_MAGNUS6");
    if (order == PM_ORDER_MAGNUS6 && ctx->precision != PM_FP64)
        return fail(ctx, PM_E_UNSUPPORTED, "the sixth-order integrator runs in PM_FP64 contexts only");
    if (!H0 || (n_ctrl > 0 && !Hk)) return fail(ctx, PM_E_INVALID_ARG, "null Hamiltonian pointer");
    pm::EngineInfo e;
    // the sixth-order exponent is formed by tile products: dimensions <= 4
    // embed in the 16-wide MFMA engine
    const int edim = order == PM_ORDER_MAGNUS6 && dim <= 4 ? 16 : (int)dim;
    if (!pm::pick_engine(edim, ctx->precision, &e))
        return fail(ctx, PM_E_UNSUPPORTED, "no engine for this dimension / precision");
    std::vector<Mat> basis;
    std::vector<std::pair<int, int>> pairs;
    std::string err;
    pm_status s = build_basis(dim, H0, n_ctrl, Hk, order, &basis, &pairs, &err);
    if (s != PM_OK) return fail(ctx, s, err);
    const int M = (int)basis.size();
    std::vector<double> flat((size_t)M * dim * dim * 2), norms(M);
    for (int m = 0; m < M; ++m) {
        for (int64_t i = 0; i < dim * dim; ++i) {
            flat[((size_t)m * dim * dim + i) * 2 + 0] = basis[m][i].real();
            flat[((size_t)m * dim * dim + i) * 2 + 1] = basis[m][i].imag();
        }
        norms[m] = norm1(basis[m], dim);
    }
    std::vector<double> lay((size_t)pm::basis_layout_doubles(e, M));
    pm::basis_to_layout(e, M, (int)dim, flat.data(), lay.data());

    DeviceGuard g(ctx->device);
    if (!g.ok) return hip_fail(ctx, hipErrorInvalidDevice, "hipSetDevice");
    hipError_t he = hipDeviceSynchronize();
    if (he != hipSuccess) return hip_fail(ctx, he, "hipDeviceSynchronize");
    dfree(ctx->d_basis);
    he = hipMalloc((void**)&ctx->d_basis, lay.size() * sizeof(double));
    if (he != hipSuccess) {
        ctx->d_basis = nullptr;
        (void)hipGetLastError();
        ctx->ready = false;
        return fail(ctx, PM_E_OOM, "hipMalloc failed for the basis");
    }
    he = hipMemcpy(ctx->d_basis, lay.data(), lay.size() * sizeof(double), hipMemcpyHostToDevice);
    if (he != hipSuccess) return hip_fail(ctx, he, "hipMemcpy basis");
    // the gradient runs on the FP64 MFMA engine; d <= 4 gets its own
    // embedded basis there
    dfree(ctx->d_basis_grad);
    if (ctx->precision == PM_FP64) {
        pm::EngineInfo ge;
        pm::pick_engine(dim <= 16 ? 16 : (int)dim, PM_FP64, &ge);
        ctx->geng = ge;
        if (e.kind != pm::ENGINE_MFMA) {
            std::vector<double> glay((size_t)pm::basis_layout_doubles(ge, M));
            pm::basis_to_layout(ge, M, (int)dim, flat.data(), glay.data());
            he = hipMalloc((void**)&ctx->d_basis_grad, glay.size() * sizeof(double));
            if (he != hipSuccess) {
                ctx->d_basis_grad = nullptr;
                (void)hipGetLastError();
                ctx->ready = false;
                return fail(ctx, PM_E_OOM, "hipMalloc failed for the gradient basis");
            }
            he = hipMemcpy(ctx->d_basis_grad, glay.data(), glay.size() * sizeof(double), hipMemcpyHostToDevice);
            if (he != hipSuccess) return hip_fail(ctx, he, "hipMemcpy gradient basis");
        }
    }
    // slice pairs: the basis in both diagonal 8 x 8 blocks of the 16-wide
    // tile, for dimensions <= 8 and at most 32 basis matrices
    dfree(ctx->d_basis_pair);
    if (e.kind == pm::ENGINE_MFMA && e.D == 16 && dim <= 8 && M <= 32 && order != PM_ORDER_MAGNUS6) {
        std::vector<double> dual((size_t)M * 16 * 16 * 2, 0.0);
        for (int m = 0; m < M; ++m)
            for (int64_t r = 0; r < dim; ++r)
                for (int64_t c = 0; c < dim; ++c)
                    for (int half = 0; half < 2; ++half) {
                        const size_t at = (((size_t)m * 16 + r + 8 * half) * 16 + c + 8 * half) * 2;
                        dual[at + 0] = flat[((size_t)m * dim * dim + r * dim + c) * 2 + 0];
                        dual[at + 1] = flat[((size_t)m * dim * dim + r * dim + c) * 2 + 1];
                    }
        std::vector<double> play((size_t)pm::basis_layout_doubles(e, M));
        pm::basis_to_layout(e, M, 16, dual.data(), play.data());
        he = hipMalloc((void**)&ctx->d_basis_pair, play.size() * sizeof(double));
        if (he != hipSuccess) {
            ctx->d_basis_pair = nullptr;
            (void)hipGetLastError();
            ctx->ready = false;
            return fail(ctx, PM_E_OOM, "hipMalloc failed for the slice-pair basis");
        }
        he = hipMemcpy(ctx->d_basis_pair, play.data(), play.size() * sizeof(double), hipMemcpyHostToDevice);
        if (he != hipSuccess) return hip_fail(ctx, he, "hipMemcpy slice-pair basis");
    }
    ctx->dim = dim;
    ctx->n_ctrl = n_ctrl;
    ctx->order = order;
    ctx->M = M;
    ctx->eng = e;
    ctx->basis = flat;
    ctx->norms = norms;
    std::memset(ctx->pair_a, 0, sizeof(ctx->pair_a));
    std::memset(ctx->pair_b, 0, sizeof(ctx->pair_b));
    for (size_t q = 0; q < pairs.size(); ++q) {
        const int m = 1 + 2 * (int)n_ctrl + (int)q;
        ctx->pair_a[m] = (uint8_t)pairs[q].first;
        ctx->pair_b[m] = (uint8_t)pairs[q].second;
    }
    ctx->ready = true;
    ctx->err.clear();
    return PM_OK;
}

pm_status pm_equiprop_dev(pm_ctx* ctx, const double* samples_dev, int64_t n_samples, double dt,
                          double* U_out_dev, void* slices_out_dev, void* stream) {
    pm_status s = check_prop_args(ctx, n_samples, dt);
    if (s != PM_OK) return s;
    if (!U_out_dev) return fail(ctx, PM_E_INVALID_ARG, "U_out is null");
    if (ctx->n_ctrl > 0 && !samples_dev) return fail(ctx, PM_E_INVALID_ARG, "samples is null");
    if (slices_out_dev && ctx->order == PM_ORDER_CF4)
        return fail(ctx, PM_E_INVALID_ARG, "per-slice output is not available with PM_ORDER_CF4");
    DeviceGuard g(ctx->device);
    if (!g.ok) return hip_fail(ctx, hipErrorInvalidDevice, "hipSetDevice");
    int64_t chunk = 0;
    s = begin_call(ctx, ctx->eng, n_samples, PM_WORK_PROPAGATE, slices_out_dev != nullptr, 0, &chunk);
    if (s != PM_OK) return s;
    CallChunk cc(ctx, chunk);
    return launch(ctx, samples_dev, n_samples, dt, U_out_dev, slices_out_dev, (hipStream_t)stream);
}

}  // extern "C"

namespace pm {

// pm_equiprop_dev with the tree's tickets and nodes in a fixed device
// workspace [base, base + bytes) instead of the context's buffers; nothing
// is allocated.  The tickets are cleared on the stream by a fill kernel
// before the launch.
pm_status equiprop_fixed_workspace(pm_ctx* ctx, const double* samples_dev, int64_t n_samples, double dt,
                                   double* U_out_dev, void* slices_out_dev, void* stream, void* base,
                                   size_t bytes) {
    pm_status s = check_prop_args(ctx, n_samples, dt);
    if (s != PM_OK) return s;
    if (!U_out_dev) return fail(ctx, PM_E_INVALID_ARG, "U_out is null");
    if (ctx->n_ctrl > 0 && !samples_dev) return fail(ctx, PM_E_INVALID_ARG, "samples is null");
    if (slices_out_dev && ctx->order == PM_ORDER_CF4)
        return fail(ctx, PM_E_INVALID_ARG, "per-slice output is not available with PM_ORDER_CF4");
    DeviceGuard g(ctx->device);
    if (!g.ok) return hip_fail(ctx, hipErrorInvalidDevice, "hipSetDevice");
    PropParams p;
    const FixedWorkspace fw{base, bytes};
    s = prepare(ctx, ctx->eng, false, ctx->d_basis, samples_dev, n_samples, dt, U_out_dev, slices_out_dev, &p,
                &fw);
    if (s != PM_OK) return s;
    const hipStream_t st = (hipStream_t)stream;
    const int64_t words = 2 * p.n_leaves + 64;
    hipError_t he = launch_zero(reinterpret_cast<double*>(p.counters), (words + 1) / 2, st);
    if (he != hipSuccess) return hip_fail(ctx, he, "ticket clear");
    he = launch_propagate(ctx->eng, ctx->precision, p, st);
    if (he != hipSuccess) return hip_fail(ctx, he, "kernel launch");
    return PM_OK;
}

int context_device(const pm_ctx* ctx) { return ctx ? ctx->device : -1; }

pm_status context_device_fail(pm_ctx* ctx, hipError_t e, const char* where) { return hip_fail(ctx, e, where); }

}  // namespace pm

extern "C" {

pm_status pm_equiprop(pm_ctx* ctx, const double* samples, int64_t n_samples, double dt,
                      double* U_out, void* slices_out) {
    pm_status s = check_prop_args(ctx, n_samples, dt);
    if (s != PM_OK) return s;
    if (!U_out) return fail(ctx, PM_E_INVALID_ARG, "U_out is null");
    if (ctx->n_ctrl > 0 && !samples) return fail(ctx, PM_E_INVALID_ARG, "samples is null");
    if (slices_out && ctx->order == PM_ORDER_CF4)
        return fail(ctx, PM_E_INVALID_ARG, "per-slice output is not available with PM_ORDER_CF4");
    const int64_t K = ctx->n_ctrl;
    for (int64_t i = 0; i < K * n_samples; ++i)
        if (!std::isfinite(samples[i])) return fail(ctx, PM_E_INVALID_ARG, "non-finite control sample");
    DeviceGuard g(ctx->device);
    if (!g.ok) return hip_fail(ctx, hipErrorInvalidDevice, "hipSetDevice");
    const int64_t N = n_slices_of(ctx->order, n_samples);
    const size_t sbytes = sizeof(double) * (size_t)std::max<int64_t>(K * n_samples, 1);
    const size_t elem = ctx->precision == PM_FP64 ? 16 : 8;
    const size_t slbytes = elem * (size_t)N * ctx->dim * ctx->dim;
    int64_t chunk = 0;
    s = begin_call(ctx, ctx->eng, n_samples, PM_WORK_PROPAGATE, slices_out != nullptr,
                   alloc_bytes(sbytes) + 16 * PM_MAX_DIM * PM_MAX_DIM + (slices_out ? alloc_bytes(slbytes) : 0),
                   &chunk);
    if (s != PM_OK) return s;
    CallChunk cc(ctx, chunk);
    s = ensure(ctx, (void**)&ctx->d_samples, &ctx->samples_bytes, sbytes, "samples");
    if (s != PM_OK) return s;
    s = ensure(ctx, (void**)&ctx->d_U, &ctx->u_bytes, 16 * PM_MAX_DIM * PM_MAX_DIM, "U");
    if (s != PM_OK) return s;
    if (slices_out) {
        s = ensure(ctx, &ctx->d_slices, &ctx->slices_bytes, slbytes, "slices");
        if (s != PM_OK) return s;
    }
    hipError_t he = hipSuccess;
    if (K > 0) {
        he = hipMemcpy(ctx->d_samples, samples, sizeof(double) * K * n_samples, hipMemcpyHostToDevice);
        if (he != hipSuccess) return hip_fail(ctx, he, "hipMemcpy samples");
    }
    s = launch(ctx, ctx->d_samples, n_samples, dt, ctx->d_U, slices_out ? ctx->d_slices : nullptr,
               nullptr);
    if (s != PM_OK) return s;
    he = hipDeviceSynchronize();
    if (he != hipSuccess) return hip_fail(ctx, he, "kernel execution");
    he = hipMemcpy(U_out, ctx->d_U, 16 * ctx->dim * ctx->dim, hipMemcpyDeviceToHost);
    if (he != hipSuccess) return hip_fail(ctx, he, "hipMemcpy U");
    if (slices_out) {
        he = hipMemcpy(slices_out, ctx->d_slices, slbytes, hipMemcpyDeviceToHost);
        if (he != hipSuccess) return hip_fail(ctx, he, "hipMemcpy slices");
    }
    return PM_OK;
}

pm_status check_grad_args(pm_ctx* ctx) {
    if (ctx->precision != PM_FP64)
        return fail(ctx, PM_E_UNSUPPORTED, "gradients are computed by PM_FP64 contexts");
    if (ctx->order == PM_ORDER_MAGNUS6)
        return fail(ctx, PM_E_UNSUPPORTED, "the sixth-order integrator has no adjoint or trajectory");
    return PM_OK;
}

pm_status pm_backward_dev(pm_ctx* ctx, const double* samples_dev, int64_t n_samples, double dt,
                          const double* W_dev, double* grad_dev, double* U_out_dev, void* stream) {
    pm_status s = check_prop_args(ctx, n_samples, dt);
    if (s != PM_OK) return s;
    s = check_grad_args(ctx);
    if (s != PM_OK) return s;
    if (!W_dev || (ctx->n_ctrl > 0 && (!samples_dev || !grad_dev)))
        return fail(ctx, PM_E_INVALID_ARG, "null pointer");
    DeviceGuard g(ctx->device);
    if (!g.ok) return hip_fail(ctx, hipErrorInvalidDevice, "hipSetDevice");
    int64_t chunk = 0;
    s = begin_call(ctx, ctx->geng, n_samples, PM_WORK_GRADIENT, false, 0, &chunk);
    if (s != PM_OK) return s;
    CallChunk cc(ctx, chunk);
    hipStream_t st = (hipStream_t)stream;
    // with U_out the forward writes U(T) there itself (no copy)
    return launch_grad(ctx, samples_dev, n_samples, dt, W_dev, grad_dev, st, true, true, U_out_dev);
}

pm_status pm_trajectory_dev(pm_ctx* ctx, const double* samples_dev, int64_t n_samples, double dt, int kind,
                            const double* x0_dev, int64_t n_vec, double* out_dev, void* stream) {
    pm_status s = check_prop_args(ctx, n_samples, dt);
    if (s != PM_OK) return s;
    if (ctx->precision != PM_FP64) return fail(ctx, PM_E_UNSUPPORTED, "trajectories are built for PM_FP64 contexts");
    if (ctx->order == PM_ORDER_MAGNUS6)
        return fail(ctx, PM_E_UNSUPPORTED, "the sixth-order integrator has no adjoint or trajectory");
    if (kind != PM_TRAJ_PROPAGATORS && kind != PM_TRAJ_STATES && kind != PM_TRAJ_DENSITY)
        return fail(ctx, PM_E_INVALID_ARG, "unknown trajectory kind");
    if (kind == PM_TRAJ_STATES && (n_vec < 1 || n_vec > ctx->dim))
        return fail(ctx, PM_E_INVALID_ARG, "n_vec must be in [1, dim]");
    if (!out_dev || (kind != PM_TRAJ_PROPAGATORS && !x0_dev) || (ctx->n_ctrl > 0 && !samples_dev))
        return fail(ctx, PM_E_INVALID_ARG, "null pointer");
    DeviceGuard g(ctx->device);
    if (!g.ok) return hip_fail(ctx, hipErrorInvalidDevice, "hipSetDevice");
    int64_t chunk = 0;
    s = begin_call(ctx, ctx->geng, n_samples, PM_WORK_TRAJECTORY, false, 0, &chunk);
    if (s != PM_OK) return s;
    CallChunk cc(ctx, chunk);
    hipStream_t st = (hipStream_t)stream;
    pm::TrajParams tp;
    s = forward_keep(ctx, samples_dev, n_samples, dt, st, true, &tp.p);
    if (s != PM_OK) return s;
    tp.kind = kind;
    tp.x0 = x0_dev;
    tp.n_vec = kind == PM_TRAJ_STATES ? (int)n_vec : (int)ctx->dim;
    tp.out = out_dev;
    const hipError_t he = pm::launch_trajectory(ctx->geng.D, tp, st);
    if (he != hipSuccess) return hip_fail(ctx, he, "trajectory launch");
    return PM_OK;
}

pm_status pm_grape_dev(pm_ctx* ctx, double* samples_dev, int64_t n_samples, double dt, const double* V_dev,
                       int iters, double step, int optimizer, double* loss_dev, void* stream) {
    pm_status s = check_prop_args(ctx, n_samples, dt);
    if (s != PM_OK) return s;
    s = check_grad_args(ctx);
    if (s != PM_OK) return s;
    if (iters < 0 || !(step > 0.0) || !std::isfinite(step) || (optimizer != PM_OPT_GD && optimizer != PM_OPT_ADAM))
        return fail(ctx, PM_E_INVALID_ARG, "iters >= 0, step > 0, optimizer PM_OPT_GD or PM_OPT_ADAM");
    if (!V_dev || !loss_dev || (ctx->n_ctrl > 0 && !samples_dev)) return fail(ctx, PM_E_INVALID_ARG, "null pointer");
    DeviceGuard g(ctx->device);
    if (!g.ok) return hip_fail(ctx, hipErrorInvalidDevice, "hipSetDevice");
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = ctx->n_ctrl * n_samples;
    int64_t chunk = 0;
    s = begin_call(ctx, ctx->geng, n_samples, PM_WORK_GRADIENT, false,
                   16 * PM_MAX_DIM * PM_MAX_DIM + alloc_bytes(sizeof(double) * (size_t)std::max<int64_t>(n, 1)) +
                       alloc_bytes(sizeof(double) * (size_t)std::max<int64_t>(2 * n, 1)),
                   &chunk);
    if (s != PM_OK) return s;
    CallChunk cc(ctx, chunk);
    s = ensure(ctx, (void**)&ctx->d_W, &ctx->w_bytes, 16 * PM_MAX_DIM * PM_MAX_DIM, "W");
    if (s != PM_OK) return s;
    s = ensure(ctx, (void**)&ctx->d_grad, &ctx->grad_bytes, sizeof(double) * (size_t)std::max<int64_t>(n, 1),
               "gradient");
    if (s != PM_OK) return s;
    s = ensure(ctx, (void**)&ctx->d_mom, &ctx->mom_bytes, sizeof(double) * (size_t)std::max<int64_t>(2 * n, 1),
               "optimiser moments");
    if (s != PM_OK) return s;
    hipError_t he = pm::launch_zero(ctx->d_mom, 2 * n, st);
    if (he != hipSuccess) return hip_fail(ctx, he, "moment reset");
    for (int it = 0; it <= iters; ++it) {
        // forward (keeping checkpoints), loss and W from U(T)
        s = launch_grad(ctx, samples_dev, n_samples, dt, nullptr, nullptr, st, true, false);
        if (s != PM_OK) return s;
        he = pm::launch_fidelity(ctx->d_UT, V_dev, (int)ctx->dim, ctx->d_W, loss_dev + it, st);
        if (he != hipSuccess) return hip_fail(ctx, he, "fidelity");
        if (it == iters) break;
        // adjoint on the same forward, then the control update
        s = launch_grad(ctx, samples_dev, n_samples, dt, ctx->d_W, ctx->d_grad, st, false, true);
        if (s != PM_OK) return s;
        he = pm::launch_update(samples_dev, ctx->d_grad, ctx->d_mom, ctx->d_mom + n, n, step, optimizer, it + 1,
                               0.9, 0.999, 1e-8, st);
        if (he != hipSuccess) return hip_fail(ctx, he, "control update");
    }
    return PM_OK;
}

pm_status pm_fidelity_grad(pm_ctx* ctx, const double* samples, int64_t n_samples, double dt,
                           const double* V, double* loss, double* grad, double* U_out) {
    pm_status s = check_prop_args(ctx, n_samples, dt);
    if (s != PM_OK) return s;
    s = check_grad_args(ctx);
    if (s != PM_OK) return s;
    if (!V || !loss || (ctx->n_ctrl > 0 && (!samples || !grad)))
        return fail(ctx, PM_E_INVALID_ARG, "null pointer");
    const int64_t K = ctx->n_ctrl, d = ctx->dim;
    for (int64_t i = 0; i < K * n_samples; ++i)
        if (!std::isfinite(samples[i])) return fail(ctx, PM_E_INVALID_ARG, "non-finite control sample");
    DeviceGuard g(ctx->device);
    if (!g.ok) return hip_fail(ctx, hipErrorInvalidDevice, "hipSetDevice");
    const size_t kb = alloc_bytes(sizeof(double) * (size_t)std::max<int64_t>(K * n_samples, 1));
    int64_t chunk = 0;
    s = begin_call(ctx, ctx->geng, n_samples, PM_WORK_GRADIENT, false, 2 * kb + 16 * PM_MAX_DIM * PM_MAX_DIM,
                   &chunk);
    if (s != PM_OK) return s;
    CallChunk cc(ctx, chunk);
    s = ensure(ctx, (void**)&ctx->d_samples, &ctx->samples_bytes,
               sizeof(double) * (size_t)std::max<int64_t>(K * n_samples, 1), "samples");
    if (s != PM_OK) return s;
    s = ensure(ctx, (void**)&ctx->d_W, &ctx->w_bytes, 16 * PM_MAX_DIM * PM_MAX_DIM, "W");
    if (s != PM_OK) return s;
    s = ensure(ctx, (void**)&ctx->d_grad, &ctx->grad_bytes,
               sizeof(double) * (size_t)std::max<int64_t>(K * n_samples, 1), "gradient");
    if (s != PM_OK) return s;
    hipError_t he;
    if (K > 0) {
        he = hipMemcpy(ctx->d_samples, samples, sizeof(double) * K * n_samples, hipMemcpyHostToDevice);
        if (he != hipSuccess) return hip_fail(ctx, he, "hipMemcpy samples");
    }
    s = launch_grad(ctx, ctx->d_samples, n_samples, dt, nullptr, nullptr, nullptr, true, false);
    if (s != PM_OK) return s;
    std::vector<double> U(2 * d * d), W(2 * d * d);
    he = hipMemcpy(U.data(), ctx->d_UT, 16 * d * d, hipMemcpyDeviceToHost);
    if (he != hipSuccess) return hip_fail(ctx, he, "hipMemcpy U");
    // L = 1 - |g|^2 / d^2, g = Tr(V^H U);  W = 2 dL/d conj(U) = -(2 g / d^2) V
    cplx gg(0, 0);
    for (int64_t a = 0; a < d; ++a)
        for (int64_t b = 0; b < d; ++b)
            gg += std::conj(cplx(V[(a * d + b) * 2], V[(a * d + b) * 2 + 1])) *
                  cplx(U[(a * d + b) * 2], U[(a * d + b) * 2 + 1]);
    const double d2 = (double)(d * d);
    const cplx f = -2.0 * gg / d2;
    for (int64_t i = 0; i < d * d; ++i) {
        const cplx w = f * cplx(V[2 * i], V[2 * i + 1]);
        W[2 * i] = w.real();
        W[2 * i + 1] = w.imag();
    }
    he = hipMemcpy(ctx->d_W, W.data(), 16 * d * d, hipMemcpyHostToDevice);
    if (he != hipSuccess) return hip_fail(ctx, he, "hipMemcpy W");
    // the backward reuses the forward's checkpoints (same launch parameters)
    s = launch_grad(ctx, ctx->d_samples, n_samples, dt, ctx->d_W, ctx->d_grad, nullptr, false, true);
    if (s != PM_OK) return s;
    he = hipDeviceSynchronize();
    if (he != hipSuccess) return hip_fail(ctx, he, "gradient kernels");
    if (K > 0) {
        he = hipMemcpy(grad, ctx->d_grad, sizeof(double) * K * n_samples, hipMemcpyDeviceToHost);
        if (he != hipSuccess) return hip_fail(ctx, he, "hipMemcpy gradient");
    }
    *loss = 1.0 - std::norm(gg) / d2;
    if (U_out) std::memcpy(U_out, U.data(), 16 * d * d);
    return PM_OK;
}

// ------------------------------------------------------------------ batches

}  // extern "C"

struct pm_batch {
    int device = 0;
    int precision = PM_FP64;
    int64_t chunk_cfg[3] = {0, 0, 0};   // dimension classes 16, 32, 64
    std::vector<pm::PropParams> inst;
    std::vector<pm::BatchPacket> packets;
    int64_t out_doubles = 0;
    double* d_basis = nullptr;
    double* d_samples = nullptr;
    double* d_nodes = nullptr;
    unsigned* d_counters = nullptr;
    double* d_out = nullptr;
    pm::PropParams* d_inst = nullptr;
    pm::BatchPacket* d_packets = nullptr;
    unsigned* d_queue = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int blocks = 0;
    bool broken = false;
    std::string err;
};

namespace {

int class_of(int64_t dim) { return dim <= 16 ? 16 : (dim <= 32 ? 32 : 64); }
int class_index(int D) { return D == 16 ? 0 : (D == 32 ? 1 : 2); }
int64_t default_batch_chunk(int D) { return D == 16 ? 64 : (D == 32 ? 32 : 16); }

pm_status bfail(pm_batch* b, pm_status s, const std::string& msg) {
    b->err = msg;
    return s;
}

pm_status bhip(pm_batch* b, hipError_t e, const char* where) {
    b->broken = true;
    b->err = std::string(where) + ": " + hipGetErrorString(e);
    return PM_E_DEVICE;
}

void batch_free(pm_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    dfree(b->d_basis);
    dfree(b->d_samples);
    dfree(b->d_nodes);
    dfree(b->d_counters);
    dfree(b->d_out);
    dfree(b->d_inst);
    dfree(b->d_packets);
    dfree(b->d_queue);
    b->inst.clear();
    b->packets.clear();
    b->out_doubles = 0;
}

template <typename P>
hipError_t upload(P** dst, const void* src, size_t bytes) {
    hipError_t e = hipMalloc((void**)dst, std::max<size_t>(bytes, 256));
    if (e != hipSuccess) {
        *dst = nullptr;
        return e;
    }
    if (src && bytes) e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
    return e;
}

}  // namespace

extern "C" {

pm_status pm_batch_create(pm_batch** out, int device, int precision) {
    if (!out) return PM_E_INVALID_ARG;
    *out = nullptr;
    g_create_err.clear();
    if (unit_roundoff(precision) < 0) return create_fail(PM_E_INVALID_ARG, "unknown precision");
    int n = 0;
    const hipError_t de = hipGetDeviceCount(&n);
    if (de != hipSuccess || n <= 0) return create_fail(PM_E_DEVICE, "no HIP device", de);
    if (device < 0 || device >= n) return PM_E_INVALID_ARG;
    pm_batch* b = new (std::nothrow) pm_batch();
    if (!b) return PM_E_OOM;
    b->device = device;
    b->precision = precision;
    DeviceGuard g(device);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
        cus = 256;
    b->blocks = cus;
    const hipError_t se = pm::batch_setup(precision);
    if (se != hipSuccess) {
        delete b;
        return create_fail(PM_E_DEVICE, "batch kernel setup (dynamic LDS attribute)", se);
    }
    const hipError_t ce = hipStreamCreate(&b->cap);
    if (ce != hipSuccess) {
        delete b;
        return create_fail(PM_E_DEVICE, "capture stream", ce);
    }
    *out = b;
    return PM_OK;
}

pm_status pm_batch_destroy(pm_batch* b) {
    if (!b) return PM_OK;
    {
        DeviceGuard g(b->device);
        (void)hipDeviceSynchronize();
        batch_free(b);
        if (b->cap) (void)hipStreamDestroy(b->cap);
    }
    delete b;
    return PM_OK;
}

pm_status pm_batch_set_chunk(pm_batch* b, int dim_class, int64_t chunk) {
    if (!b) return PM_E_INVALID_ARG;
    if ((dim_class != 16 && dim_class != 32 && dim_class != 64) || chunk < 0)
        return bfail(b, PM_E_INVALID_ARG, "dim_class in {16, 32, 64}, chunk >= 0");
    b->chunk_cfg[class_index(dim_class)] = chunk;
    return PM_OK;
}

pm_status pm_batch_set(pm_batch* b, const pm_instance* inst, int64_t n_inst) {
    if (!b) return PM_E_INVALID_ARG;
    if (b->broken) return bfail(b, PM_E_DEVICE, "batch unusable after a device error");
    if (n_inst < 1 || !inst) return bfail(b, PM_E_INVALID_ARG, "need at least one instance");
    std::vector<pm::PropParams> P((size_t)n_inst);
    std::vector<double> hbasis, hsamples;
    std::vector<int64_t> boff(n_inst), soff(n_inst), noff(n_inst), coff(n_inst), ooff(n_inst);
    std::vector<pm::BatchPacket> packets;
    int64_t nodes_d = 0, counters_n = 0, out_d = 0;
    for (int64_t i = 0; i < n_inst; ++i) {
        const pm_instance& q = inst[i];
        const std::string tag = "instance " + std::to_string(i) + ": ";
        if (q.dim < 1 || q.dim > PM_MAX_DIM) return bfail(b, PM_E_INVALID_ARG, tag + "dim must be in [1, 64]");
        if (q.n_ctrl < 0 || q.n_ctrl > pm::kMaxCtrl) return bfail(b, PM_E_INVALID_ARG, tag + "n_ctrl in [0, 8]");
        if (q.order == PM_ORDER_MAGNUS6)
            return bfail(b, PM_E_UNSUPPORTED, tag + "batches take orders 2, 4 and PM_ORDER_CF4");
        if (!order_ok(q.order)) return bfail(b, PM_E_INVALID_ARG, tag + "order must be 2, 4 or PM_ORDER_CF4");
        if (!q.H0 || (q.n_ctrl > 0 && (!q.Hk || !q.samples))) return bfail(b, PM_E_INVALID_ARG, tag + "null pointer");
        if (!(q.dt > 0.0) || !std::isfinite(q.dt)) return bfail(b, PM_E_INVALID_ARG, tag + "dt must be finite and > 0");
        if ((q.order == 2 && q.n_samples < 1) || (q.order != 2 && (q.n_samples < 3 || q.n_samples % 2 == 0)))
            return bfail(b, PM_E_INVALID_ARG, tag + "bad n_samples for the order");
        for (int64_t k = 0; k < q.n_ctrl * q.n_samples; ++k)
            if (!std::isfinite(q.samples[k])) return bfail(b, PM_E_INVALID_ARG, tag + "non-finite sample");
        std::vector<Mat> basis;
        std::vector<std::pair<int, int>> pairs;
        std::string err;
        pm_status st = build_basis(q.dim, q.H0, q.n_ctrl, q.Hk, q.order, &basis, &pairs, &err);
        if (st != PM_OK) return bfail(b, st, tag + err);
        const int M = (int)basis.size();
        const int D = class_of(q.dim);
        pm::EngineInfo e;
        pm::pick_engine(D, b->precision, &e);
        std::vector<double> flat((size_t)M * q.dim * q.dim * 2);
        for (int m = 0; m < M; ++m)
            for (int64_t x = 0; x < q.dim * q.dim; ++x) {
                flat[((size_t)m * q.dim * q.dim + x) * 2 + 0] = basis[m][x].real();
                flat[((size_t)m * q.dim * q.dim + x) * 2 + 1] = basis[m][x].imag();
            }
        std::vector<double> lay((size_t)pm::basis_layout_doubles(e, M));
        pm::basis_to_layout(e, M, (int)q.dim, flat.data(), lay.data());
        boff[i] = (int64_t)hbasis.size();
        hbasis.insert(hbasis.end(), lay.begin(), lay.end());
        soff[i] = (int64_t)hsamples.size();
        if (q.n_ctrl > 0) hsamples.insert(hsamples.end(), q.samples, q.samples + q.n_ctrl * q.n_samples);
        const int64_t N = n_exps_of(q.order, q.n_samples);
        const int TEAMS = pm::batch_teams(D);
        int64_t chunk = b->chunk_cfg[class_index(D)];
        if (chunk <= 0) chunk = g_tune_batch_chunk[class_index(D)][b->precision];
        if (chunk <= 0) chunk = default_batch_chunk(D);
        if (q.order == PM_ORDER_CF4 && (chunk & 1)) ++chunk;   // chains start at slice boundaries
        chunk = std::min(chunk, N);
        const int64_t chains = (N + chunk - 1) / chunk;
        const int64_t npk = (chains + TEAMS - 1) / TEAMS;
        noff[i] = nodes_d;
        nodes_d += (2 * npk + 64) * (int64_t)D * D * 2;
        coff[i] = counters_n;
        counters_n += 2 * npk + 64;
        ooff[i] = out_d;
        out_d += q.dim * q.dim * 2;
        pm::PropParams& p = P[i];
        std::memset(&p, 0, sizeof(p));
        p.n_samples = q.n_samples;
        p.n_slices = N;
        p.chunk = chunk;
        p.n_chains = chains;
        p.n_leaves = npk;
        p.h = q.dt;
        fill_theta(p.theta, b->precision, N);
        p.K = (int)q.n_ctrl;
        p.M = M;
        p.order = q.order;
        p.du = (int)q.dim;
        p.max_degree = PM_MAX_TAYLOR_DEGREE;
        p.force_s = -1;
        for (size_t x = 0; x < pairs.size(); ++x) {
            const int m = 1 + 2 * (int)q.n_ctrl + (int)x;
            p.pair_a[m] = (uint8_t)pairs[x].first;
            p.pair_b[m] = (uint8_t)pairs[x].second;
        }
        for (int64_t pk = 0; pk < npk; ++pk) {
            pm::BatchPacket bp;
            bp.inst = (int)i;
            bp.D = D;
            bp.chain0 = pk * TEAMS;
            bp.nchains = (int)std::min<int64_t>(TEAMS, chains - bp.chain0);
            bp.leaf = (int)pk;
            bp.steps = std::min(chunk, N - bp.chain0 * chunk);
            packets.push_back(bp);
        }
    }
    // longest first: a block's work per packet ~ steps * teams * D^3
    auto cost = [](const pm::BatchPacket& x) {
        return (double)x.steps * pm::batch_teams(x.D) * (double)x.D * x.D * x.D;
    };
    std::stable_sort(packets.begin(), packets.end(),
                     [&](const pm::BatchPacket& a, const pm::BatchPacket& c) { return cost(a) > cost(c); });

    DeviceGuard g(b->device);
    if (!g.ok) return bhip(b, hipErrorInvalidDevice, "hipSetDevice");
    hipError_t he = hipDeviceSynchronize();
    if (he != hipSuccess) return bhip(b, he, "hipDeviceSynchronize");
    batch_free(b);
    he = upload(&b->d_basis, hbasis.data(), hbasis.size() * sizeof(double));
    if (he == hipSuccess) he = upload(&b->d_samples, hsamples.data(), hsamples.size() * sizeof(double));
    if (he == hipSuccess) he = upload(&b->d_nodes, nullptr, (size_t)nodes_d * sizeof(double));
    if (he == hipSuccess) he = upload(&b->d_counters, nullptr, (size_t)counters_n * sizeof(unsigned));
    if (he == hipSuccess) he = hipMemset(b->d_counters, 0, std::max<size_t>((size_t)counters_n * sizeof(unsigned), 256));
    if (he == hipSuccess) he = upload(&b->d_out, nullptr, (size_t)out_d * sizeof(double));
    if (he == hipSuccess) he = upload(&b->d_queue, nullptr, sizeof(unsigned));
    if (he != hipSuccess) {
        (void)hipGetLastError();
        batch_free(b);
        return bfail(b, PM_E_OOM, "device allocation for the batch failed");
    }
    for (int64_t i = 0; i < n_inst; ++i) {
        pm::PropParams& p = P[i];
        p.basis = b->d_basis + boff[i];
        p.samples = b->d_samples + soff[i];
        p.nodes = b->d_nodes + noff[i];
        p.counters = b->d_counters + coff[i];
        p.U_out = b->d_out + ooff[i];
    }
    he = upload(&b->d_inst, P.data(), P.size() * sizeof(pm::PropParams));
    if (he == hipSuccess) he = upload(&b->d_packets, packets.data(), packets.size() * sizeof(pm::BatchPacket));
    if (he == hipSuccess) he = hipDeviceSynchronize();
    if (he != hipSuccess) {
        (void)hipGetLastError();
        batch_free(b);
        return bfail(b, PM_E_OOM, "device allocation for the batch failed");
    }
    b->inst = P;
    b->packets = packets;
    b->out_doubles = out_d;
    b->err.clear();
    return PM_OK;
}

pm_status pm_batch_run(pm_batch* b, void* stream) {
    if (!b) return PM_E_INVALID_ARG;
    if (b->broken) return bfail(b, PM_E_DEVICE, "batch unusable after a device error");
    if (b->inst.empty()) return bfail(b, PM_E_NOT_READY, "pm_batch_set has not been called");
    DeviceGuard g(b->device);
    if (!g.ok) return bhip(b, hipErrorInvalidDevice, "hipSetDevice");
    hipError_t he;
    if (!b->exec) {
        pm::BatchParams bp;
        bp.inst = b->d_inst;
        bp.packets = b->d_packets;
        bp.n_packets = (int)b->packets.size();
        bp.queue = b->d_queue;
        he = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
        if (he != hipSuccess) return bhip(b, he, "hipStreamBeginCapture");
        he = pm::launch_batch(b->precision, bp, b->blocks, b->cap);
        hipGraph_t gr = nullptr;
        const hipError_t he2 = hipStreamEndCapture(b->cap, &gr);
        if (he != hipSuccess) return bhip(b, he, "batch launch");
        if (he2 != hipSuccess) return bhip(b, he2, "hipStreamEndCapture");
        b->graph = gr;
        he = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (he != hipSuccess) return bhip(b, he, "hipGraphInstantiate");
    }
    he = hipGraphLaunch(b->exec, (hipStream_t)stream);
    if (he != hipSuccess) return bhip(b, he, "hipGraphLaunch");
    return PM_OK;
}

pm_status pm_batch_result(pm_batch* b, double* U_out, int64_t n_doubles) {
    if (!b || !U_out) return PM_E_INVALID_ARG;
    if (b->inst.empty()) return bfail(b, PM_E_NOT_READY, "pm_batch_set has not been called");
    if (n_doubles < b->out_doubles) return bfail(b, PM_E_INVALID_ARG, "output buffer too small");
    DeviceGuard g(b->device);
    hipError_t he = hipDeviceSynchronize();
    if (he != hipSuccess) return bhip(b, he, "batch execution");
    he = hipMemcpy(U_out, b->d_out, sizeof(double) * b->out_doubles, hipMemcpyDeviceToHost);
    if (he != hipSuccess) return bhip(b, he, "hipMemcpy results");
    return PM_OK;
}

pm_status pm_batch_output_dev(pm_batch* b, const double** out) {
    if (!b || !out) return PM_E_INVALID_ARG;
    if (b->inst.empty()) return bfail(b, PM_E_NOT_READY, "pm_batch_set has not been called");
    *out = b->d_out;
    return PM_OK;
}

int64_t pm_batch_packets(const pm_batch* b) { return b ? (int64_t)b->packets.size() : -1; }

int64_t pm_batch_output_doubles(const pm_batch* b) { return b ? b->out_doubles : -1; }

const char* pm_batch_last_error(const pm_batch* b) { return b ? b->err.c_str() : g_create_err.c_str(); }

pm_status pm_tuning_set(const char* key, int dim_class, int precision, int64_t value) {
    if (!key || value < 0 || precision < 0 || precision > 3) return PM_E_INVALID_ARG;
    const std::string k(key);
    if (k == "chains") {
        const int tc = tune_class(dim_class);
        if (tc < 0) return PM_E_INVALID_ARG;
        g_tune_chains[tc][precision] = value;
        return PM_OK;
    }
    if (k == "batch_chunk") {
        if (dim_class != 16 && dim_class != 32 && dim_class != 64) return PM_E_INVALID_ARG;
        g_tune_batch_chunk[class_index(dim_class)][precision] = value;
        return PM_OK;
    }
    return PM_E_INVALID_ARG;
}

}  // extern "C"
