// Device side of the gradient-based control optimisation (GRAPE, Applications
// and outlook section): the gate-fidelity loss and its U(T)-gradient from
// U(T), and the control update (gradient descent or Adam), so that an
// optimisation loop runs without host synchronisation.
#include "pm_internal.h"

namespace pm {
namespace {

// g = Tr(V^H U) over du x du, L = 1 - |g|^2 / du^2, W = -(2 g / du^2) V.
// One block of 256 threads.
__global__ void __launch_bounds__(256) fidelity_kernel(const double* U, const double* V, int du, double* W,
                                                      double* loss) {
    __shared__ double sre[256], sim[256];
    const int t = threadIdx.x;
    const int n = du * du;
    double gr = 0.0, gi = 0.0;
    for (int e = t; e < n; e += 256) {
        const double vr = V[2 * e], vi = V[2 * e + 1], ur = U[2 * e], ui = U[2 * e + 1];
        gr += vr * ur + vi * ui;   // conj(V) U
        gi += vr * ui - vi * ur;
    }
    sre[t] = gr;
    sim[t] = gi;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) {
            sre[t] += sre[t + s];
            sim[t] += sim[t + s];
        }
        __syncthreads();
    }
    const double d2 = (double)n;
    const double fr = -2.0 * sre[0] / d2, fi = -2.0 * sim[0] / d2;
    for (int e = t; e < n; e += 256) {
        const double vr = V[2 * e], vi = V[2 * e + 1];
        W[2 * e] = fr * vr - fi * vi;
        W[2 * e + 1] = fr * vi + fi * vr;
    }
    if (t == 0 && loss) *loss = 1.0 - (sre[0] * sre[0] + sim[0] * sim[0]) / d2;
}

// c <- c - step * g (optimizer 0), or the Adam update with moments m, v and
// bias correction for step number `it` (1-based; optimizer 1).
__global__ void __launch_bounds__(256) update_kernel(double* c, const double* g, double* m, double* v, int64_t n,
                                                    double step, int optimizer, int it, double b1, double b2,
                                                    double eps) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double gi = g[i];
    if (optimizer == 0) {
        c[i] -= step * gi;
        return;
    }
    const double mi = b1 * m[i] + (1.0 - b1) * gi;
    const double vi = b2 * v[i] + (1.0 - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const double mh = mi / (1.0 - pow(b1, (double)it));
    const double vh = vi / (1.0 - pow(b2, (double)it));
    c[i] -= step * mh / (sqrt(vh) + eps);
}

__global__ void fill_zero(double* a, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) a[i] = 0.0;
}

}  // namespace

hipError_t launch_fidelity(const double* U, const double* V, int du, double* W, double* loss, hipStream_t st) {
    hipLaunchKernelGGL(fidelity_kernel, dim3(1), dim3(256), 0, st, U, V, du, W, loss);
    return hipGetLastError();
}

hipError_t launch_update(double* c, const double* g, double* m, double* v, int64_t n, double step, int optimizer,
                         int it, double b1, double b2, double eps, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(update_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, c, g, m, v, n, step,
                       optimizer, it, b1, b2, eps);
    return hipGetLastError();
}

hipError_t launch_zero(double* a, int64_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, n);
    return hipGetLastError();
}

}  // namespace pm
