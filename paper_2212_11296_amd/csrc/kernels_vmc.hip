// Variational Monte Carlo step kernels: the weights of the energy
// gradient estimator and the parameter update.
//
// For a real, positive psi the gradient of E = <H> over Born samples is
// dE/dtheta = 2 < (E_loc - E) d log psi / d theta >  (eq. 3 with the
// normalisation of a batch mean), so the weighted gradient of log psi with
// w_i = 2 (E_loc(s_i) - mean E_loc) / B is the energy gradient.
#include "kernels.h"

namespace vq {

__global__ void k_vmc_weights(const double* __restrict__ eloc,
                              const double* __restrict__ stats, int64_t B,
                              double* __restrict__ w) {
    const double mean = stats[0];
    const double scale = 2.0 / (double)B;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < B;
         i += (int64_t)gridDim.x * blockDim.x)
        w[i] = scale * (eloc[i] - mean);
}

hipError_t launch_vmc_weights(const double* eloc, const double* stats,
                              int64_t B, double* w, hipStream_t st) {
    int64_t blocks = (B + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_vmc_weights, dim3((unsigned)blocks), dim3(256), 0,
                       st, eloc, stats, B, w);
    return hipGetLastError();
}

// theta <- theta - lr g (plain gradient descent) when m == nullptr, else
// Adam (Kingma & Ba 2015) with bias-corrected moments at step t >= 1:
// m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
// theta <- theta - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
template <typename T>
__global__ void k_update(T* __restrict__ p, const T* __restrict__ g,
                         T* __restrict__ m, T* __restrict__ v, int64_t n,
                         double lr, double b1, double b2, double eps,
                         double c1, double c2) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const double gk = (double)g[k];
        if (!m) {
            p[k] = (T)((double)p[k] - lr * gk);
            continue;
        }
        const double mk = b1 * (double)m[k] + (1.0 - b1) * gk;
        const double vk = b2 * (double)v[k] + (1.0 - b2) * gk * gk;
        m[k] = (T)mk;
        v[k] = (T)vk;
        p[k] = (T)((double)p[k] - lr * (mk / c1) / (sqrt(vk / c2) + eps));
    }
}

template <typename T>
hipError_t launch_update(T* p, const T* g, T* m, T* v, int64_t n, double lr,
                         double b1, double b2, double eps, int64_t step,
                         hipStream_t st) {
    const double c1 = 1.0 - pow(b1, (double)step);
    const double c2 = 1.0 - pow(b2, (double)step);
    int64_t blocks = (n + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_update<T>, dim3((unsigned)blocks), dim3(256), 0, st,
                       p, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

template hipError_t launch_update<float>(float*, const float*, float*, float*,
                                         int64_t, double, double, double,
                                         double, int64_t, hipStream_t);
template hipError_t launch_update<double>(double*, const double*, double*,
                                          double*, int64_t, double, double,
                                          double, double, int64_t,
                                          hipStream_t);

}  // namespace vq
