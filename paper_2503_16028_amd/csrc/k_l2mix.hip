// Potential of a mixture likelihood in L^2 (the paper's Example 1, Sec. 3.1, eq. (example1phi)):
//   exp(-Phi(u)) = sum_i exp(-|u - f_i|^2 / (2 sigma^2)),
// with u = sum_k sqrt(lambda_k) xi_k phi_k and each f_i given by its coefficients c_ik on the same
// orthonormal basis, so |u - f_i|^2 = sum_k (sqrt(lambda_k) xi_k - c_ik)^2 (Parseval).  No PDE.
#include "common.hpp"

namespace smc {

// Sixteen lanes per particle (four particles per wave, sixteen per workgroup); the lanes of a
// particle stride over the modes and each likelihood term is summed by one 16-lane butterfly.
__global__ __launch_bounds__(256) void l2mix_phi_kernel(int64_t N, int K, const double* __restrict__ sqrt_lam,
                                                        const double* __restrict__ c, int T, double inv2s2,
                                                        const double* __restrict__ xi, double* __restrict__ phi,
                                                        int32_t* __restrict__ iters) {
    const int sub = threadIdx.x & 15;
    const int64_t n = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
    if (n >= N) return;   // the same for all 16 lanes of a particle; the butterflies stay inside them
    double acc[MAX_TERMS];
#pragma unroll
    for (int i = 0; i < MAX_TERMS; ++i) acc[i] = 0.0;
    for (int k = sub; k < K; k += 16) {
        const double a = sqrt_lam[k] * xi[n * K + k];
#pragma unroll
        for (int i = 0; i < MAX_TERMS; ++i) {
            if (i < T) {
                const double d = a - c[(int64_t)i * K + k];
                acc[i] += d * d;
            }
        }
    }
    double ll[MAX_TERMS];
    double mx = -INFINITY;
#pragma unroll
    for (int i = 0; i < MAX_TERMS; ++i) {
        if (i < T) {
            double v = acc[i];
#pragma unroll
            for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off, 16);
            ll[i] = -v * inv2s2;
            mx = fmax(mx, ll[i]);
        }
    }
    double se = 0.0;
#pragma unroll
    for (int i = 0; i < MAX_TERMS; ++i)
        if (i < T) se += exp(ll[i] - mx);
    if (sub == 0) {
        phi[n] = -(mx + log(se));
        if (iters) iters[n] = 0;
    }
}

hipError_t launch_l2mix_phi(int64_t N, int K, const double* sqrt_lam, const double* c, int T, double inv2s2,
                            const double* xi, double* phi, int32_t* iters, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    l2mix_phi_kernel<<<dim3((unsigned)((N + 15) / 16)), dim3(256), 0, s>>>(N, K, sqrt_lam, c, T, inv2s2, xi, phi,
                                                                          iters);
    return hipGetLastError();
}

}  // namespace smc
