// Karhunen-Loeve synthesis u = sum_i sqrt(lambda_i) xi_i phi_i at the grid nodes.
//
// 2D: the cosine basis is separable, phi_kl(x_i, y_j) = B[i][k] B[j][l], so per particle
//     u[j][i] = sum_k sum_l B[i][k] X[k][l] B[j][l],   X[k][l] = sqrt(lambda_kl) xi_kl,
// i.e. two small dense products T = X B^T (32 x (n+1)) and U = T^T B^T ((n+1) x (n+1)).
// Both run on the FP64 matrix cores (v_mfma_f64_16x16x4f64) with the operands staged in
// LDS; the epilogue optionally returns exp(u/2), the nodal factor of the geometric-mean face
// coefficient exp((u_P + u_Q)/2) = exp(u_P/2) exp(u_Q/2) of the forward operator.
#include "common.hpp"

namespace smc {

typedef double d4 __attribute__((ext_vector_type(4)));

// MFMA f64 16x16x4 operand layout (one double per lane), checked on the device:
//   A[16][4]: lane = row + 16 * k     B[4][16]: lane = col + 16 * k
//   D[16][16]: lane = col + 16 * (row % 4), element row / 4
template <bool EXPHALF>
__global__ __launch_bounds__(256) void synth2d_kernel(const double* __restrict__ xi, int K, int kl,
                                                      const double* __restrict__ sqrt_lam,
                                                      const double* __restrict__ basis, int n,
                                                      double* __restrict__ out, int64_t out_stride) {
    extern __shared__ double smem[];
    const int np1 = n + 1;
    const int npad = (np1 + 15) & ~15;
    constexpr int LD = KLP + 1;                 // padded row stride: conflict-free column reads
    double* X = smem;                           // [KLP][LD]
    double* Bs = X + KLP * LD;                  // [npad][LD]
    double* T = Bs + npad * LD;                 // [KLP][npad]
    const int64_t p = blockIdx.x;
    const double* xp = xi + p * K;

    for (int t = threadIdx.x; t < KLP * KLP; t += 256) {
        const int k = t / KLP, l = t % KLP;
        X[k * LD + l] = (k < kl && l < kl) ? sqrt_lam[k * kl + l] * xp[k * kl + l] : 0.0;
    }
    for (int t = threadIdx.x; t < npad * KLP; t += 256) {
        const int i = t / KLP, k = t % KLP;
        Bs[i * LD + k] = (i < np1) ? basis[i * KLP + k] : 0.0;
    }
    __syncthreads();

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const int ntj = npad / 16;
    // T[k][j] = sum_l X[k][l] B[j][l]
    for (int tile = wave; tile < 2 * ntj; tile += 4) {
        const int k0 = (tile & 1) * 16, j0 = (tile >> 1) * 16;
        d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int l0 = 0; l0 < KLP; l0 += 4) {
            const double a = X[(k0 + lr) * LD + l0 + lk];
            const double b = Bs[(j0 + lr) * LD + l0 + lk];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) T[(k0 + lk + 4 * v) * npad + j0 + lr] = acc[v];
    }
    __syncthreads();
    // U[j][i] = sum_k T[k][j] B[i][k]
    double* op = out + p * out_stride;
    for (int tile = wave; tile < ntj * ntj; tile += 4) {
        const int j0 = (tile / ntj) * 16, i0 = (tile % ntj) * 16;
        d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k0 = 0; k0 < KLP; k0 += 4) {
            const double a = T[(k0 + lk) * npad + j0 + lr];
            const double b = Bs[(i0 + lr) * LD + k0 + lk];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
        const int i = i0 + lr;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int j = j0 + lk + 4 * v;
            if (i < np1 && j < np1) op[j * np1 + i] = EXPHALF ? exp(0.5 * acc[v]) : acc[v];
        }
    }
}

// 1D: u[i] = sum_k S[i][k] sqrt(lambda_k) xi_k with S[i][k] = sqrt(2) sin(k pi i / n).
template <bool EXPHALF>
__global__ __launch_bounds__(256) void synth1d_kernel(const double* __restrict__ xi, int kl,
                                                      const double* __restrict__ sqrt_lam,
                                                      const double* __restrict__ basis, int n,
                                                      double* __restrict__ out, int64_t out_stride) {
    __shared__ double c[64];
    const int64_t p = blockIdx.x;
    if (threadIdx.x < kl) c[threadIdx.x] = sqrt_lam[threadIdx.x] * xi[p * kl + threadIdx.x];
    __syncthreads();
    for (int i = threadIdx.x; i <= n; i += 256) {
        double s = 0.0;
        for (int k = 0; k < kl; ++k) s = fma(basis[i * kl + k], c[k], s);
        out[p * out_stride + i] = EXPHALF ? exp(0.5 * s) : s;
    }
}

hipError_t launch_synth2d(const double* xi, int K, int kl, const double* sqrt_lam, const double* basis, int n,
                          double* out, int64_t out_stride, int64_t N, bool exp_half, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    const int npad = (n + 1 + 15) & ~15;
    const size_t lds = sizeof(double) * ((size_t)KLP * (KLP + 1) + (size_t)npad * (KLP + 1) + (size_t)KLP * npad);
    if (exp_half) {
        hipError_t e = hipFuncSetAttribute((const void*)synth2d_kernel<true>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        synth2d_kernel<true><<<dim3((unsigned)N), dim3(256), lds, s>>>(xi, K, kl, sqrt_lam, basis, n, out, out_stride);
    } else {
        hipError_t e = hipFuncSetAttribute((const void*)synth2d_kernel<false>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        synth2d_kernel<false><<<dim3((unsigned)N), dim3(256), lds, s>>>(xi, K, kl, sqrt_lam, basis, n, out, out_stride);
    }
    return hipGetLastError();
}

hipError_t launch_synth1d(const double* xi, int kl, const double* sqrt_lam, const double* basis, int n, double* out,
                          int64_t out_stride, int64_t N, bool exp_half, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    if (exp_half)
        synth1d_kernel<true><<<dim3((unsigned)N), dim3(256), 0, s>>>(xi, kl, sqrt_lam, basis, n, out, out_stride);
    else
        synth1d_kernel<false><<<dim3((unsigned)N), dim3(256), 0, s>>>(xi, kl, sqrt_lam, basis, n, out, out_stride);
    return hipGetLastError();
}

}  // namespace smc
