// Karhunen-Loeve synthesis u = sum_i sqrt(lambda_i) xi_i phi_i at the grid nodes.
//
// 2D: the cosine basis is separable, phi_kl(x_i, y_j) = B[i][k] B[j][l], so per particle
//     u[j][i] = sum_k sum_l B[i][k] X[k][l] B[j][l],   X[k][l] = sqrt(lambda_kl) xi_kl,
// i.e. two small dense products T = X B^T (32 x (n+1)) and U = T^T B^T ((n+1) x (n+1)).
// Both run on the FP64 matrix cores (v_mfma_f64_16x16x4f64), X and T in LDS (T written over
// X) and B read straight into registers; the epilogue optionally returns exp(u/2), the nodal
// factor of the geometric-mean face coefficient exp((u_P + u_Q)/2) = exp(u_P/2) exp(u_Q/2) of the
// forward operator.
#include "common.hpp"
#include "synth_body.hpp"

namespace smc {

template <bool EXPHALF>
__global__ __launch_bounds__(SYN_THREADS) void synth2d_kernel(const double* __restrict__ xi, int K, int kl,
                                                      const double* __restrict__ sqrt_lam,
                                                      const double* __restrict__ basis, int n,
                                                      double* __restrict__ out, int64_t out_stride) {
    extern __shared__ double smem[];
    const int64_t p = blockIdx.x;
    synth2d_body<EXPHALF>(xi + p * K, kl, sqrt_lam, basis, n, out + p * out_stride, smem);
}

// The same for particles on several grids: particle p on grid level[p] (others are skipped).
template <bool EXPHALF>
__global__ __launch_bounds__(SYN_THREADS) void synth2d_levels_kernel(const double* __restrict__ xi, int K, int kl,
                                                             const double* __restrict__ sqrt_lam, LevelTable lt,
                                                             const int32_t* __restrict__ level,
                                                             double* __restrict__ out, int64_t out_stride) {
    extern __shared__ double smem[];
    const int64_t p = blockIdx.x;
    const int l = level[p];
    if (l < 0 || l >= lt.n_levels) return;
    synth2d_body<EXPHALF>(xi + p * K, kl, sqrt_lam, lt.basis[l], lt.n[l], out + p * out_stride, smem);
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

// Gradient of Phi with respect to the whitened coefficients from the forward solution w and the
// adjoint solution lam (the extra solve of gradient-informed moves, Sec. 2.4).  With
// A(u) w = f and lam^T A w = sum over faces (P,Q) of a_PQ (lam_P - lam_Q)(w_P - w_Q) / h^2,
// d a_PQ / d u_P = a_PQ / 2 gives at every node P (boundary nodes included, w = lam = 0 there)
//   dU[P] = dPhi/du_P = -(1/2) sum_{Q nbr P} a_PQ (lam_P - lam_Q)(w_P - w_Q) / h^2,  a_PQ = e_P e_Q,
// and the transpose of the separable synthesis gives
//   g_kl = sqrt(lambda_kl) sum_j sum_i B[i][k] dU[j][i] B[j][l].
// dU is formed 32 grid rows at a time in LDS (or read from `du`, where the on-chip adjoint solve
// formed it already) and contracted on the FP64 matrix cores:
//   T[j][k] = sum_i dU[j][i] B[i][k] for the block's rows j, then H[k][l] += sum_j T[j][k] B[j][l].
// With B[n - i][k] = (-1)^k B[i][k] the first product runs over the first half of the row only:
// even k take dU[j][i] + dU[j][n - i], odd k dU[j][i] - dU[j][n - i] (i < n/2), and the middle
// node once.  The blocks cover rows 0 .. n-1; row n is summed apart on the vector units.
// A particle whose solves did not converge (iters < 0) gets a NaN gradient.
__global__ __launch_bounds__(256) void gradsynth2d_kernel(const double* __restrict__ e, int64_t e_stride,
                                                          const double* __restrict__ w, int64_t w_stride,
                                                          const double* __restrict__ lam, int64_t lam_stride,
                                                          const int32_t* __restrict__ iters,
                                                          const double* __restrict__ sqrt_lam,
                                                          const double* __restrict__ basis, int n, int kl, int K,
                                                          double* __restrict__ grad, const double* __restrict__ du,
                                                          int64_t du_stride) {
    extern __shared__ double smem[];
    const int np1 = n + 1;
    const int h = n >> 1;
    const int ipad = (np1 + 3) & ~3;
    const int LDD = ipad + 1;
    constexpr int LDT = KLP + 1;
    double* D = smem;                  // [32][LDD] dU of the block's rows
    double* Tb = D + 32 * LDD;         // [32][LDT]
    const int64_t p = blockIdx.x;
    const double* ep = e + p * e_stride;
    const double* wp = w + p * w_stride;
    const double* lp = lam + p * lam_stride;
    const double* dp = du ? du + p * du_stride : nullptr;
    const double scale = -0.5 * (double)n * (double)n;
    // interior values are stored at (j - 1) n + (i - 1); boundary nodes are zero
    auto at = [&](const double* v, int j, int i) -> double {
        return (i >= 1 && i < n && j >= 1 && j < n) ? v[(j - 1) * n + (i - 1)] : 0.0;
    };
    // dPhi/du at node (j, i) from e, w and lam (when the adjoint solve did not form it)
    auto form = [&](int j, int i) -> double {
        const double wP = at(wp, j, i), lP = at(lp, j, i);
        double acc = 0.0;
        if (i > 0) acc += ep[j * np1 + i - 1] * (lP - at(lp, j, i - 1)) * (wP - at(wp, j, i - 1));
        if (i < n) acc += ep[j * np1 + i + 1] * (lP - at(lp, j, i + 1)) * (wP - at(wp, j, i + 1));
        if (j > 0) acc += ep[(j - 1) * np1 + i] * (lP - at(lp, j - 1, i)) * (wP - at(wp, j - 1, i));
        if (j < n) acc += ep[(j + 1) * np1 + i] * (lP - at(lp, j + 1, i)) * (wP - at(wp, j + 1, i));
        return scale * ep[j * np1 + i] * acc;
    };
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const int tj0 = (wave >> 1) * 16, par = wave & 1;          // this wave's T tile: 16 block rows, k = 2 lr + par
    const int hk0 = (wave & 1) * 16, hl0 = (wave >> 1) * 16;   // this wave's H tile (k, l)
    const int nsteps = (h + 1 + 3) >> 2;                       // first-product steps over i = 0 .. h
    d4 hacc[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
    for (int jb = 0; jb < n; jb += 32) {
        if (dp) {   // formed by the adjoint solve: thread t holds column t (and t + 256) of the 32 rows,
                    // all 32 loads in flight before the first store
            const int i = threadIdx.x;
            double v[32];
#pragma unroll
            for (int r = 0; r < 32; ++r) {
                const int j = jb + r;
                const bool ok = j < n && i <= n;
                v[r] = dp[ok ? j * np1 + i : 0];
                v[r] = ok ? v[r] : 0.0;
            }
#pragma unroll
            for (int r = 0; r < 32; ++r)
                if (i < ipad) D[r * LDD + i] = v[r];
            if (i + 256 < ipad) {   // 257 nodes per row at n = 256
#pragma unroll 4
                for (int r = 0; r < 32; ++r) {
                    const int j = jb + r, i2 = i + 256;
                    D[r * LDD + i2] = (j < n && i2 <= n) ? dp[j * np1 + i2] : 0.0;
                }
            }
        }
        for (int t = threadIdx.x; !dp && t < 32 * ipad; t += 256) {
            const int r = t / ipad, i = t % ipad, j = jb + r;
            D[r * LDD + i] = (j < n && i <= n) ? form(j, i) : 0.0;
        }
        __syncthreads();
        {   // T[r][k] = sum_{i <= h} A[r][i] B[i][k] with A = dU[r][i] +- dU[r][n - i] (i < h) or
            // dU[r][h] (i = h); four independent accumulation chains
            const double sgn = par ? -1.0 : 1.0;
            const double* Dr = D + (tj0 + lr) * LDD;
            d4 acc[4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
            for (int s0 = 0; s0 < nsteps; s0 += 4) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (s0 + q < nsteps) {
                        const int ii = 4 * (s0 + q) + lk;
                        const int ic = ii < h ? ii : h;                  // clamped, selected below
                        const double d0 = Dr[ic], d1 = Dr[n - ic];
                        const double av = ii < h ? fma(sgn, d1, d0) : (ii == h ? d0 : 0.0);
                        const double bv = basis[ic * KLP + 2 * lr + par];
                        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[q], 0, 0, 0);
                    }
                }
            }
#pragma unroll
            for (int v = 0; v < 4; ++v)
                Tb[(tj0 + lk + 4 * v) * LDT + 2 * lr + par] = (acc[0][v] + acc[1][v]) + (acc[2][v] + acc[3][v]);
        }
        __syncthreads();
#pragma unroll
        for (int r0 = 0; r0 < 32; r0 += 8) {   // H[k][l] += sum_r T[r][k] B[jb + r][l], two chains
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int jj = jb + r0 + 4 * q + lk;
                const double av = Tb[(r0 + 4 * q + lk) * LDT + hk0 + lr];
                const double bv = (jj < n) ? basis[jj * KLP + hl0 + lr] : 0.0;
                hacc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, hacc[q], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // row n: T[n][k] = sum_i dU[n][i] B[i][k] as eight strided partial sums per k, added in a
    // fixed order, then H[k][l] += T[n][k] B[n][l]
    for (int i = threadIdx.x; i <= n; i += 256) D[i] = dp ? dp[n * np1 + i] : form(n, i);
    __syncthreads();
    {
        const int k = threadIdx.x & 31, c = threadIdx.x >> 5;
        double s = 0.0;
        for (int i = c; i <= n; i += 8) s = fma(D[i], basis[i * KLP + k], s);
        Tb[c * LDT + k] = s;
    }
    __syncthreads();
    const bool bad = iters && iters[p] < 0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int k = hk0 + lk + 4 * v, l = hl0 + lr;
        double tn = 0.0;
#pragma unroll
        for (int c = 0; c < 8; ++c) tn += Tb[c * LDT + k];
        const double g = fma(tn, basis[n * KLP + l], hacc[0][v] + hacc[1][v]);
        if (k < kl && l < kl) grad[p * K + k * kl + l] = bad ? NAN : sqrt_lam[k * kl + l] * g;
    }
}

hipError_t launch_gradsynth2d(const double* e, int64_t e_stride, const double* w, int64_t w_stride,
                              const double* lam, int64_t lam_stride, const int32_t* iters, const double* sqrt_lam,
                              const double* basis, int n, int kl, int K, double* grad, int64_t N, const double* du,
                              int64_t du_stride, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    const int ipad = (n + 1 + 3) & ~3;
    const size_t lds = sizeof(double) * (32 * (size_t)(ipad + 1) + 32 * (size_t)(KLP + 1));
    gradsynth2d_kernel<<<dim3((unsigned)N), dim3(256), lds, s>>>(e, e_stride, w, w_stride, lam, lam_stride, iters,
                                                                 sqrt_lam, basis, n, kl, K, grad, du, du_stride);
    return hipGetLastError();
}

hipError_t launch_synth2d(const double* xi, int K, int kl, const double* sqrt_lam, const double* basis, int n,
                          double* out, int64_t out_stride, int64_t N, bool exp_half, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    const size_t lds = sizeof(double) * (size_t)synth2d_lds_doubles(n);
    if (exp_half)
        synth2d_kernel<true><<<dim3((unsigned)N), dim3(SYN_THREADS), lds, s>>>(xi, K, kl, sqrt_lam, basis, n, out, out_stride);
    else
        synth2d_kernel<false><<<dim3((unsigned)N), dim3(SYN_THREADS), lds, s>>>(xi, K, kl, sqrt_lam, basis, n, out, out_stride);
    return hipGetLastError();
}

hipError_t launch_synth2d_levels(const double* xi, int K, int kl, const double* sqrt_lam, const LevelTable& lt,
                                 const int32_t* level, double* out, int64_t out_stride, int64_t N, bool exp_half,
                                 hipStream_t s) {
    if (N <= 0) return hipSuccess;
    int nmax = 0;
    for (int l = 0; l < lt.n_levels; ++l) nmax = lt.n[l] > nmax ? lt.n[l] : nmax;
    const size_t lds = sizeof(double) * (size_t)synth2d_lds_doubles(nmax);
    if (exp_half)
        synth2d_levels_kernel<true><<<dim3((unsigned)N), dim3(SYN_THREADS), lds, s>>>(xi, K, kl, sqrt_lam, lt, level, out,
                                                                             out_stride);
    else
        synth2d_levels_kernel<false><<<dim3((unsigned)N), dim3(SYN_THREADS), lds, s>>>(xi, K, kl, sqrt_lam, lt, level, out,
                                                                              out_stride);
    return hipGetLastError();
}

// Dynamic LDS limits of the synthesis kernels, set once for the largest grid (256 intervals), so
// that no launch needs an attribute call (launches may be captured into graphs).
hipError_t prepare_kernels() {
    constexpr int ipad = (256 + 1 + 3) & ~3;
    const int synth = (int)sizeof(double) * synth2d_lds_doubles(256);
    const int grad = (int)sizeof(double) * (32 * (ipad + 1) + 32 * (KLP + 1));
    const hipFuncAttribute A = hipFuncAttributeMaxDynamicSharedMemorySize;
    hipError_t e = hipSuccess;
    auto ck = [&](hipError_t r) { if (e == hipSuccess) e = r; };
    ck(hipFuncSetAttribute((const void*)synth2d_kernel<true>, A, synth));
    ck(hipFuncSetAttribute((const void*)synth2d_kernel<false>, A, synth));
    ck(hipFuncSetAttribute((const void*)synth2d_levels_kernel<true>, A, synth));
    ck(hipFuncSetAttribute((const void*)synth2d_levels_kernel<false>, A, synth));
    ck(hipFuncSetAttribute((const void*)gradsynth2d_kernel, A, grad));
    ck(prepare_gmfit_kernels());
    return e;
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
