// Per-particle body of the 2D Karhunen-Loeve synthesis (two FP64 matrix-core products), shared by
// the synthesis kernels and the persistent stage launch.
#pragma once
#include "common.hpp"

namespace smc {

typedef double d4 __attribute__((ext_vector_type(4)));

// Waves of a 2D synthesis workgroup: the kernel alternates matrix-core, exponential and store
// phases and is bound by their latency, so eight waves share one workgroup's LDS (three
// workgroups, 24 waves, per compute unit at 128^2).
constexpr int SYN_WAVES = 8;
constexpr int SYN_THREADS = 64 * SYN_WAVES;

// MFMA f64 16x16x4 operand layout (one double per lane), checked on the device:
//   A[16][4]: lane = row + 16 * k     B[4][16]: lane = col + 16 * k
//   D[16][16]: lane = col + 16 * (row % 4), element row / 4
// One particle by one workgroup of NWAVES waves (every thread calls it: it has barriers).
template <bool EXPHALF, int NWAVES = SYN_WAVES>
__device__ __forceinline__ void synth2d_body(const double* __restrict__ xp, int kl, const double* __restrict__ sqrt_lam,
                                             const double* __restrict__ basis, int n, double* __restrict__ op,
                                             double* smem) {
    constexpr int NTH = 64 * NWAVES;
    const int np1 = n + 1;
    const int npad = (np1 + 15) & ~15;
    constexpr int LD = KLP + 1;                 // padded row stride: conflict-free column reads
    constexpr int KS = KLP / 4;                 // MFMA steps over the 32 modes of an axis
    double* X = smem;                           // [KLP][LD]
    double* T = X + KLP * LD;                   // [KLP][npad]

    for (int t = threadIdx.x; t < KLP * KLP; t += NTH) {
        const int k = t / KLP, l = t % KLP;
        X[k * LD + l] = (k < kl && l < kl) ? sqrt_lam[k * kl + l] * xp[k * kl + l] : 0.0;
    }
    __syncthreads();

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const int ntj = npad / 16;
    // B operand of the 16 grid nodes r0 .. r0+15, straight from the (cache-resident) basis table:
    // b[s] = B[r0 + lr][4 s + lk], zero past the last node (rows clamped, zeros selected after)
    auto bfrag = [&](int r0, double (&b)[KS]) {
        const int r = r0 + lr, rc = r < np1 ? r : np1 - 1;
#pragma unroll
        for (int s2 = 0; s2 < KS; ++s2) {
            const double v = basis[rc * KLP + 4 * s2 + lk];
            b[s2] = r < np1 ? v : 0.0;
        }
    };
    // T[k][j] = sum_l X[k][l] B[j][l]; a wave takes node blocks jb = wave, wave + NWAVES, ...
    for (int jb = wave; jb < ntj; jb += NWAVES) {
        double b[KS];
        bfrag(16 * jb, b);
#pragma unroll
        for (int k0 = 0; k0 < KLP; k0 += 16) {
            d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s2 = 0; s2 < KS; ++s2)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(X[(k0 + lr) * LD + 4 * s2 + lk], b[s2], acc, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 4; ++v) T[(k0 + lk + 4 * v) * npad + 16 * jb + lr] = acc[v];
        }
    }
    __syncthreads();
    // U[j][i] = sum_k T[k][j] B[i][k]; a wave keeps the B operand of its column block ib and
    // sweeps the row blocks
    for (int ib = wave; ib < ntj; ib += NWAVES) {
        double b[KS];
        bfrag(16 * ib, b);
        const int i = 16 * ib + lr;
        for (int jb = 0; jb < ntj; ++jb) {
            d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s2 = 0; s2 < KS; ++s2)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(T[(4 * s2 + lk) * npad + 16 * jb + lr], b[s2], acc, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int j = 16 * jb + lk + 4 * v;
                if (i < np1 && j < np1) op[j * np1 + i] = EXPHALF ? exp(0.5 * acc[v]) : acc[v];
            }
        }
    }
}

}  // namespace smc
