// Per-particle body of the 2D Karhunen-Loeve synthesis (two FP64 matrix-core products), shared by
// the synthesis kernels and the persistent stage launch.
#pragma once
#include "common.hpp"

namespace smc {

typedef double d4 __attribute__((ext_vector_type(4)));

// Waves of a 2D synthesis workgroup: the kernel alternates matrix-core, exponential and store
// phases and is bound by their latency, so eight waves share one workgroup's LDS (the 33 KB of
// one particle's intermediate product at 128^2: four workgroups, 32 waves, per compute unit).
// LDS doubles a 2D synthesis of an n-interval grid needs.
__host__ __device__ constexpr int synth2d_lds_doubles(int n) {
    return KLP * (KLP + 1) > KLP * (n + 1) ? KLP * (KLP + 1) : KLP * (n + 1);
}
constexpr int SYN_WAVES = 8;
constexpr int SYN_THREADS = 64 * SYN_WAVES;

// MFMA f64 16x16x4 operand layout (one double per lane), checked on the device:
//   A[16][4]: lane = row + 16 * k     B[4][16]: lane = col + 16 * k
//   D[16][16]: lane = col + 16 * (row % 4), element row / 4
// The cosine basis is symmetric about the middle node, B[n - i][k] = (-1)^k B[i][k], so a product
// over the modes splits into its even-mode part E and odd-mode part O, and node i and its mirror
// n - i take E + O and E - O: each product runs over the first half of an axis only (nodes
// i < n/2), with the middle node n/2 and the last row summed apart on the vector units.
// One particle by one workgroup of NWAVES waves (every thread calls it: it has barriers).
template <bool EXPHALF, int NWAVES = SYN_WAVES>
__device__ __forceinline__ void synth2d_body(const double* __restrict__ xp, int kl, const double* __restrict__ sqrt_lam,
                                             const double* __restrict__ basis, int n, double* __restrict__ op,
                                             double* smem) {
    constexpr int NTH = 64 * NWAVES;
    const int np1 = n + 1;
    const int h = n >> 1;                       // nodes i < h pair with n - i; node h is its own mirror
    constexpr int LD = KLP + 1;                 // padded row stride of X: conflict-free column reads
    constexpr int KH = KLP / 8;                 // MFMA steps over the 16 even (or odd) modes of an axis
    // Products of the first stage per wave, held in registers until X is dead: 2 n / 16 units
    // (n <= 256, the largest 2D grid) over at least 8 waves
    constexpr int MAXU = 2;
    static_assert(NWAVES >= 8, "first-stage units of a 256-interval grid: 2 per wave need 8 waves");
    double* X = smem;                           // [KLP][LD], the first stage's operand
    double* T = smem;                           // [KLP][n + 1], written over X after the first stage
    auto out = [&](double v) { return EXPHALF ? exp(0.5 * v) : v; };

    for (int t = threadIdx.x; t < KLP * KLP; t += NTH) {
        const int k = t / KLP, l = t % KLP;
        X[k * LD + l] = (k < kl && l < kl) ? sqrt_lam[k * kl + l] * xp[k * kl + l] : 0.0;
    }
    __syncthreads();

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const int nhb = (h + 15) >> 4;              // 16-node blocks of the first half of an axis
    // B operands of the 16 nodes r0 .. r0+15, straight from the (cache-resident) basis table:
    // be[s] = B[r0 + lr][2 (4 s + lk)], bo[s] = B[r0 + lr][2 (4 s + lk) + 1]; nodes past the half
    // read a clamped row and only feed result columns that are not stored
    auto bfrag = [&](int r0, double (&be)[KH], double (&bo)[KH]) {
        const int r = r0 + lr, rc = r < h ? r : h - 1;
#pragma unroll
        for (int s2 = 0; s2 < KH; ++s2) {
            be[s2] = basis[rc * KLP + 8 * s2 + 2 * lk];
            bo[s2] = basis[rc * KLP + 8 * s2 + 2 * lk + 1];
        }
    };
    // T[k][j] = sum_l X[k][l] B[j][l] for j < h (E + O) and its mirror n - j (E - O); a wave
    // takes the units (node block, 16 modes k) = wave, wave + NWAVES
    d4 tp[MAXU], tm[MAXU];
#pragma unroll
    for (int q = 0; q < MAXU; ++q) {
        const int u = wave + q * NWAVES;
        if (u < 2 * nhb) {
            const int jb = u >> 1, k0 = 16 * (u & 1);
            double be[KH], bo[KH];
            bfrag(16 * jb, be, bo);
            d4 ae = {0.0, 0.0, 0.0, 0.0}, ao = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s2 = 0; s2 < KH; ++s2) {
                ae = __builtin_amdgcn_mfma_f64_16x16x4f64(X[(k0 + lr) * LD + 8 * s2 + 2 * lk], be[s2], ae, 0, 0, 0);
                ao = __builtin_amdgcn_mfma_f64_16x16x4f64(X[(k0 + lr) * LD + 8 * s2 + 2 * lk + 1], bo[s2], ao, 0, 0, 0);
            }
            tp[q] = ae + ao;
            tm[q] = ae - ao;
        }
    }
    // the middle column T[k][h], on the last wave (the one with the fewest units)
    double mid = 0.0;
    if (wave == NWAVES - 1 && lane < KLP) {
#pragma unroll 8
        for (int l = 0; l < KLP; ++l) mid = fma(X[lane * LD + l], basis[h * KLP + l], mid);
    }
    __syncthreads();   // X is dead: T takes its place
#pragma unroll
    for (int q = 0; q < MAXU; ++q) {
        const int u = wave + q * NWAVES;
        const int jb = u >> 1, k0 = 16 * (u & 1), j = 16 * jb + lr;
        if (u < 2 * nhb && j < h) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int k = k0 + lk + 4 * v;
                T[k * np1 + j] = tp[q][v];
                T[k * np1 + n - j] = tm[q][v];
            }
        }
    }
    if (wave == NWAVES - 1 && lane < KLP) T[lane * np1 + h] = mid;
    __syncthreads();
    // U[j][i] = sum_k T[k][j] B[i][k] for rows j < n and columns i < h and n - i; a wave takes
    // the units (row block jb, column block ib) = wave, wave + NWAVES, ... and reloads its B
    // operands only when its column block changes
    const int njb = (n + 15) >> 4;
    int ib_held = -1;
    double be[KH], bo[KH];
    for (int u = wave; u < njb * nhb; u += NWAVES) {
        const int ib = u % nhb, jb = u / nhb;
        const int jc = 16 * jb + lr < n ? 16 * jb + lr : n;   // rows past n (none when 16 | n) are not stored
        if (ib != ib_held) {
            bfrag(16 * ib, be, bo);
            ib_held = ib;
        }
        d4 ae = {0.0, 0.0, 0.0, 0.0}, ao = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s2 = 0; s2 < KH; ++s2) {
            ae = __builtin_amdgcn_mfma_f64_16x16x4f64(T[(8 * s2 + 2 * lk) * np1 + jc], be[s2], ae, 0, 0, 0);
            ao = __builtin_amdgcn_mfma_f64_16x16x4f64(T[(8 * s2 + 2 * lk + 1) * np1 + jc], bo[s2], ao, 0, 0, 0);
        }
        const int i = 16 * ib + lr;
        if (i < h) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int j = 16 * jb + lk + 4 * v;
                if (j < n) {
                    op[j * np1 + i] = out(ae[v] + ao[v]);
                    op[j * np1 + n - i] = out(ae[v] - ao[v]);
                }
            }
        }
    }
    // the last row U[n][i] (i <= n) and the middle column U[j][h] (j < n) on the vector units
    for (int t = threadIdx.x; t < 2 * n + 1; t += NTH) {
        const bool last_row = t <= n;
        const int i = last_row ? t : h, j = last_row ? n : t - np1;
        double s = 0.0;
#pragma unroll 8
        for (int k = 0; k < KLP; ++k) s = fma(T[k * np1 + j], basis[i * KLP + k], s);
        op[j * np1 + i] = out(s);
    }
}

}  // namespace smc
