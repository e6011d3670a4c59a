// Per-particle bodies of the pCN-GM move, shared by the one-kernel-per-step launches (one
// workgroup per particle) and the persistent stage launch that runs a particle's whole stage.
#pragma once
#include "common.hpp"

namespace smc {

// Log-sum-exp of each half of the wave, every lane of a half holding one value (-inf for none).
__device__ __forceinline__ double half_lse(double x) {
    double mx = x;
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    double e = (x > -INFINITY) ? exp(x - mx) : 0.0;
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
    return mx + log(e);
}

// The proposal of particle n by one workgroup of NT threads (every thread calls it: it has a
// barrier).
template <int NT>
__device__ __forceinline__ void propose_body(int64_t n, int K, const int32_t* __restrict__ active,
                                             const int32_t* __restrict__ slot, const MoveParams& q,
                                             const double* __restrict__ tab, const double* __restrict__ xi,
                                             double* __restrict__ v, double* __restrict__ logr, int32_t* flags) {
    const int grp = mp_group(q, n);
    const double beta = grp >= 0 ? mp_beta(q, grp) : 0.0, tau = grp >= 0 ? mp_tau(q, grp) : 0.0;
    const double* xp = xi + n * K;
    double* vp = v + n * K;
    if (grp < 0 || !mp_valid(beta, tau)) {   // no valid parameters: propose the current state, reject it
        for (int k = threadIdx.x; k < K; k += NT) vp[k] = xp[k];
        if (threadIdx.x == 0) {
            logr[n] = -INFINITY;
            if (grp >= 0 && flags) atomicOr(flags, SMC_FLAG_BADPARAM);
        }
        return;
    }
    const int M = q.M, kr = q.kr;
    const double* logw = q.logw + (int64_t)grp * M;
    const double* mean = q.mean + (int64_t)grp * M * kr;
    const double* scale = q.scale + (int64_t)grp * M * kr;
    const double* invs = tab + (int64_t)grp * MIXTAB;
    const double* half_logs = invs + MAX_M * MAX_KR;
    const double* cumw = half_logs + MAX_M;
    const uint64_t ctr = mp_ctr(q);
    const double gamma = sqrt(1.0 - beta * beta);
    int j = M - 1;   // component: the first whose running weight sum exceeds U_comp (every lane alike)
    {
        const uint4 w = draw(q.seed, ctr, UNIFORM_BLOCK, (uint32_t)n);
        const double uc = res53(w.x, w.y);
        for (int m = 0; m < M; ++m)
            if (cumw[m] > uc) {
                j = m;
                break;
            }
    }
    const int nb = (K + 1) / 2;
    for (int blk = threadIdx.x; blk < nb; blk += NT) {
        double z[2];
        box_muller(draw(q.seed, ctr, (uint32_t)blk, (uint32_t)n), z[0], z[1]);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int k = 2 * blk + h;
            if (k >= K) break;
            const int sl = slot[k];
            double val = gamma * xp[k] + beta * z[h];
            if (sl >= 0) {
                const double m = mean[j * kr + sl], s = scale[j * kr + sl];
                val = gamma * xp[k] + (1.0 - gamma) * m + beta * sqrt(s) * z[h];
            }
            vp[k] = val;
        }
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const double inv2b2 = 0.5 / (beta * beta), omg = 1.0 - gamma;
        double d1 = 0.0, d2 = 0.0;   // reverse (xi - g v) and forward (v - g xi) displacements
        if (lane < kr) {
            const int k = active[lane];
            const double a_x = xp[k], a_v = vp[k];
            d1 = a_x - gamma * a_v;
            d2 = a_v - gamma * a_x;
        }
        const double nf = wave_sum(d1 * d1), nbk = wave_sum(d2 * d2);
        double mine = -INFINITY;   // lane m: alpha_m(xi, v) + log w_m; lane 32 + m: alpha_m(v, xi) + log w_m
        for (int m = 0; m < M; ++m) {
            double pf = 0.0, pb = 0.0;
            if (lane < kr) {
                const double mm = omg * mean[m * kr + lane], is = invs[m * MAX_KR + lane];
                const double e1 = d1 - mm, e2 = d2 - mm;
                pf = e1 * e1 * is;
                pb = e2 * e2 * is;
            }
            pf = wave_sum(pf);
            pb = wave_sum(pb);
            const double lw = logw[m] - half_logs[m];
            if (lane == m) mine = lw + (nf - pf) * inv2b2;
            if (lane == 32 + m) mine = lw + (nbk - pb) * inv2b2;
        }
        const double lse = half_lse(mine);
        const double lse_b = __shfl(lse, 32, 64);
        if (lane == 0) logr[n] = lse - lse_b;
    }
}

// Metropolis-Hastings decision (Alg. 2): log a = min(0, tau (Phi(xi) - Phi(v)) + log R);
// accept iff log U_acc < log a; a proposal without a finite potential or log R is rejected.
// Particle n by one workgroup of NT threads; acc is a workgroup-shared int (every thread calls it).
template <int NT>
__device__ __forceinline__ void accept_body(int64_t n, int K, const MoveParams& q, const double* __restrict__ v,
                                            const double* __restrict__ logr, const double* __restrict__ phinew,
                                            double* __restrict__ xi, double* __restrict__ phi,
                                            int32_t* __restrict__ n_acc, int& acc) {
    if (threadIdx.x == 0) {
        const int grp = mp_group(q, n);
        const uint4 w = draw(q.seed, mp_ctr(q), UNIFORM_BLOCK, (uint32_t)n);
        const double ua = res53(w.z, w.w);
        const double pn = phinew[n], lr = logr[n];
        bool ok = false;
        if (grp >= 0 && isfinite(pn) && lr > -INFINITY) {
            const double la = fmin(0.0, mp_tau(q, grp) * (phi[n] - pn) + lr);
            ok = log(ua) < la;
        }
        acc = ok;
        if (ok) {
            phi[n] = pn;
            n_acc[n] += 1;
        }
    }
    __syncthreads();
    if (acc) {
        for (int k = threadIdx.x; k < K; k += NT) xi[n * K + k] = v[n * K + k];
    }
}

}  // namespace smc
