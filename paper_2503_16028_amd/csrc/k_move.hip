// Particle-level kernels of the move stage: prior draw, potential, the proposal's mixture table,
// pCN-GM proposal with its acceptance ratio, Metropolis accept/reject (one workgroup per particle
// above 128 modes, sixteen lanes per particle up to 128), the mixture draw of SMC-GM, and the
// pCN-Langevin proposal and decision, and the row gather after resampling.
#include "common.hpp"
#include "move_body.hpp"

namespace smc {

// xi[N][K] ~ N(0, I): normal i of particle n is element i % 2 of block i / 2.
__global__ __launch_bounds__(256) void prior_kernel(int64_t N, int K, uint64_t seed, uint64_t ctr,
                                                    double* __restrict__ xi) {
    const int nb = (K + 1) / 2;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= N * nb) return;
    const int64_t n = t / nb;
    const int blk = (int)(t % nb);
    double z0, z1;
    box_muller(draw(seed, ctr, (uint32_t)blk, (uint32_t)n), z0, z1);
    xi[n * K + 2 * blk] = z0;
    if (2 * blk + 1 < K) xi[n * K + 2 * blk + 1] = z1;
}

hipError_t launch_prior(int64_t N, int K, uint64_t seed, uint64_t ctr, double* xi, hipStream_t s) {
    const int64_t work = N * ((K + 1) / 2);
    if (work <= 0) return hipSuccess;
    prior_kernel<<<dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s>>>(N, K, seed, ctr, xi);
    return hipGetLastError();
}

// Phi = |G - y|^2 / (2 sigma^2), +inf for a non-finite row (Sec. 2.1).
__global__ __launch_bounds__(256) void potential_kernel(int64_t N, int n_obs, const double* __restrict__ G,
                                                        const double* __restrict__ y, double inv2s2,
                                                        double* __restrict__ phi) {
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    double s = 0.0;
    bool fin = true;
    for (int k = 0; k < n_obs; ++k) {
        const double g = G[n * n_obs + k];
        fin = fin && isfinite(g);
        s += (g - y[k]) * (g - y[k]);
    }
    phi[n] = fin ? s * inv2s2 : INFINITY;
}

hipError_t launch_potential(int64_t N, int n_obs, const double* G, const double* y, double inv2s2, double* phi,
                            hipStream_t s) {
    if (N <= 0) return hipSuccess;
    potential_kernel<<<dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s>>>(N, n_obs, G, y, inv2s2, phi);
    return hipGetLastError();
}

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k < n) p[k] = v;
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    fill_i32_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(p, n, v);
    return hipGetLastError();
}

// Mixture component of particle n: j = min{j : w_0 + ... + w_j > U_comp} (U_comp from words 0, 1
// of block UNIFORM_BLOCK at counter ctr), the last component if rounding leaves the sum below U.
__device__ __forceinline__ int choose_component(uint64_t seed, uint64_t ctr, int64_t n, int M,
                                                const double* __restrict__ logw) {
    const uint4 w = draw(seed, ctr, UNIFORM_BLOCK, (uint32_t)n);
    const double uc = res53(w.x, w.y);
    double cum = 0.0;
    for (int m = 0; m < M; ++m) {
        cum += exp(logw[m]);
        if (cum > uc) return m;
    }
    return M - 1;
}

// pCN-GM proposal (Sec. 2.3, eq. (pCN-GM proposal), component-wise) and its log ratio.
//
// The Metropolis-Hastings ratio rho(dv) Q(v, dxi) / (rho(dxi) Q(xi, dv)) of eq. (auv of
// pCN-GMM) factors into exp(tau (Phi(xi) - Phi(v))) times the ratio R of the two mixture
// joint measures mu_0(dv)Q(v, dxi) / mu_0(dxi)Q(xi, dv) (eq. (auv of pCN-GMM2)).  In whitened
// coordinates the off-mixture modes contribute the symmetric pCN factor, which cancels, and
// subtracting the same symmetric pCN term inside every component leaves
//   log R = LSE_j[log w_j + alpha_j(xi, v)] - LSE_j[log w_j + alpha_j(v, xi)],
//   alpha_j(a, b) = sum_{i active} (a_i - g b_i)^2 / (2 beta^2)
//                   - (a_i - g b_i - (1 - g) m_ji)^2 / (2 beta^2 s_ji) - log(s_ji) / 2,
// a sum over the active modes only (g = gamma).  The first argument of alpha is where the
// reverse move lands.  This is the ratio of the Gaussian components' Radon-Nikodym
// derivatives of eq. (auv of pCN-GMM4) written out for diagonal covariances.
//
// Split as alpha_j(a, b) = (|d|^2 - sum_i (d_i - (1 - g) m_ji)^2 / s_ji) / (2 beta^2) - h_j with
// d = a - g b over the active modes and h_j = sum_i log(s_ji) / 2: |d|^2 is one reduction for
// every component, and 1/s_ji, h_j and the running weight sums that pick the component come from
// a table built once per call (they depend on the mixture only).
__global__ __launch_bounds__(64) void mixtab_kernel(MoveParams q, double* __restrict__ tab) {
    const int g = blockIdx.x, lane = threadIdx.x, M = q.M, kr = q.kr;
    const double* logw = q.logw + (int64_t)g * M;
    const double* scale = q.scale + (int64_t)g * M * kr;
    double* t = tab + (int64_t)g * MIXTAB;
    for (int m = 0; m < M; ++m) {
        double h = 0.0;
        if (lane < kr) {
            const double sv = scale[m * kr + lane];
            t[m * MAX_KR + lane] = 1.0 / sv;
            h = 0.5 * log(sv);
        }
        h = wave_sum(h);
        if (lane == 0) t[MAX_M * MAX_KR + m] = h;
    }
    if (lane == 0) {   // the same running sum as choose_component, so the same component is picked
        double cum = 0.0;
        for (int m = 0; m < M; ++m) {
            cum += exp(logw[m]);
            t[MAX_M * MAX_KR + MAX_M + m] = cum;
        }
    }
}

hipError_t launch_mixtab(const MoveParams& q, double* tab, hipStream_t s) {
    mixtab_kernel<<<dim3((unsigned)q.n_groups), dim3(64), 0, s>>>(q, tab);
    return hipGetLastError();
}

template <int NT>
__global__ __launch_bounds__(NT) void propose_kernel(int K, const int32_t* __restrict__ active,
                                                      const int32_t* __restrict__ slot, MoveParams q,
                                                      const double* __restrict__ tab,
                                                      const double* __restrict__ xi, double* __restrict__ v,
                                                      double* __restrict__ logr, int32_t* flags) {
    propose_body<NT>(blockIdx.x, K, active, slot, q, tab, xi, v, logr, flags);
}

// Log-sum-exp over a particle's 16 lanes, each holding one value (-inf for none).
__device__ __forceinline__ double lse16(double x) {
    double mx = x;
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 16));
    double e = (x > -INFINITY) ? exp(x - mx) : 0.0;
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) e += __shfl_xor(e, off, 16);
    return mx + log(e);
}

__device__ __forceinline__ double sum16(double v) {
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off, 16);
    return v;
}

// The same proposal for K <= 128 modes: sixteen lanes per particle (four particles per wave,
// sixteen per workgroup); a lane draws normal blocks sub, sub + 16, ... and holds the active
// slots sub, sub + 16, ... (at most four), so each component's two sums are 16-lane butterflies.
constexpr int P16_SLOTS = MAX_KR / 16;
__global__ __launch_bounds__(256) void propose16_kernel(int64_t N, int K, const int32_t* __restrict__ active,
                                                        const int32_t* __restrict__ slot, MoveParams q,
                                                        const double* __restrict__ tab,
                                                        const double* __restrict__ xi, double* __restrict__ v,
                                                        double* __restrict__ logr, int32_t* flags) {
    const int sub = threadIdx.x & 15;
    const int64_t n = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
    const bool live = n < N;
    const int grp = live ? mp_group(q, n) : -1;
    const double beta = grp >= 0 ? mp_beta(q, grp) : 0.0, tau = grp >= 0 ? mp_tau(q, grp) : 0.0;
    const bool valid = grp >= 0 && mp_valid(beta, tau);
    const double* xp = xi + (live ? n : 0) * K;
    double* vp = v + (live ? n : 0) * K;
    const int M = q.M, kr = q.kr;
    const double gamma = valid ? sqrt(1.0 - beta * beta) : 0.0;
    const double* logw = q.logw + (int64_t)(grp >= 0 ? grp : 0) * M;
    const double* mean = q.mean + (int64_t)(grp >= 0 ? grp : 0) * M * kr;
    const double* scale = q.scale + (int64_t)(grp >= 0 ? grp : 0) * M * kr;
    const double* invs = tab + (int64_t)(grp >= 0 ? grp : 0) * MIXTAB;
    const double* half_logs = invs + MAX_M * MAX_KR;
    const double* cumw = half_logs + MAX_M;
    const uint64_t ctr = mp_ctr(q);
    if (live && !valid) {   // no valid parameters: propose the current state, reject it
        for (int k = sub; k < K; k += 16) vp[k] = xp[k];
        if (sub == 0) {
            logr[n] = -INFINITY;
            if (grp >= 0 && flags) atomicOr(flags, SMC_FLAG_BADPARAM);
        }
    }
    if (valid) {
        int j = M - 1;   // component: the first whose running weight sum exceeds U_comp
        const uint4 w = draw(q.seed, ctr, UNIFORM_BLOCK, (uint32_t)n);
        const double uc = res53(w.x, w.y);
        for (int m = 0; m < M; ++m)
            if (cumw[m] > uc) {
                j = m;
                break;
            }
        const int nb = (K + 1) / 2;
        for (int blk = sub; blk < nb; blk += 16) {
            double z[2];
            box_muller(draw(q.seed, ctr, (uint32_t)blk, (uint32_t)n), z[0], z[1]);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int k = 2 * blk + h;
                if (k >= K) break;
                const int sl = slot[k];
                double val = gamma * xp[k] + beta * z[h];
                if (sl >= 0) {
                    const double mj = mean[j * kr + sl], sj = scale[j * kr + sl];
                    val = gamma * xp[k] + (1.0 - gamma) * mj + beta * sqrt(sj) * z[h];
                }
                vp[k] = val;
            }
        }
    }
    __syncthreads();   // every thread reaches it; the proposals are read back by the particle's lanes
    if (!valid) return;
    const double inv2b2 = 0.5 / (beta * beta), omg = 1.0 - gamma;
    double d1[P16_SLOTS], d2[P16_SLOTS];   // reverse (xi - g v) and forward (v - g xi) displacements
    double pnf = 0.0, pnb = 0.0;
#pragma unroll
    for (int s = 0; s < P16_SLOTS; ++s) {
        const int i = sub + 16 * s;
        d1[s] = 0.0;
        d2[s] = 0.0;
        if (i < kr) {
            const int k = active[i];
            const double a_x = xp[k], a_v = vp[k];
            d1[s] = a_x - gamma * a_v;
            d2[s] = a_v - gamma * a_x;
        }
        pnf += d1[s] * d1[s];
        pnb += d2[s] * d2[s];
    }
    const double nf = sum16(pnf), nbk = sum16(pnb);
    double mf = -INFINITY, mb = -INFINITY;   // lane m: log w_m + alpha_m(xi, v), log w_m + alpha_m(v, xi)
    for (int m = 0; m < M; ++m) {
        double pf = 0.0, pb = 0.0;
#pragma unroll
        for (int s = 0; s < P16_SLOTS; ++s) {
            const int i = sub + 16 * s;
            if (i < kr) {
                const double mm = omg * mean[m * kr + i], is = invs[m * MAX_KR + i];
                const double e1 = d1[s] - mm, e2 = d2[s] - mm;
                pf += e1 * e1 * is;
                pb += e2 * e2 * is;
            }
        }
        pf = sum16(pf);
        pb = sum16(pb);
        if (sub == m) {
            const double lw = logw[m] - half_logs[m];
            mf = lw + (nf - pf) * inv2b2;
            mb = lw + (nbk - pb) * inv2b2;
        }
    }
    const double lf = lse16(mf), lb = lse16(mb);
    if (sub == 0) logr[n] = lf - lb;
}

hipError_t launch_propose(int64_t N, int K, const int32_t* active, const int32_t* slot, const MoveParams& q,
                          const double* tab, const double* xi, double* v, double* logr, int32_t* flags,
                          hipStream_t s) {
    if (N <= 0) return hipSuccess;
    if (K <= 128)
        propose16_kernel<<<dim3((unsigned)((N + 15) / 16)), dim3(256), 0, s>>>(N, K, active, slot, q, tab, xi, v, logr,
                                                                               flags);
    else
        propose_kernel<256><<<dim3((unsigned)N), dim3(256), 0, s>>>(K, active, slot, q, tab, xi, v, logr, flags);
    return hipGetLastError();
}

// Independent draws from the mixture, the mutation of SMC-GM (Alg. 3): the pCN-GM proposal with
// beta = 1 (Sec. 2.4, eq. (GMM beta=1)), where gamma = 0 drops the current state, so
// v = m_j + sqrt(s_j) z on the active modes and v = z elsewhere; the component and the normals are
// the ones a pCN-GM move of the same particle would draw at this counter.
template <int NT>
__global__ __launch_bounds__(NT) void gm_draw_kernel(int K, const int32_t* __restrict__ slot, uint64_t seed,
                                                      uint64_t ctr, int M, int kr, const double* __restrict__ logw,
                                                      const double* __restrict__ mean,
                                                      const double* __restrict__ scale, double* __restrict__ v) {
    __shared__ int comp;
    const int64_t n = blockIdx.x;
    if (threadIdx.x == 0) comp = choose_component(seed, ctr, n, M, logw);
    __syncthreads();
    const int j = comp;
    double* vp = v + n * K;
    const int nb = (K + 1) / 2;
    for (int blk = threadIdx.x; blk < nb; blk += NT) {
        double z[2];
        box_muller(draw(seed, ctr, (uint32_t)blk, (uint32_t)n), z[0], z[1]);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int k = 2 * blk + h;
            if (k >= K) break;
            const int sl = slot[k];
            vp[k] = sl >= 0 ? mean[j * kr + sl] + sqrt(scale[j * kr + sl]) * z[h] : z[h];
        }
    }
}

hipError_t launch_gm_draw(int64_t N, int K, const int32_t* slot, uint64_t seed, uint64_t ctr, int M, int kr,
                          const double* logw, const double* mean, const double* scale, double* v, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    if (K <= 128)
        gm_draw_kernel<64><<<dim3((unsigned)N), dim3(64), 0, s>>>(K, slot, seed, ctr, M, kr, logw, mean, scale, v);
    else
        gm_draw_kernel<256><<<dim3((unsigned)N), dim3(256), 0, s>>>(K, slot, seed, ctr, M, kr, logw, mean, scale, v);
    return hipGetLastError();
}

template <int NT>
__global__ __launch_bounds__(NT) void accept_kernel(int K, MoveParams q, const double* __restrict__ v,
                                                     const double* __restrict__ logr,
                                                     const double* __restrict__ phinew, double* __restrict__ xi,
                                                     double* __restrict__ phi, int32_t* __restrict__ n_acc) {
    __shared__ int acc;
    accept_body<NT>(blockIdx.x, K, q, v, logr, phinew, xi, phi, n_acc, acc);
}

// The same decision for K <= 128 modes, sixteen lanes per particle: every lane takes the same
// decision from the same uniform and copies every sixteenth mode of an accepted proposal.
__global__ __launch_bounds__(256) void accept16_kernel(int64_t N, int K, MoveParams q, const double* __restrict__ v,
                                                       const double* __restrict__ logr,
                                                       const double* __restrict__ phinew, double* __restrict__ xi,
                                                       double* __restrict__ phi, int32_t* __restrict__ n_acc) {
    const int sub = threadIdx.x & 15;
    const int64_t n = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
    if (n >= N) return;
    const int grp = mp_group(q, n);
    const uint4 w = draw(q.seed, mp_ctr(q), UNIFORM_BLOCK, (uint32_t)n);
    const double ua = res53(w.z, w.w);
    const double pn = phinew[n], lr = logr[n];
    bool ok = false;
    if (grp >= 0 && isfinite(pn) && lr > -INFINITY) {
        const double la = fmin(0.0, mp_tau(q, grp) * (phi[n] - pn) + lr);
        ok = log(ua) < la;
    }
    if (!ok) return;
    for (int k = sub; k < K; k += 16) xi[n * K + k] = v[n * K + k];
    if (sub == 0) {
        phi[n] = pn;
        n_acc[n] += 1;
    }
}

hipError_t launch_accept(int64_t N, int K, const MoveParams& q, const double* v, const double* logr,
                         const double* phinew, double* xi, double* phi, int32_t* n_acc, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    if (K <= 128)
        accept16_kernel<<<dim3((unsigned)((N + 15) / 16)), dim3(256), 0, s>>>(N, K, q, v, logr, phinew, xi, phi, n_acc);
    else
        accept_kernel<256><<<dim3((unsigned)N), dim3(256), 0, s>>>(K, q, v, logr, phinew, xi, phi, n_acc);
    return hipGetLastError();
}

// pCN-Langevin proposal in whitened coordinates (Sec. 2.4 names the move; App. B gives the
// Langevin equation and its Crank-Nicolson step, here with the tempered potential's drift kept
// explicit):  v = gamma xi - (1 - gamma) tau g(xi) + beta z,  g = grad_xi Phi,  gamma^2 + beta^2 = 1.
// Normal i of a particle is element i % 2 of block i / 2, as for the prior draw.
__global__ __launch_bounds__(256) void pcnl_propose_kernel(int64_t N, int K, double beta, double tau, uint64_t seed,
                                                           uint64_t ctr, const double* __restrict__ xi,
                                                           const double* __restrict__ grad,
                                                           double* __restrict__ v) {
    const int nb = (K + 1) / 2;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= N * nb) return;
    const int64_t n = t / nb;
    const int blk = (int)(t % nb);
    const double gamma = sqrt(1.0 - beta * beta), drift = (1.0 - gamma) * tau;
    double z[2];
    box_muller(draw(seed, ctr, (uint32_t)blk, (uint32_t)n), z[0], z[1]);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int k = 2 * blk + h;
        if (k < K) v[n * K + k] = gamma * xi[n * K + k] - drift * grad[n * K + k] + beta * z[h];
    }
}

hipError_t launch_pcnl_propose(int64_t N, int K, double beta, double tau, uint64_t seed, uint64_t ctr,
                               const double* xi, const double* grad, double* v, hipStream_t s) {
    const int64_t work = N * ((K + 1) / 2);
    if (work <= 0) return hipSuccess;
    pcnl_propose_kernel<<<dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s>>>(N, K, beta, tau, seed, ctr, xi,
                                                                                  grad, v);
    return hipGetLastError();
}

// pCN-Langevin decision: the Metropolis-Hastings ratio of Sec. 2.3 with the Langevin kernel,
// i.e. the plain ratio of densities in whitened coordinates,
//   log r = [-tau Phi(v) - |v|^2/2 - |xi - m(v)|^2 / (2 beta^2)]
//         - [-tau Phi(xi) - |xi|^2/2 - |v - m(xi)|^2 / (2 beta^2)],  m(a) = gamma a - (1 - gamma) tau g(a),
// summed over the K modes in a fixed order; accept iff log U_acc < min(0, log r).  A proposal
// whose forward or adjoint solve failed (iters < 0) or whose potential is not finite is rejected.
__global__ __launch_bounds__(256) void pcnl_accept_kernel(int K, double beta, double tau, uint64_t seed, uint64_t ctr,
                                                          const double* __restrict__ v,
                                                          const double* __restrict__ gnew,
                                                          const double* __restrict__ phinew,
                                                          const int32_t* __restrict__ iters_new,
                                                          double* __restrict__ xi, double* __restrict__ grad,
                                                          double* __restrict__ phi, int32_t* __restrict__ n_acc) {
    __shared__ double red[4];
    __shared__ int acc;
    const int64_t n = blockIdx.x;
    const double gamma = sqrt(1.0 - beta * beta), drift = (1.0 - gamma) * tau;
    const double inv2b2 = 0.5 / (beta * beta);
    const double* xp = xi + n * K;
    const double* gp = grad + n * K;
    const double* vp = v + n * K;
    const double* hp = gnew + n * K;
    double s = 0.0;
    for (int k = threadIdx.x; k < K; k += 256) {
        const double a = xp[k], b = vp[k];
        const double back = a - (gamma * b - drift * hp[k]);   // xi - m(v)
        const double fwd = b - (gamma * a - drift * gp[k]);    // v - m(xi)
        s += 0.5 * (a * a - b * b) + (fwd * fwd - back * back) * inv2b2;
    }
    const double lr = block_sum<4>(s, red);
    if (threadIdx.x == 0) {
        const uint4 wd = draw(seed, ctr, UNIFORM_BLOCK, (uint32_t)n);
        const double ua = res53(wd.z, wd.w);
        const double pn = phinew[n];
        bool ok = false;
        if (isfinite(pn) && iters_new[n] >= 0) {
            const double la = fmin(0.0, tau * (phi[n] - pn) + lr);
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
        for (int k = threadIdx.x; k < K; k += 256) {
            xi[n * K + k] = vp[k];
            grad[n * K + k] = hp[k];
        }
    }
}

hipError_t launch_pcnl_accept(int64_t N, int K, double beta, double tau, uint64_t seed, uint64_t ctr, const double* v,
                              const double* gnew, const double* phinew, const int32_t* iters_new, double* xi,
                              double* grad, double* phi, int32_t* n_acc, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    pcnl_accept_kernel<<<dim3((unsigned)N), dim3(256), 0, s>>>(K, beta, tau, seed, ctr, v, gnew, phinew, iters_new,
                                                               xi, grad, phi, n_acc);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void gather_kernel(int64_t N, int K, const int32_t* __restrict__ idx,
                                                     const double* __restrict__ xi_in,
                                                     const double* __restrict__ phi_in, double* __restrict__ xi_out,
                                                     double* __restrict__ phi_out) {
    const int64_t n = blockIdx.x;
    const int64_t src = idx[n];
    if (src < 0 || src >= N) return;   // indices come from smc_resample; others leave the row untouched
    for (int k = threadIdx.x; k < K; k += 256) xi_out[n * K + k] = xi_in[src * K + k];
    if (threadIdx.x == 0 && phi_in && phi_out) phi_out[n] = phi_in[src];
}

hipError_t launch_gather(int64_t N, int K, const int32_t* idx, const double* xi_in, const double* phi_in,
                         double* xi_out, double* phi_out, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    gather_kernel<<<dim3((unsigned)N), dim3(256), 0, s>>>(N, K, idx, xi_in, phi_in, xi_out, phi_out);
    return hipGetLastError();
}

}  // namespace smc
