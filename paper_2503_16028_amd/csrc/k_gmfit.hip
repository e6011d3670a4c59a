// Gaussian-mixture fit of the particle cloud on the device: the stage input of the pCN-GM move
// (Sec. 2.3) and the mutation of SMC-GM (Alg. 3, Sec. 2.4).  The paper takes its estimator from
// its reference [Feng2018] without describing it; this is expectation-maximisation with diagonal
// covariances on the K_r active whitened coordinates, seeded by k-means++ and floored in variance.
//
// Seeding (k-means++): centre 0 is row floor(u_0 N / 2^53); centre m >= 1 is drawn with probability
// proportional to the squared distance d2_n of row n to its nearest centre so far.  The draw is
// exact integer arithmetic: with D = max d2 = f 2^e (f in [1/2, 1)), q_n = floor(d2_n 2^(40 - e)),
// C_n = q_0 + ... + q_n, Q = C_{N-1}, and the centre is min{n : C_n > floor(u_m Q / 2^53)} (row
// floor(u_m N / 2^53) when Q = 0).  u_m is the 53-bit integer of Philox block KMPP_BLOCK, particle
// word m, at the call's counter.  Each squared distance is summed over the coordinates, zero-padded
// to 64, in pairwise halving order (s <- s[:w] + s[w:2w], w = 32 .. 1), without fused products, so
// every d2_n, and with it every choice, is reproducible to the bit.
//
// EM: E-step R_nj = w_j N(x_n; m_j, s_j) / sum_i w_i N(x_n; m_i, s_i) in log space; M-step
// N_j = sum_n R_nj (+1e-300), w_j = N_j / N, m_j = sum_n R_nj x_n / N_j,
// s_j = max(sum_n R_nj x_n^2 / N_j - m_j^2, floor).  One launch per iteration: each workgroup
// reduces 128 particles to partial sums; the last workgroup to finish adds the partials in a fixed
// order (so the result does not depend on scheduling) and writes the next parameters.
#include "common.hpp"

namespace smc {

namespace {

constexpr uint32_t KMPP_BLOCK = 0x80000002u;
constexpr int QBITS = 40;
constexpr int EM_P = 128;            // particles per EM workgroup
constexpr int EM_LDX = EM_P + 1;     // padded row of the transposed particle slice

__device__ __forceinline__ uint64_t kmpp_u53(uint64_t seed, uint64_t ctr, int m) {
    const uint4 w = draw(seed, ctr, KMPP_BLOCK, (uint32_t)m);
    return ((uint64_t)(w.x >> 5) << 26) | (uint64_t)(w.y >> 6);
}

// floor(u X / 2^53) for u < 2^53 and X < 2^63 (the product needs 116 bits)
__device__ __forceinline__ uint64_t scale53(uint64_t u, uint64_t X) {
    return (__umul64hi(u, X) << 11) | ((u * X) >> 53);
}

__device__ __forceinline__ uint64_t qweight(double d2, int shift) {
    return (d2 > 0.0 && d2 < INFINITY) ? (uint64_t)floor(ldexp(d2, shift)) : 0ull;
}

}  // namespace

// d2_n <- min(d2_n, |x_n - x_c|^2) for the last chosen centre c (d2_n <- |x_n - x_c|^2 when m = 1).
__global__ __launch_bounds__(256) void kmpp_dist_kernel(int64_t N, int K, int kr, const int32_t* __restrict__ active,
                                                        const double* __restrict__ xi,
                                                        const int32_t* __restrict__ centers, int m,
                                                        double* __restrict__ d2) {
#pragma clang fp contract(off)
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    const double* x = xi + n * K;
    const double* c = xi + (int64_t)centers[m - 1] * K;
    double s[32];
#pragma unroll
    for (int d = 0; d < 32; ++d) {
        double a = 0.0, b = 0.0;
        if (d < kr) {
            const int k = active[d];
            const double t = x[k] - c[k];
            a = t * t;
        }
        if (d + 32 < kr) {
            const int k = active[d + 32];
            const double t = x[k] - c[k];
            b = t * t;
        }
        s[d] = a + b;
    }
#pragma unroll
    for (int w = 16; w >= 1; w >>= 1)
#pragma unroll
        for (int d = 0; d < w; ++d) s[d] = s[d] + s[d + w];
    d2[n] = (m == 1) ? s[0] : fmin(d2[n], s[0]);
}

// Centre m from d2 (m >= 1) or uniformly (m = 0); one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void kmpp_pick_kernel(int64_t N, int m, uint64_t seed, uint64_t ctr,
                                                         const double* __restrict__ d2, int32_t* centers) {
    __shared__ double red_d[16];
    __shared__ unsigned long long red_q[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t u = kmpp_u53(seed, ctr, m);
    if (m == 0) {
        if (tid == 0) centers[0] = (int32_t)scale53(u, (uint64_t)N);
        return;
    }
    double dm = 0.0;
    for (int64_t n = tid; n < N; n += 1024) {
        const double v = d2[n];
        if (v < INFINITY) dm = fmax(dm, v);
    }
    dm = wave_max(dm);
    if (lane == 0) red_d[wave] = dm;
    __syncthreads();
    dm = 0.0;
    for (int w = 0; w < 16; ++w) dm = fmax(dm, red_d[w]);
    dm = uniform(dm);
    if (!(dm > 0.0)) {   // every row is a centre already
        if (tid == 0) centers[m] = (int32_t)scale53(u, (uint64_t)N);
        return;
    }
    int e;
    (void)frexp(dm, &e);
    const int shift = QBITS - e;
    // thread t owns rows [t L, (t + 1) L): local integer sum, then an exclusive scan over threads
    const int64_t L = (N + 1023) / 1024, lo = tid * L, hi = lo + L < N ? lo + L : N;
    unsigned long long loc = 0;
    for (int64_t n = lo; n < hi; ++n) loc += qweight(d2[n], shift);
    unsigned long long inc = loc;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned long long o = __shfl_up(inc, off, 64);
        if (lane >= off) inc += o;
    }
    if (lane == 63) red_q[wave] = inc;
    __syncthreads();
    unsigned long long before = 0, Q = 0;
    for (int w = 0; w < 16; ++w) {
        if (w < wave) before += red_q[w];
        Q += red_q[w];
    }
    const unsigned long long excl = before + inc - loc;
    const unsigned long long t = scale53(u, Q);
    if (excl <= t && t < excl + loc) {   // exactly one thread: C crosses t inside its rows
        unsigned long long c = excl;
        for (int64_t n = lo; n < hi; ++n) {
            c += qweight(d2[n], shift);
            if (c > t) {
                centers[m] = (int32_t)n;
                break;
            }
        }
    }
}

// EM start: w_j = 1/M, m_j = the seeded rows, s_j = max(population variance of the cloud, floor).
// par[j] = {log w_j, m_j[0..kr), s_j[0..kr)}.  One workgroup of 1024 threads; lanes are coordinates.
__global__ __launch_bounds__(1024) void gm_start_kernel(int64_t N, int K, int kr, const int32_t* __restrict__ active,
                                                        const double* __restrict__ xi,
                                                        const int32_t* __restrict__ centers, int M,
                                                        double var_floor, double* __restrict__ par) {
    __shared__ double red[16][64];
    __shared__ double mu[64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int k = lane < kr ? active[lane] : 0;
    double acc = 0.0;
    if (lane < kr)
        for (int64_t n = wave; n < N; n += 16) acc += xi[n * K + k];
    red[wave][lane] = acc;
    __syncthreads();
    if (tid < 64) {
        double s = 0.0;
        for (int w = 0; w < 16; ++w) s += red[w][tid];
        mu[tid] = s / (double)N;
    }
    __syncthreads();
    const double mean = mu[lane];
    acc = 0.0;
    if (lane < kr)
        for (int64_t n = wave; n < N; n += 16) {
            const double t = xi[n * K + k] - mean;
            acc += t * t;
        }
    __syncthreads();
    red[wave][lane] = acc;
    __syncthreads();
    const int E = 1 + 2 * kr;
    if (tid < kr) {
        double s = 0.0;
        for (int w = 0; w < 16; ++w) s += red[w][tid];
        const double v = fmax(s / (double)N, var_floor);
        for (int j = 0; j < M; ++j) {
            par[j * E + 1 + tid] = xi[(int64_t)centers[j] * K + active[tid]];
            par[j * E + 1 + kr + tid] = v;
        }
    }
    if (tid < M) par[tid * E] = -log((double)M);
}

// One EM iteration (see the file comment).  par_in -> par_out, or -> the outputs when `last`.
__global__ __launch_bounds__(256) void em_iter_kernel(int64_t N, int K, int kr, const int32_t* __restrict__ active,
                                                      const double* __restrict__ xi, int M, double var_floor,
                                                      const double* __restrict__ par_in, double* part,
                                                      unsigned int* counter, int last, double* __restrict__ par_out,
                                                      double* __restrict__ out_logw, double* __restrict__ out_mean,
                                                      double* __restrict__ out_scale) {
    extern __shared__ double smem[];
    double* xs = smem;                         // [kr][EM_LDX]  the workgroup's particles, transposed
    double* ms = xs + MAX_KR * EM_LDX;         // [M][kr]       means
    double* is = ms + MAX_M * MAX_KR;          // [M][kr]       1 / variances
    double* cs = is + MAX_M * MAX_KR;          // [M]           log w_j - sum_d log(2 pi s_jd) / 2
    double* sp = cs + MAX_M;                   // [2][EM_P][M]  half sums of the E-step, then R
    __shared__ int is_last;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int E = 1 + 2 * kr;
    const int64_t n0 = (int64_t)blockIdx.x * EM_P;
    const int np = (int)(N - n0 < EM_P ? N - n0 : EM_P);

    for (int i = tid; i < M * kr; i += 256) {
        const int j = i / kr, d = i % kr;
        ms[j * MAX_KR + d] = par_in[j * E + 1 + d];
        is[j * MAX_KR + d] = 1.0 / par_in[j * E + 1 + kr + d];
    }
    if (tid < M) {
        double s = 0.0;
        for (int d = 0; d < kr; ++d) s += log(2.0 * M_PI * par_in[tid * E + 1 + kr + d]);
        cs[tid] = par_in[tid * E] - 0.5 * s;
    }
    if (lane < kr) {
        const int k = active[lane];
        for (int p = wave; p < EM_P; p += 4) xs[lane * EM_LDX + p] = p < np ? xi[(n0 + p) * K + k] : 0.0;
    }
    __syncthreads();

    {   // E-step, half the coordinates per thread
        const int p = tid & (EM_P - 1), h = tid >> 7;
        const int dlo = h ? kr / 2 : 0, dhi = h ? kr : kr / 2;
        for (int j = 0; j < M; ++j) {
            double s = 0.0;
            for (int d = dlo; d < dhi; ++d) {
                const double t = xs[d * EM_LDX + p] - ms[j * MAX_KR + d];
                s += t * t * is[j * MAX_KR + d];
            }
            sp[(h * EM_P + p) * MAX_M + j] = s;
        }
    }
    __syncthreads();
    if (tid < EM_P) {
        const int p = tid;
        double ll[MAX_M];
        double mx = -INFINITY;
#pragma unroll
        for (int j = 0; j < MAX_M; ++j) {
            if (j < M) {
                ll[j] = cs[j] - 0.5 * (sp[p * MAX_M + j] + sp[(EM_P + p) * MAX_M + j]);
                mx = fmax(mx, ll[j]);
            }
        }
        double se = 0.0;
#pragma unroll
        for (int j = 0; j < MAX_M; ++j)
            if (j < M) se += exp(ll[j] - mx);
        const double lse = mx + log(se);
#pragma unroll
        for (int j = 0; j < MAX_M; ++j)
            if (j < M) sp[p * MAX_M + j] = p < np ? exp(ll[j] - lse) : 0.0;
    }
    __syncthreads();

    // M-step partial sums: wave w takes particles [32 w, 32 w + 32); lanes are coordinates
    double a1[MAX_M], a2[MAX_M], a0 = 0.0;
#pragma unroll
    for (int j = 0; j < MAX_M; ++j) a1[j] = a2[j] = 0.0;
    for (int p = 32 * wave; p < 32 * wave + 32; ++p) {
        const double x = lane < kr ? xs[lane * EM_LDX + p] : 0.0, xx = x * x;
#pragma unroll
        for (int j = 0; j < MAX_M; ++j) {
            if (j < M) {
                const double r = sp[p * MAX_M + j];
                a1[j] += r * x;
                a2[j] += r * xx;
            }
        }
        if (lane < M) a0 += sp[p * MAX_M + lane];
    }
    __syncthreads();                       // xs is reused for the per-wave partials below
    double* wpart = xs;                    // [4][M][E]
#pragma unroll
    for (int j = 0; j < MAX_M; ++j) {
        if (j < M && lane < kr) {
            wpart[(wave * MAX_M + j) * E + 1 + lane] = a1[j];
            wpart[(wave * MAX_M + j) * E + 1 + kr + lane] = a2[j];
        }
    }
    if (lane < M) wpart[(wave * MAX_M + lane) * E] = a0;
    __syncthreads();
    double* bpart = part + (int64_t)blockIdx.x * MAX_M * E;
    for (int i = tid; i < M * E; i += 256) {
        const int j = i / E, e = i % E;
        double s = 0.0;
        for (int w = 0; w < 4; ++w) s += wpart[(w * MAX_M + j) * E + e];
        bpart[j * E + e] = s;
    }
    __threadfence();
    __syncthreads();
    if (tid == 0) is_last = atomicAdd(counter, 1u) == gridDim.x - 1;
    __syncthreads();
    if (!__builtin_amdgcn_readfirstlane(is_last)) return;

    // the last workgroup: add the partials in workgroup order, then the M-step
    __threadfence();
    double* tot = smem;                    // [M][E]
    const int B = gridDim.x;
    for (int i = tid; i < M * E; i += 256) {
        const int j = i / E, e = i % E;
        double s = 0.0;
        for (int b = 0; b < B; ++b) s += part[((int64_t)b * MAX_M + j) * E + e];
        tot[j * E + e] = s;
    }
    __syncthreads();
    double* lw = tot + MAX_M * E;          // [M]
    if (tid < M) {
        const double nk = tot[tid * E] + 1e-300;
        lw[tid] = log(nk / (double)N);
    }
    __syncthreads();
    double lse = 0.0;
    if (last) {
        double mx = -INFINITY;
        for (int j = 0; j < M; ++j) mx = fmax(mx, lw[j]);
        double s = 0.0;
        for (int j = 0; j < M; ++j) s += exp(lw[j] - mx);
        lse = mx + log(s);
    }
    for (int i = tid; i < M * kr; i += 256) {
        const int j = i / kr, d = i % kr;
        const double nk = tot[j * E] + 1e-300;
        const double m = tot[j * E + 1 + d] / nk;
        const double v = fmax(tot[j * E + 1 + kr + d] / nk - m * m, var_floor);
        if (last) {
            out_mean[j * kr + d] = m;
            out_scale[j * kr + d] = v;
        } else {
            par_out[j * E + 1 + d] = m;
            par_out[j * E + 1 + kr + d] = v;
        }
    }
    if (tid < M) {
        if (last)
            out_logw[tid] = lw[tid] - lse;
        else
            par_out[tid * E] = lw[tid];
    }
    if (tid == 0) atomicExch(counter, 0u);   // ready for the next launch (and graph replays)
}

// No EM steps: the start itself, weights normalised.
__global__ void gm_copy_start_kernel(int M, int kr, const double* __restrict__ par, double* __restrict__ out_logw,
                                     double* __restrict__ out_mean, double* __restrict__ out_scale) {
    const int E = 1 + 2 * kr;
    for (int i = threadIdx.x; i < M * kr; i += blockDim.x) {
        const int j = i / kr, d = i % kr;
        out_mean[j * kr + d] = par[j * E + 1 + d];
        out_scale[j * kr + d] = par[j * E + 1 + kr + d];
    }
    if ((int)threadIdx.x < M) out_logw[threadIdx.x] = par[threadIdx.x * E];
}

size_t em_smem_bytes() {
    return sizeof(double) * (MAX_KR * EM_LDX + 2 * MAX_M * MAX_KR + MAX_M + 2 * EM_P * MAX_M);
}

int64_t em_blocks(int64_t N) { return (N + EM_P - 1) / EM_P; }

hipError_t launch_gm_fit(int64_t N, int K, int kr, const int32_t* active, const double* xi, int M, int iters,
                         double var_floor, uint64_t seed, uint64_t ctr, const FitWorkspace& w, int32_t* centers,
                         double* logw, double* mean, double* scale, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    const unsigned gd = (unsigned)((N + 255) / 256);
    kmpp_pick_kernel<<<1, 1024, 0, s>>>(N, 0, seed, ctr, w.d2, centers);
    for (int m = 1; m < M; ++m) {
        kmpp_dist_kernel<<<gd, 256, 0, s>>>(N, K, kr, active, xi, centers, m, w.d2);
        kmpp_pick_kernel<<<1, 1024, 0, s>>>(N, m, seed, ctr, w.d2, centers);
    }
    gm_start_kernel<<<1, 1024, 0, s>>>(N, K, kr, active, xi, centers, M, var_floor, w.par);
    if (iters == 0) {
        gm_copy_start_kernel<<<1, 256, 0, s>>>(M, kr, w.par, logw, mean, scale);
        return hipGetLastError();
    }
    const unsigned B = (unsigned)em_blocks(N);
    const size_t pe = (size_t)MAX_M * (1 + 2 * MAX_KR);
    for (int it = 0; it < iters; ++it) {
        const double* pin = w.par + (it & 1) * pe;
        double* pout = w.par + ((it + 1) & 1) * pe;
        em_iter_kernel<<<B, 256, em_smem_bytes(), s>>>(N, K, kr, active, xi, M, var_floor, pin, w.part, w.counter,
                                                       it == iters - 1, pout, logw, mean, scale);
    }
    return hipGetLastError();
}

hipError_t prepare_gmfit_kernels() {
    return hipFuncSetAttribute((const void*)em_iter_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)em_smem_bytes());
}

}  // namespace smc
