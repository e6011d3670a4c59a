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
// s_j = max(sum_n R_nj x_n^2 / N_j - m_j^2, floor).
//
// Layout of the work: every pass over the cloud runs on workgroups of 64 particles whose active
// coordinates are first staged, transposed, in LDS (lanes read one row's coordinates together).
// Reductions over the cloud leave one partial per workgroup in global memory and a one-workgroup
// kernel adds them in workgroup order, so results never depend on scheduling.  Passing partials
// between kernels, rather than through a last-workgroup handshake inside one kernel, avoids a
// device-scope fence per workgroup (an L2 write-back on this part) in every iteration.
#include <mutex>

#include "common.hpp"
#include "stage_graph.hpp"

namespace smc {

namespace {

constexpr uint32_t KMPP_BLOCK = 0x80000002u;
constexpr int QBITS = 40;
constexpr int EM_P = 64;             // particles per workgroup
constexpr int EM_LDX = EM_P + 1;     // padded row of the transposed particle slice

// Parameter block (GM_PAR doubles, two of them ping-pong between iterations):
//   logw [MAX_M], cst [MAX_M] (log w_j - sum_d log(2 pi s_jd) / 2), mean [MAX_M][MAX_KR],
//   var [MAX_M][MAX_KR], and for the E-step, coordinate-major: meanT [MAX_KR][MAX_M], ivT (1 / var).
constexpr int PAR_LOGW = 0, PAR_CST = MAX_M, PAR_MEAN = 2 * MAX_M, PAR_VAR = PAR_MEAN + MAX_M * MAX_KR,
              PAR_MEANT = PAR_VAR + MAX_M * MAX_KR, PAR_IVT = PAR_MEANT + MAX_KR * MAX_M;
static_assert(PAR_IVT + MAX_KR * MAX_M == GM_PAR, "parameter block layout");

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

// The workgroup's particles [n0, n0 + np) staged transposed: xs[d * EM_LDX + p] = x_{n0+p, d}
// (zero beyond np).  Four waves; the 16 loads of a lane go out before the first store (rows
// clamped into range, zeros selected afterwards).
__device__ __forceinline__ void stage_rows(double* xs, const double* __restrict__ xi, const int32_t* __restrict__ active,
                                           int K, int kr, int64_t n0, int np) {
    constexpr int PER = EM_P / 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int k = active[lane < kr ? lane : 0];
    double v[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int p = wave + 4 * i;
        v[i] = xi[(n0 + (p < np ? p : np - 1)) * K + k];
    }
    if (lane < kr) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int p = wave + 4 * i;
            xs[lane * EM_LDX + p] = p < np ? v[i] : 0.0;
        }
    }
}

// Sum of a[b * stride + e] over b = 0 .. B-1, added in that order; the loads go out 32 at a time.
__device__ __forceinline__ double ordered_sum(const double* __restrict__ a, int B, int64_t stride, int e) {
    double s = 0.0;
    for (int b0 = 0; b0 < B; b0 += 32) {
        double v[32];
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            const int b = b0 + k < B ? b0 + k : B - 1;
            v[k] = a[(int64_t)b * stride + e];
        }
#pragma unroll
        for (int k = 0; k < 32; ++k) s += b0 + k < B ? v[k] : 0.0;
    }
    return s;
}

// Publish parameters held in LDS (lw[M], mu[M][MAX_KR], va[M][MAX_KR]) into a parameter block
// (the LDS arrays must be complete: callers put a barrier before).
__device__ __forceinline__ void publish(double* __restrict__ par, int M, int kr, const double* lw, const double* mu,
                                        const double* va) {
    for (int i = threadIdx.x; i < M * kr; i += blockDim.x) {
        const int j = i / kr, d = i % kr;
        const double m = mu[j * MAX_KR + d], v = va[j * MAX_KR + d];
        par[PAR_MEAN + j * MAX_KR + d] = m;
        par[PAR_VAR + j * MAX_KR + d] = v;
        par[PAR_MEANT + d * MAX_M + j] = m;
        par[PAR_IVT + d * MAX_M + j] = 1.0 / v;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int j = wave; j < M; j += nw) {   // one wave per component, lanes are coordinates
        const double s = wave_sum(lane < kr ? log(2.0 * M_PI * va[j * MAX_KR + lane]) : 0.0);
        if (lane == 0) {
            par[PAR_LOGW + j] = lw[j];
            par[PAR_CST + j] = lw[j] - 0.5 * s;
        }
    }
}

}  // namespace

// ------------------------------------------------------------------ seeding

// d2_n <- min(d2_n, |x_n - x_c|^2) for the last chosen centre c (d2_n <- |x_n - x_c|^2 when m = 1);
// 64 particles per workgroup, one thread per particle after staging.
__global__ __launch_bounds__(256) void kmpp_dist_kernel(int64_t N, int K, int kr, const int32_t* __restrict__ active,
                                                        const double* __restrict__ xi,
                                                        const int32_t* __restrict__ centers, int m,
                                                        double* __restrict__ d2) {
#pragma clang fp contract(off)
    __shared__ double xs[MAX_KR * EM_LDX];
    __shared__ double cs[64];
    const int64_t n0 = (int64_t)blockIdx.x * EM_P;
    const int np = (int)(N - n0 < EM_P ? N - n0 : EM_P);
    stage_rows(xs, xi, active, K, kr, n0, np);
    if (threadIdx.x < 64) {
        const int d = threadIdx.x;
        cs[d] = d < kr ? xi[(int64_t)centers[m - 1] * K + active[d]] : 0.0;
    }
    __syncthreads();
    const int p = threadIdx.x;
    if (p >= np) return;
    double s[32];
#pragma unroll
    for (int d = 0; d < 32; ++d) {
        const double ta = xs[(d < kr ? d : 0) * EM_LDX + p] - cs[d];
        const double tb = xs[(d + 32 < kr ? d + 32 : 0) * EM_LDX + p] - cs[d + 32];
        const double a = d < kr ? ta * ta : 0.0, b = d + 32 < kr ? tb * tb : 0.0;
        s[d] = a + b;
    }
#pragma unroll
    for (int w = 16; w >= 1; w >>= 1)
#pragma unroll
        for (int d = 0; d < w; ++d) s[d] = s[d] + s[d + w];
    const int64_t n = n0 + p;
    d2[n] = (m == 1) ? s[0] : fmin(d2[n], s[0]);
}

// Centre m from d2 (m >= 1) or uniformly (m = 0); one workgroup of 1024 threads.
// The counter is ctr, or *ctr_dev + ctr when ctr_dev is given (a stage replayed from a graph).
__global__ __launch_bounds__(1024) void kmpp_pick_kernel(int64_t N, int m, uint64_t seed, uint64_t ctr,
                                                         const uint64_t* ctr_dev, const double* __restrict__ d2,
                                                         int32_t* centers) {
    __shared__ double red_d[16];
    __shared__ unsigned long long red_q[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t u = kmpp_u53(seed, ctr_dev ? *ctr_dev + ctr : ctr, m);
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

// ------------------------------------------------------------------ EM start

// Column sums of x - c and (x - c)^2 per workgroup (c = the first seeded row, a shift that keeps
// the one-pass variance accurate): part[b][0..kr) and part[b][kr..2kr).
__global__ __launch_bounds__(256) void gm_colstats_kernel(int64_t N, int K, int kr, const int32_t* __restrict__ active,
                                                          const double* __restrict__ xi,
                                                          const int32_t* __restrict__ centers,
                                                          double* __restrict__ part) {
    __shared__ double xs[MAX_KR * EM_LDX];
    __shared__ double red[4][2][64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t n0 = (int64_t)blockIdx.x * EM_P;
    const int np = (int)(N - n0 < EM_P ? N - n0 : EM_P);
    stage_rows(xs, xi, active, K, kr, n0, np);
    __syncthreads();
    double s1 = 0.0, s2 = 0.0;
    if (lane < kr) {
        const double c = xi[(int64_t)centers[0] * K + active[lane]];
        for (int p = 16 * wave; p < 16 * wave + 16 && p < np; ++p) {
            const double t = xs[lane * EM_LDX + p] - c;
            s1 += t;
            s2 += t * t;
        }
    }
    red[wave][0][lane] = s1;
    red[wave][1][lane] = s2;
    __syncthreads();
    if (tid < 2 * kr) {
        const int q = tid / kr, d = tid % kr;
        double s = 0.0;
        for (int w = 0; w < 4; ++w) s += red[w][q][d];
        part[(int64_t)blockIdx.x * 2 * kr + tid] = s;
    }
}

// EM start: w_j = 1/M, m_j = the seeded rows, s_j = max(population variance of the cloud, floor).
__global__ __launch_bounds__(256) void gm_start_kernel(int64_t N, int K, int kr, const int32_t* __restrict__ active,
                                                       const double* __restrict__ xi,
                                                       const int32_t* __restrict__ centers, int M,
                                                       double var_floor, int B, const double* __restrict__ part,
                                                       double* __restrict__ par) {
    __shared__ double lw[MAX_M], mu[MAX_M * MAX_KR], va[MAX_M * MAX_KR], col[2 * MAX_KR];
    const int tid = threadIdx.x;
    if (tid < 2 * kr) col[(tid / kr) * MAX_KR + tid % kr] = ordered_sum(part, B, 2 * kr, tid);
    __syncthreads();
    for (int i = tid; i < M * kr; i += 256) {
        const int j = i / kr, d = i % kr;
        const double m1 = col[d] / (double)N;
        mu[j * MAX_KR + d] = xi[(int64_t)centers[j] * K + active[d]];
        va[j * MAX_KR + d] = fmax(col[MAX_KR + d] / (double)N - m1 * m1, var_floor);
    }
    if (tid < M) lw[tid] = -log((double)M);
    __syncthreads();
    publish(par, M, kr, lw, mu, va);
}

// ------------------------------------------------------------------ EM iterations

// E-step and the M-step's partial sums of one workgroup: part[b][j] = {sum R, sum R x, sum R x^2}
// over its 64 particles (E = 1 + 2 kr entries per component).  MB >= M components are computed
// without branches; those beyond M are masked out of the responsibilities and never written.
template <int MB>
__global__ __launch_bounds__(256) void em_partial_kernel(int64_t N, int K, int kr, const int32_t* __restrict__ active,
                                                         const double* __restrict__ xi, int M,
                                                         const double* __restrict__ par,
                                                         double* __restrict__ part) {
    extern __shared__ double smem[];
    double* xs = smem;                         // [kr][EM_LDX]  the workgroup's particles, transposed
    double* sp = xs + MAX_KR * EM_LDX;         // [4][EM_P][MAX_M]  quarter sums of the E-step, then R
    double* pm = sp + 4 * EM_P * MAX_M;        // [kr][MB]  means, coordinate-major
    double* pv = pm + MAX_KR * MB;             // [kr][MB]  1 / variances
    double* pc = pv + MAX_KR * MB;             // [MB]      log w_j - sum_d log(2 pi s_jd) / 2
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int E = 1 + 2 * kr;
    const int64_t n0 = (int64_t)blockIdx.x * EM_P;
    const int np = (int)(N - n0 < EM_P ? N - n0 : EM_P);
    for (int i = tid; i < kr * MB; i += 256) {   // the parameters go out with the rows' loads
        pm[i] = par[PAR_MEANT + (i / MB) * MAX_M + i % MB];
        pv[i] = par[PAR_IVT + (i / MB) * MAX_M + i % MB];
    }
    if (tid < MB) pc[tid] = par[PAR_CST + tid];
    stage_rows(xs, xi, active, K, kr, n0, np);
    __syncthreads();

    {   // E-step, a quarter of the coordinates per thread (wave); parameters are LDS broadcasts
        const int p = tid & (EM_P - 1), h = __builtin_amdgcn_readfirstlane(tid >> 6);
        const int dlo = h * kr / 4, dhi = (h + 1) * kr / 4;
        double s[MB];
#pragma unroll
        for (int j = 0; j < MB; ++j) s[j] = 0.0;
#pragma unroll 4
        for (int d = dlo; d < dhi; ++d) {
            const double x = xs[d * EM_LDX + p];
#pragma unroll
            for (int j = 0; j < MB; ++j) {
                const double t = x - pm[d * MB + j];
                s[j] += t * t * pv[d * MB + j];
            }
        }
#pragma unroll
        for (int j = 0; j < MB; ++j) sp[(h * EM_P + p) * MAX_M + j] = s[j];
    }
    __syncthreads();
    if (tid < EM_P) {
        const int p = tid;
        double ll[MB];
        double mx = -INFINITY;
#pragma unroll
        for (int j = 0; j < MB; ++j) {
            const double q = ((sp[p * MAX_M + j] + sp[(EM_P + p) * MAX_M + j]) + sp[(2 * EM_P + p) * MAX_M + j]) +
                             sp[(3 * EM_P + p) * MAX_M + j];
            const double v = pc[j] - 0.5 * q;
            ll[j] = j < M ? v : -INFINITY;
            mx = fmax(mx, ll[j]);
        }
        double se = 0.0;
#pragma unroll
        for (int j = 0; j < MB; ++j) se += j < M ? exp(ll[j] - mx) : 0.0;
        const double lse = mx + log(se);
#pragma unroll
        for (int j = 0; j < MB; ++j) sp[p * MAX_M + j] = (p < np && j < M) ? exp(ll[j] - lse) : 0.0;
    }
    __syncthreads();

    // M-step partial sums: wave w takes particles [16 w, 16 w + 16); lanes are coordinates
    double a1[MB], a2[MB], a0 = 0.0;
#pragma unroll
    for (int j = 0; j < MB; ++j) a1[j] = a2[j] = 0.0;
#pragma unroll 4
    for (int p = 16 * wave; p < 16 * wave + 16; ++p) {
        const double x = lane < kr ? xs[lane * EM_LDX + p] : 0.0, xx = x * x;
#pragma unroll
        for (int j = 0; j < MB; ++j) {
            const double r = sp[p * MAX_M + j];
            a1[j] += r * x;
            a2[j] += r * xx;
        }
        if (lane < M) a0 += sp[p * MAX_M + lane];
    }
    __syncthreads();                       // xs and sp are reused for the per-wave partials below
    double* wpart = smem;                  // [4][MAX_M][E]
#pragma unroll
    for (int j = 0; j < MB; ++j) {
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
}

// M-step of component j = blockIdx.x: its partials from B workgroups added in workgroup order,
// then its entries of the next parameter block.  One workgroup per component.
__global__ __launch_bounds__(256) void em_final_kernel(int64_t N, int kr, double var_floor, int B,
                                                       const double* __restrict__ part, double* __restrict__ par) {
    __shared__ double tot[1 + 2 * MAX_KR];
    const int tid = threadIdx.x, lane = tid & 63, j = blockIdx.x;
    const int E = 1 + 2 * kr;
    if (tid < E) tot[tid] = ordered_sum(part + (int64_t)j * E, B, (int64_t)MAX_M * E, tid);
    __syncthreads();
    const double nk = tot[0] + 1e-300;
    const double lw = log(nk / (double)N);
    if (tid < 64) {   // wave 0: lanes are coordinates
        const int d = lane;
        double lg = 0.0;
        if (d < kr) {
            const double m = tot[1 + d] / nk;
            const double v = fmax(tot[1 + kr + d] / nk - m * m, var_floor);
            par[PAR_MEAN + j * MAX_KR + d] = m;
            par[PAR_VAR + j * MAX_KR + d] = v;
            par[PAR_MEANT + d * MAX_M + j] = m;
            par[PAR_IVT + d * MAX_M + j] = 1.0 / v;
            lg = log(2.0 * M_PI * v);
        }
        const double s = wave_sum(lg);
        if (lane == 0) {
            par[PAR_LOGW + j] = lw;
            par[PAR_CST + j] = lw - 0.5 * s;
        }
    }
}

// The fit's outputs from a parameter block: weights normalised (log w_j - LSE_i log w_i), means and
// variances.
__global__ void gm_output_kernel(int M, int kr, const double* __restrict__ par, double* __restrict__ out_logw,
                                 double* __restrict__ out_mean, double* __restrict__ out_scale) {
    for (int i = threadIdx.x; i < M * kr; i += blockDim.x) {
        const int j = i / kr, d = i % kr;
        out_mean[j * kr + d] = par[PAR_MEAN + j * MAX_KR + d];
        out_scale[j * kr + d] = par[PAR_VAR + j * MAX_KR + d];
    }
    if ((int)threadIdx.x < M) {
        double mx = -INFINITY;
        for (int j = 0; j < M; ++j) mx = fmax(mx, par[PAR_LOGW + j]);
        double se = 0.0;
        for (int j = 0; j < M; ++j) se += exp(par[PAR_LOGW + j] - mx);
        out_logw[threadIdx.x] = par[PAR_LOGW + threadIdx.x] - (mx + log(se));
    }
}

static size_t em_smem_bytes() {
    constexpr size_t work = MAX_KR * EM_LDX + 4 * EM_P * MAX_M + 2 * MAX_KR * MAX_M + MAX_M,
                     wpart = 4 * MAX_M * (1 + 2 * MAX_KR);
    return sizeof(double) * (work > wpart ? work : wpart);
}

int64_t em_blocks(int64_t N) { return (N + EM_P - 1) / EM_P; }

namespace {
hipError_t gm_fit(int64_t N, int K, int kr, const int32_t* active, const double* xi, int M, int iters,
                  double var_floor, uint64_t seed, uint64_t ctr, const uint64_t* ctr_dev, const FitWorkspace& w,
                  int32_t* centers, double* logw, double* mean, double* scale, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    const unsigned B = (unsigned)em_blocks(N);
    kmpp_pick_kernel<<<1, 1024, 0, s>>>(N, 0, seed, ctr, ctr_dev, w.d2, centers);
    for (int m = 1; m < M; ++m) {
        kmpp_dist_kernel<<<B, 256, 0, s>>>(N, K, kr, active, xi, centers, m, w.d2);
        kmpp_pick_kernel<<<1, 1024, 0, s>>>(N, m, seed, ctr, ctr_dev, w.d2, centers);
    }
    gm_colstats_kernel<<<B, 256, 0, s>>>(N, K, kr, active, xi, centers, w.part);
    gm_start_kernel<<<1, 256, 0, s>>>(N, K, kr, active, xi, centers, M, var_floor, (int)B, w.part, w.par);
    const size_t lds = em_smem_bytes();
    for (int it = 0; it < iters; ++it) {
        const double* pin = w.par + (it & 1) * GM_PAR;
        double* pout = w.par + ((it + 1) & 1) * GM_PAR;
        if (M <= 4)
            em_partial_kernel<4><<<B, 256, lds, s>>>(N, K, kr, active, xi, M, pin, w.part);
        else if (M <= 8)
            em_partial_kernel<8><<<B, 256, lds, s>>>(N, K, kr, active, xi, M, pin, w.part);
        else
            em_partial_kernel<16><<<B, 256, lds, s>>>(N, K, kr, active, xi, M, pin, w.part);
        em_final_kernel<<<M, 256, 0, s>>>(N, kr, var_floor, (int)B, w.part, pout);
    }
    gm_output_kernel<<<1, 256, 0, s>>>(M, kr, w.par + (iters & 1) * GM_PAR, logw, mean, scale);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_gm_fit(int64_t N, int K, int kr, const int32_t* active, const double* xi, int M, int iters,
                         double var_floor, uint64_t seed, uint64_t ctr, const FitWorkspace& w, int32_t* centers,
                         double* logw, double* mean, double* scale, hipStream_t s) {
    return gm_fit(N, K, kr, active, xi, M, iters, var_floor, seed, ctr, nullptr, w, centers, logw, mean, scale, s);
}

hipError_t launch_gm_fit_ctr(int64_t N, int K, int kr, const int32_t* active, const double* xi, int M, int iters,
                             double var_floor, uint64_t seed, const uint64_t* ctr, uint64_t ctr_off,
                             const FitWorkspace& w, int32_t* centers, double* logw, double* mean, double* scale,
                             hipStream_t s) {
    return gm_fit(N, K, kr, active, xi, M, iters, var_floor, seed, ctr_off, ctr, w, centers, logw, mean, scale, s);
}

// ------------------------------------------------------------------ fit without allocation
// The same fit for callers that cannot allocate device memory (code under graph capture, serving
// loops): its workspace is one fixed array in the library's device image instead of a problem's
// allocation, sized for STATIC_FIT_N particles.  Layout in doubles: d2 [STATIC_FIT_N], two parameter
// blocks [2][GM_PAR], partial sums [em_blocks(STATIC_FIT_N)][MAX_M][1 + 2 MAX_KR], then MAX_M int32
// seeded rows.  Nothing in it must start at zero: every entry a kernel reads was written earlier in
// the same call.  Each device holds its own copy, so concurrent calls on one device share it and race.
namespace {
constexpr int64_t STATIC_FIT_PART = ((STATIC_FIT_N + EM_P - 1) / EM_P) * MAX_M * (1 + 2 * MAX_KR);
constexpr int64_t STATIC_FIT_DOUBLES = STATIC_FIT_N + 2 * GM_PAR + STATIC_FIT_PART + MAX_M / 2;
static_assert(MAX_M % 2 == 0, "seeded rows fill whole doubles");
static __device__ __align__(256) double scratch[STATIC_FIT_DOUBLES];

constexpr int MAX_DEVICES = 64;
double* g_scratch[MAX_DEVICES];   // device address of `scratch` on each device, once resolved
bool g_prepared[MAX_DEVICES];
std::mutex g_scratch_mu;
}  // namespace

size_t static_fit_bytes() { return sizeof(double) * (size_t)STATIC_FIT_DOUBLES; }

// Resolve the device address of the scratch array on the current device (first call per device):
// the array's name in host code is only a host-side handle, so kernels get this address.
static hipError_t static_fit_scratch(double** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch[dev] = (double*)ptr;
    }
    if (!g_prepared[dev]) {   // the E-step's LDS above the default limit, set once per device
        e = prepare_gmfit_kernels();
        if (e != hipSuccess) return e;
        g_prepared[dev] = true;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

hipError_t launch_gm_fit_static(int64_t N, int K, int kr, const int32_t* active, const double* xi, int M, int iters,
                                double var_floor, uint64_t seed, uint64_t ctr, int32_t* centers, double* logw,
                                double* mean, double* scale, hipStream_t s) {
    if (N <= 0 || N > STATIC_FIT_N) return hipErrorInvalidValue;
    double* base = nullptr;
    const hipError_t e = static_fit_scratch(&base);
    if (e != hipSuccess) return e;
    FitWorkspace w{base, base + STATIC_FIT_N, base + STATIC_FIT_N + 2 * GM_PAR};
    int32_t* rows = centers ? centers : (int32_t*)(base + STATIC_FIT_N + 2 * GM_PAR + STATIC_FIT_PART);
    return launch_gm_fit(N, K, kr, active, xi, M, iters, var_floor, seed, ctr, w, rows, logw, mean, scale, s);
}

hipError_t prepare_gmfit_kernels() {
    const hipFuncAttribute A = hipFuncAttributeMaxDynamicSharedMemorySize;
    const int bytes = (int)em_smem_bytes();
    hipError_t e = hipFuncSetAttribute((const void*)em_partial_kernel<4>, A, bytes);
    if (e == hipSuccess) e = hipFuncSetAttribute((const void*)em_partial_kernel<8>, A, bytes);
    if (e == hipSuccess) e = hipFuncSetAttribute((const void*)em_partial_kernel<16>, A, bytes);
    return e;
}

}  // namespace smc
