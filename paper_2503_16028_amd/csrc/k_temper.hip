// Re-weighting, next temperature and systematic resampling (Alg. 1; App. C).
// Both run in one workgroup: the work is a few dozen reductions over N values, so the cost
// is latency, and a single workgroup keeps every reduction in one fixed order.
#include "common.hpp"
#include "stage_graph.hpp"

namespace smc {

constexpr int TB = 1024;
constexpr int TW = TB / 64;

__device__ __forceinline__ double block_max_all(double v, double* red) {
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double m = -INFINITY;
#pragma unroll
    for (int w = 0; w < TW; ++w) m = fmax(m, red[w]);
    __syncthreads();
    return m;
}

// ESS(h) = (sum W)^2 / sum W^2 with W_n = exp(-h d_n), d_n = Phi_n - Phi_min; non-finite Phi weigh 0.
// One pass gives S1 = sum W, S2 = sum W^2, D1 = sum d W, D2 = sum d W^2 and Q = sum d^2 W, so that
//   f(h) = log ESS(h) - log(rho N) = 2 log S1 - log S2 - log(rho N),
//   f'(h) = -2 D1 / S1 + 2 D2 / S2,
// and at h = 0, Q / S1 - (D1 / S1)^2 is the variance of d.  Thread t takes particles t, t + TB, ...;
// their d sit in registers when N <= TCACHE TB, and the sums run in the same order either way.
constexpr int TCACHE = 8;

struct EssSums {
    double s1, s2, d1, d2, q;
};

__device__ EssSums ess_sums(const double* __restrict__ phi, int64_t N, double pmin, double h,
                            const double (&dc)[TCACHE], bool cached, double (*red)[5]) {
    double s1 = 0.0, s2 = 0.0, d1 = 0.0, d2 = 0.0, q = 0.0;
    auto add = [&](double d) {
        const double w = exp(-h * d), ww = w * w;
        s1 += w;
        s2 += ww;
        d1 += d * w;
        d2 += d * ww;
        q += d * d * w;
    };
    if (cached) {
#pragma unroll
        for (int i = 0; i < TCACHE; ++i)
            if (dc[i] >= 0.0) add(dc[i]);
    } else {
        for (int64_t k = threadIdx.x; k < N; k += TB) {
            const double p = phi[k];
            if (isfinite(p)) add(p - pmin);
        }
    }
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    d1 = wave_sum(d1);
    d2 = wave_sum(d2);
    q = wave_sum(q);
    if ((threadIdx.x & 63) == 0) {
        double* r = red[threadIdx.x >> 6];
        r[0] = s1;
        r[1] = s2;
        r[2] = d1;
        r[3] = d2;
        r[4] = q;
    }
    __syncthreads();
    EssSums o{0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int w = 0; w < TW; ++w) {
        o.s1 += red[w][0];
        o.s2 += red[w][1];
        o.d1 += red[w][2];
        o.d2 += red[w][3];
        o.q += red[w][4];
    }
    __syncthreads();   // red is reused by the next pass
    o.s1 = uniform(o.s1);
    o.s2 = uniform(o.s2);
    o.d1 = uniform(o.d1);
    o.d2 = uniform(o.d2);
    o.q = uniform(o.q);
    return o;
}

// Next increment h in (0, 1 - tau]: the whole remaining step if its ESS passes, else the root of
// the decreasing f, kept in a bracket [lo, hi] with f(lo) >= 0 > f(hi).  The first point is the
// root of the expansion f(h) ~ f(0) - h^2 Var(d); then Newton steps in log h (ESS falls off like a
// power of h for spread-out potentials), replaced by the bracket's geometric (or arithmetic) mean
// whenever a step would leave the bracket, until the bracket is 2^-52 relative or the bisection
// resolution (1 - tau) 2^-64 wide.  The returned h always has f(h) >= 0, ESS >= rho N, as the lower
// end of a bisection would; about 10 passes replace 66.  Every thread holds the same sums, so
// every branch below is uniform.
__global__ __launch_bounds__(TB) void temper_kernel(int64_t N, const double* __restrict__ phi,
                                                    const double* __restrict__ tau_in, double ess_frac,
                                                    double* __restrict__ h_out, double* __restrict__ tau_out,
                                                    double* __restrict__ W, double* __restrict__ log_z,
                                                    int32_t* __restrict__ flags) {
    __shared__ double red[TW][5];
    double pmin = INFINITY;
    for (int64_t k = threadIdx.x; k < N; k += TB) {
        const double p = phi[k];
        if (isfinite(p)) pmin = fmin(pmin, p);
    }
    pmin = uniform(-block_max_all(-pmin, &red[0][0]));
    const double tau = *tau_in;
    const double rest = 1.0 - tau;
    if (!isfinite(pmin)) {   // no finite potential: nothing to weigh
        for (int64_t k = threadIdx.x; k < N; k += TB) W[k] = 0.0;
        if (threadIdx.x == 0) {
            *h_out = 0.0;
            *tau_out = tau;
            *log_z = -INFINITY;
            if (flags) atomicOr(flags, SMC_FLAG_NONFINITE);
        }
        return;
    }
    const bool cached = N <= (int64_t)TCACHE * TB;
    double dc[TCACHE];
#pragma unroll
    for (int i = 0; i < TCACHE; ++i) {
        const int64_t k = threadIdx.x + (int64_t)i * TB;
        const double p = (cached && k < N) ? phi[k] : NAN;
        dc[i] = isfinite(p) ? p - pmin : -1.0;
    }
    const double target = log(ess_frac * (double)N);
    auto f_of = [&](const EssSums& e) { return 2.0 * log(e.s1) - log(e.s2) - target; };
    double h;
    bool last = false;
    EssSums e = ess_sums(phi, N, pmin, rest, dc, cached, red);
    if (f_of(e) >= 0.0) {
        h = rest;
        last = true;
    } else {
        double lo = 0.0, hi = rest;
        const double floor_w = rest * 0x1p-64;
        const EssSums e0 = ess_sums(phi, N, pmin, 0.0, dc, cached, red);
        const double f0 = f_of(e0), m = e0.d1 / e0.s1, v = e0.q / e0.s1 - m * m;
        double x = (v > 0.0 && f0 > 0.0) ? fmin(sqrt(f0 / v), 0.5 * rest) : 0.5 * rest;
        for (int it = 0; it < 96; ++it) {
            e = ess_sums(phi, N, pmin, x, dc, cached, red);
            const double fx = f_of(e);
            const bool pass = fx >= 0.0;
            if (pass) lo = x;
            else hi = x;
            if (!(hi - lo > fmax(floor_w, hi * 0x1p-52))) break;
            const double dfx = -2.0 * e.d1 / e.s1 + 2.0 * e.d2 / e.s2;
            const double step = -fx / (dfx * x);   // Newton in s = log h
            double xn = (fabs(step) < 50.0) ? x * exp(step) : NAN;
            if (!(xn > lo && xn < hi)) xn = lo > 0.0 ? sqrt(lo * hi) : 0.5 * (lo + hi);
            if (fabs(xn - x) <= fmax(floor_w, xn * 0x1p-52)) {   // converged next to the root
                if (pass) break;
                xn = fmax(lo, x * (1.0 - 0x1p-46));           // the root lies just below x
            }
            x = xn;
        }
        h = lo;
    }
    e = ess_sums(phi, N, pmin, h, dc, cached, red);   // normaliser at the chosen h
    const double ls1 = log(e.s1);
    for (int64_t k = threadIdx.x; k < N; k += TB) {
        const double p = phi[k];
        W[k] = isfinite(p) ? exp(-h * (p - pmin) - ls1) : 0.0;
    }
    if (threadIdx.x == 0) {
        *h_out = h;
        *tau_out = last ? 1.0 : tau + h;
        *log_z = -h * pmin + ls1 - log((double)N);
        if (h == 0.0 && rest > 0.0 && flags) atomicOr(flags, SMC_FLAG_STALL);   // tau = 1: nothing left
    }
}

hipError_t launch_temper(int64_t N, const double* phi, const double* tau_in, double ess_frac, double* h,
                         double* tau_new, double* W, double* log_z, int32_t* flags, hipStream_t s) {
    temper_kernel<<<dim3(1), dim3(TB), 0, s>>>(N, phi, tau_in, ess_frac, h, tau_new, W, log_z, flags);
    return hipGetLastError();
}

// Systematic resampling on integers: q_n = floor(W_n 2^53), inclusive scan C, Q = C_{N-1};
// idx_i = min{n : C_n > floor(T_i Q / D)} with T_i = i 2^53 + u53 and D = N 2^53.  For an
// integer C, C > floor(x) iff C > x, so output i belongs to particle n exactly when
// C_{n-1} D <= T_i Q < C_n D: every particle owns a contiguous range of outputs, starting at
//   first(C_{n-1}) = min{i : T_i Q >= C_{n-1} D} = ceil(C_{n-1} N / Q - u53 / 2^53),
// evaluated exactly on 128-bit integers.  One workgroup; thread t owns a contiguous chunk of
// particles: their integer weights are summed, the thread totals scanned, and a second pass
// writes each particle's range.  Integer sums make the result independent of summation order,
// and no CDF is stored, so N is limited only by the 32-bit output indices.
//
// The weights must be normalised: each W_n in [0, 1] and finite, and their sum at most
// 1 + 2N 2^-53 (the rounding of a normalisation in FP64), so that every q_n <= 2^53 and
// Q <= QMAX = 2^53 + 2N.  A thread stops adding once its total passes QMAX (one more addend of
// at most 2^53 cannot overflow 64 bits), and the scan adds at most TB totals of at most
// QMAX + 2^53 < 2^55 each.  Any weight outside [0, 1] (NaN included) or Q > QMAX sets
// SMC_FLAG_BADWEIGHTS and gives idx = 0..N-1, as do all-zero weights.
__device__ __forceinline__ bool weight_ok(double w) { return w >= 0.0 && w <= 1.0; }   // false for NaN

__device__ __forceinline__ uint64_t qweight53(double w) { return (uint64_t)(w * 9007199254740992.0); }

// min{i >= 0 : (i 2^53 + u53) Q >= C N 2^53} = q + [r 2^53 > u53 Q], where C N = q Q + r
// (0 <= r < Q); q <= N, found from a double estimate and corrected exactly.
__device__ __forceinline__ int64_t first_output(uint64_t C, int64_t N, uint64_t Q, uint64_t u53) {
    const unsigned __int128 A = (unsigned __int128)C * (uint64_t)N;
    int64_t q = (int64_t)floor((double)C * (double)N / (double)Q);
    if (q < 0) q = 0;
    while ((unsigned __int128)(q + 1) * Q <= A) ++q;
    while (q > 0 && (unsigned __int128)q * Q > A) --q;
    const unsigned __int128 r = A - (unsigned __int128)q * Q;
    return q + ((r << 53) > (unsigned __int128)u53 * Q ? 1 : 0);
}

// With ctr_dev the uniform is drawn here, as smc_philox_u53(seed, *ctr_dev + ctr_off) draws it on
// the host: the first two words of the counter block RESAMPLE_BLOCK, 27 + 26 bits.
__global__ __launch_bounds__(TB) void resample_kernel(int64_t N, const double* __restrict__ W, uint64_t u53,
                                                      uint64_t seed, const uint64_t* ctr_dev, uint64_t ctr_off,
                                                      int32_t* __restrict__ idx, int32_t* __restrict__ flags) {
    __shared__ uint64_t part[TB];
    __shared__ int bad;
    const int tid = threadIdx.x;
    if (ctr_dev) {
        const uint4 w = draw(seed, *ctr_dev + ctr_off, RESAMPLE_BLOCK, 0u);
        u53 = ((uint64_t)(w.x >> 5) << 26) | (uint64_t)(w.y >> 6);
    }
    if (tid == 0) bad = 0;
    __syncthreads();
    const int64_t per = (N + TB - 1) / TB;
    const int64_t beg = tid * per, end = beg + per < N ? beg + per : N;
    const uint64_t qmax = (1ull << 53) + 2ull * (uint64_t)N;
    uint64_t run = 0;
    bool ok = true;
    for (int64_t n = beg; n < end && ok; ++n) {
        const double w = W[n];
        ok = weight_ok(w);
        if (ok) run += qweight53(w);
        ok = ok && run <= qmax;
    }
    if (!ok) bad = 1;
    part[tid] = run;
    __syncthreads();
    // inclusive scan of the per-thread totals (Hillis-Steele on TB entries)
    for (int off = 1; off < TB; off <<= 1) {
        const uint64_t v = (tid >= off) ? part[tid - off] : 0ull;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    const uint64_t Q = part[TB - 1];
    if (__builtin_amdgcn_readfirstlane(bad) || Q == 0 || Q > qmax) {
        for (int64_t i = tid; i < N; i += TB) idx[i] = (int32_t)i;
        if (tid == 0 && flags) atomicOr(flags, SMC_FLAG_BADWEIGHTS);
        return;
    }
    uint64_t C = (tid > 0) ? part[tid - 1] : 0ull;   // C_{beg-1}
    int64_t lo = first_output(C, N, Q, u53);
    for (int64_t n = beg; n < end; ++n) {
        C += qweight53(W[n]);
        const int64_t hi = first_output(C, N, Q, u53);
        for (int64_t i = lo; i < hi; ++i) idx[i] = (int32_t)n;
        lo = hi;
    }
}

hipError_t launch_resample(int64_t N, const double* W, uint64_t u53, int32_t* idx, int32_t* flags, hipStream_t s) {
    resample_kernel<<<dim3(1), dim3(TB), 0, s>>>(N, W, u53, 0, nullptr, 0, idx, flags);
    return hipGetLastError();
}

hipError_t launch_resample_ctr(int64_t N, const double* W, uint64_t seed, const uint64_t* ctr, uint64_t ctr_off,
                               int32_t* idx, int32_t* flags, hipStream_t s) {
    resample_kernel<<<dim3(1), dim3(TB), 0, s>>>(N, W, 0, seed, ctr, ctr_off, idx, flags);
    return hipGetLastError();
}

// End of a tempering stage for G samplers, one workgroup: for every group still running (its first
// row not parked; always, without a level map) the acceptance rate of its moves (an integer sum),
// a record of the stage (tau, h, the beta the moves used, the rate, the log-evidence increment) at
// row ctr / stride - 1, then the step-size rule (double beta above a rate of 0.3, halve it below
// 0.15, at most 1), and a group whose temperature has reached 1 parks its rows.  Last, the counter
// moves to the next stage.
__global__ __launch_bounds__(TB) void stage_rule_kernel(StageRule r) {
    __shared__ unsigned long long part[TB];
    const int tid = threadIdx.x;
    const uint64_t c = *r.ctr;
    const int64_t row = (int64_t)(c / r.stride) - 1;
    for (int g = 0; g < r.G; ++g) {
        const int64_t off = r.off[g], n = r.count[g];
        const bool running = !r.level || r.level[off] != SMC_LEVEL_PARKED;   // uniform
        if (!running) continue;
        unsigned long long a = 0;
        for (int64_t k = tid; k < n; k += TB) a += (unsigned long long)r.n_acc[off + k];
        part[tid] = a;
        __syncthreads();
        for (int w = TB / 2; w > 0; w >>= 1) {
            if (tid < w) part[tid] += part[tid + w];
            __syncthreads();
        }
        const unsigned long long acc = part[0];
        __syncthreads();
        const double beta = r.beta[g], tau = r.tau[g];
        if (tid == 0) {
            const double rate = (double)acc / ((double)n * (double)(r.n_moves > 1 ? r.n_moves : 1));
            if (row >= 0 && row < r.max_stages) {
                double* rec = r.record + ((size_t)row * r.G + g) * 5;
                rec[0] = tau;
                rec[1] = r.h[g];
                rec[2] = beta;
                rec[3] = rate;
                rec[4] = r.log_z[g];
            }
            r.beta[g] = rate > 0.3 ? fmin(1.0, 2.0 * beta) : (rate < 0.15 ? 0.5 * beta : beta);
        }
        if (r.level && tau >= 1.0)
            for (int64_t k = tid; k < n; k += TB) r.level[off + k] = SMC_LEVEL_PARKED;
        __syncthreads();
    }
    __syncthreads();   // every thread has read the counter (the loop may have had no barrier)
    if (tid == 0) *r.ctr = c + r.stride;
}

hipError_t launch_stage_rule(const StageRule& r, hipStream_t s) {
    stage_rule_kernel<<<dim3(1), dim3(TB), 0, s>>>(r);
    return hipGetLastError();
}

}  // namespace smc
