// Re-weighting, next temperature and systematic resampling (Alg. 1; App. C).
// Both run in one workgroup: the work is a few dozen reductions over N values, so the cost
// is latency, and a single workgroup keeps every reduction in one fixed order.
#include "common.hpp"

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

// ESS(h) = (sum W)^2 / sum W^2 with W_n = exp(-h (Phi_n - Phi_min)); non-finite Phi weigh 0.
// Returns log S1 (into *ls1) and log ESS.
__device__ double log_ess(const double* phi, int64_t N, double pmin, double h, double* ls1, double* red1,
                          double* red2) {
    double s1 = 0.0, s2 = 0.0;
    for (int64_t k = threadIdx.x; k < N; k += TB) {
        const double p = phi[k];
        if (isfinite(p)) {
            const double w = exp(-h * (p - pmin));
            s1 += w;
            s2 += w * w;
        }
    }
    const double S1 = block_sum<TW>(s1, red1);
    const double S2 = block_sum<TW>(s2, red2);
    __syncthreads();   // red1/red2 are reused by the next call
    *ls1 = log(S1);
    return 2.0 * log(S1) - log(S2);
}

__global__ __launch_bounds__(TB) void temper_kernel(int64_t N, const double* __restrict__ phi,
                                                    const double* __restrict__ tau_in, double ess_frac,
                                                    double* __restrict__ h_out, double* __restrict__ tau_out,
                                                    double* __restrict__ W, double* __restrict__ log_z,
                                                    int32_t* __restrict__ flags) {
    __shared__ double red1[TW], red2[TW];
    double pmin = INFINITY;
    for (int64_t k = threadIdx.x; k < N; k += TB) {
        const double p = phi[k];
        if (isfinite(p)) pmin = fmin(pmin, p);
    }
    pmin = -block_max_all(-pmin, red1);
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
    const double target = log(ess_frac * (double)N);
    double ls1;
    double h;
    bool last = false;
    if (log_ess(phi, N, pmin, rest, &ls1, red1, red2) >= target) {
        h = rest;
        last = true;
    } else {
        double lo = 0.0, hi = rest;
        for (int it = 0; it < 64; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (log_ess(phi, N, pmin, mid, &ls1, red1, red2) >= target) lo = mid;
            else hi = mid;
        }
        h = lo;
    }
    log_ess(phi, N, pmin, h, &ls1, red1, red2);   // normaliser at the chosen h
    for (int64_t k = threadIdx.x; k < N; k += TB) {
        const double p = phi[k];
        W[k] = isfinite(p) ? exp(-h * (p - pmin) - ls1) : 0.0;
    }
    if (threadIdx.x == 0) {
        *h_out = h;
        *tau_out = last ? 1.0 : tau + h;
        *log_z = -h * pmin + ls1 - log((double)N);
        if (h == 0.0 && flags) atomicOr(flags, SMC_FLAG_STALL);
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
__device__ __forceinline__ uint64_t qweight53(double w) {
    return (w > 0.0 && w <= 1.0) ? (uint64_t)(w * 9007199254740992.0) : 0ull;
}

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

__global__ __launch_bounds__(TB) void resample_kernel(int64_t N, const double* __restrict__ W, uint64_t u53,
                                                      int32_t* __restrict__ idx, int32_t* __restrict__ flags) {
    __shared__ uint64_t part[TB];
    const int tid = threadIdx.x;
    const int64_t per = (N + TB - 1) / TB;
    const int64_t beg = tid * per, end = beg + per < N ? beg + per : N;
    uint64_t run = 0;
    for (int64_t n = beg; n < end; ++n) run += qweight53(W[n]);
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
    if (Q == 0) {
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
    resample_kernel<<<dim3(1), dim3(TB), 0, s>>>(N, W, u53, idx, flags);
    return hipGetLastError();
}

}  // namespace smc
