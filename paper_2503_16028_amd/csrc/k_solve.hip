// Forward solve of the Darcy problem, one workgroup per particle.
//
// Operator (flux form, h = 1/n, geometric-mean faces):
//   (A w)_P = sum_Q a_PQ (w_P - w_Q) / h^2,   a_PQ = e_P e_Q,  e = exp(u/2),
// at interior nodes, w = 0 on the boundary; the PDE is -div(e^u grad w) = f (Sec. 3.2).
//
// Method: conjugate gradients on the symmetrically Jacobi-scaled system
//   A^ y = D^{-1/2} r,  A^ = D^{-1/2} A D^{-1/2},  D = diag(A),
// (unit diagonal, so the preconditioner costs nothing), run inside an FP64 residual
// refinement loop: each sweep forms r = f - A x with the FP64 operator, solves the scaled
// correction in precision T to a relative reduction, and adds it to the FP64 iterate.  The
// loop stops on the FP64 residual, ||f - A x|| <= tol64 ||f||, so the accuracy is set by the
// FP64 operator whatever T is.
//
// Data layout inside a workgroup (on-chip variant): thread t owns column c = t % n of the
// padded n x n node block (x-node i = c + 1) and a strip of R consecutive rows
// (y-nodes j = (t / n) R + 1 ..).  Nodes with i = n or j = n are boundary padding and stay 0.
// Vertical neighbours are in the thread's registers; horizontal neighbours come through LDS:
// every iteration each thread publishes p and s = a^_E p (the flux coefficient times p), so
// the west term a^_W p_W of a node is read as one value written by its left neighbour.
// Dot products are wave butterflies plus a fixed-order sum over waves: every thread sees the
// same bits and a particle's result does not depend on the batch it is solved in.
#include "common.hpp"

namespace smc {

template <typename T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };

template <typename T, int NN, int R>
__global__ __launch_bounds__(NN * NN / R) void cg_onchip(SolveArgs a) {
    constexpr int NT = NN * NN / R;
    constexpr int NW = NT / 64;
    constexpr int NP1 = NN + 1;
    using T2 = typename Vec2<T>::type;
    // (p, s) pairs of the n x n block, with one zero row (plus one element) of padding on each
    // side so that every neighbour read is in bounds: reads that fall on padding, on the
    // boundary-padding column or row, or across a row end meet zero p or zero coefficients.
    constexpr int PAD = NN + 1;
    __shared__ T2 lps[PAD + NN * NN + PAD];
    __shared__ double red1[NW], red2[NW];

    const int tid = threadIdx.x;
    const int c = tid % NN, b = tid / NN;
    const int i = c + 1;
    const int64_t row = blockIdx.x;
    const double* e = a.e + row * a.e_stride;
    double* x64 = a.x64 + row * a.x_stride;
    double* sd = a.sd + row * a.x_stride;
    const double inv_h2 = (double)NN * (double)NN;
    // own node of row r: tb[NN + 1 + r * NN]; east +1, west -1, north/south +-NN
    T2* tb = lps + PAD + b * R * NN + c - NN - 1;
    for (int k = tid; k < PAD; k += NT) {
        lps[k] = T2{T(0), T(0)};
        lps[PAD + NN * NN + k] = T2{T(0), T(0)};
    }

    // ---- setup: Jacobi scaling and the scaled face coefficients.  The per-node work outside
    // the conjugate-gradient loop runs as plain (not unrolled) loops that stage values through
    // the thread's own LDS slots, so only the loop's register arrays stay live across it.
#pragma unroll 1
    for (int r = 0; r < R; ++r) {
        const int g = b * R + r, j = g + 1;
        double v = 1.0;
        if (c < NN - 1 && g < NN - 1) {
            const double d = e[j * NP1 + i] *
                             (e[j * NP1 + i + 1] + e[j * NP1 + i - 1] + e[(j + 1) * NP1 + i] + e[(j - 1) * NP1 + i]) *
                             inv_h2;
            v = 1.0 / sqrt(d);
        }
        sd[g * NN + c] = v;
    }
    __syncthreads();
#pragma unroll 1
    for (int r = 0; r < R; ++r) {
        const int g = b * R + r, j = g + 1;
        T vae = T(0), van = T(0);
        if (c < NN - 1 && g < NN - 1) {
            const double eP = e[j * NP1 + i], sP = sd[g * NN + c];
            if (c + 1 < NN - 1) vae = (T)(eP * e[j * NP1 + i + 1] * inv_h2 * sP * sd[g * NN + c + 1]);
            if (g + 1 < NN - 1) van = (T)(eP * e[(j + 1) * NP1 + i] * inv_h2 * sP * sd[(g + 1) * NN + c]);
        }
        tb[NN + 1 + r * NN] = T2{vae, van};
    }
    T ae[R], an[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const T2 v = tb[NN + 1 + r * NN];
        ae[r] = v.x;
        an[r] = v.y;
    }
    T anS = T(0);
    {
        const int g0 = b * R;
        if (c < NN - 1 && g0 < NN - 1 && g0 >= 1)
            anS = (T)(e[g0 * NP1 + i] * e[(g0 + 1) * NP1 + i] * inv_h2 * sd[(g0 - 1) * NN + c] * sd[g0 * NN + c]);
    }
    __syncthreads();

    // ---- refinement sweeps
    const double fnorm = fabs(a.f) * (double)(NN - 1);
    int total = 0, sweeps = 0;
    bool ok = false;
    T x[R], rv[R], p[R], q[R];
    for (int sweep = 0;; ++sweep) {
        sweeps = sweep;
        // FP64 residual r = f - A x, scaled by D^{-1/2} into the thread's LDS slots
        double acc = 0.0;
#pragma unroll 1
        for (int r = 0; r < R; ++r) {
            const int g = b * R + r, j = g + 1;
            T out = T(0);
            if (c < NN - 1 && g < NN - 1) {
                double res = a.f;
                if (sweep > 0) {
                    const double xP = x64[g * NN + c];
                    const double xE = (c + 1 < NN - 1) ? x64[g * NN + c + 1] : 0.0;
                    const double xW = (c > 0) ? x64[g * NN + c - 1] : 0.0;
                    const double xN = (g + 1 < NN - 1) ? x64[(g + 1) * NN + c] : 0.0;
                    const double xS = (g > 0) ? x64[(g - 1) * NN + c] : 0.0;
                    const double eP = e[j * NP1 + i];
                    res -= eP * inv_h2 *
                           (e[j * NP1 + i + 1] * (xP - xE) + e[j * NP1 + i - 1] * (xP - xW) +
                            e[(j + 1) * NP1 + i] * (xP - xN) + e[(j - 1) * NP1 + i] * (xP - xS));
                }
                acc += res * res;
                out = (T)(sd[g * NN + c] * res);
            }
            tb[NN + 1 + r * NN].x = out;
        }
        const double rr64 = block_sum<NW>(acc, red2);
        if (sqrt(rr64) <= a.tol64 * fnorm) { ok = true; break; }
        if (!(rr64 < INFINITY) || sweep >= a.max_sweeps || total >= a.max_iter) break;

        // inner conjugate gradients on the scaled system, in precision T
        double tacc = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            rv[r] = tb[NN + 1 + r * NN].x;
            x[r] = T(0);
            p[r] = rv[r];
            tacc += (double)rv[r] * (double)rv[r];
        }
        double rr = block_sum<NW>(tacc, red1);
        const double target = a.tol_inner * a.tol_inner * rr;
        bool broke = false;
        while (rr > target) {
            if (total >= a.max_iter) break;
#pragma unroll
            for (int r = 0; r < R; ++r) tb[NN + 1 + r * NN] = T2{p[r], ae[r] * p[r]};
            __syncthreads();
            // q = A^ p: unit diagonal, east/north from p, west/south as published flux terms.
            // Faces touching the boundary padding have zero coefficients and padding holds
            // p = 0, so padding nodes get q = 0 with no branches.
            T pq_acc = T(0);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const T pE = tb[NN + 2 + r * NN].x;
                const T sW = tb[NN + r * NN].y;
                const T pN = (r + 1 < R) ? p[r + 1] : tb[NN + 1 + R * NN].x;
                const T sS = (r > 0) ? an[r - 1] * p[r - 1] : anS * tb[1].x;
                q[r] = p[r] - ae[r] * pE - sW - an[r] * pN - sS;
                pq_acc += p[r] * q[r];
            }
            const double pq = block_sum<NW>((double)pq_acc, red1);
            if (!(pq > 0.0) || !(pq < INFINITY)) { broke = true; break; }
            const T alpha = (T)(rr / pq);
            T r_acc = T(0);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                x[r] += alpha * p[r];
                rv[r] -= alpha * q[r];
                r_acc += rv[r] * rv[r];
            }
            const double rrn = block_sum<NW>((double)r_acc, red2);
            const T beta = (T)(rrn / rr);
            rr = rrn;
#pragma unroll
            for (int r = 0; r < R; ++r) p[r] = rv[r] + beta * p[r];
            ++total;
        }
        // x64 += D^{-1/2} y through the thread's own LDS slots (the stencil reads of other
        // threads finished before the last reduction's barrier)
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r) tb[NN + 1 + r * NN].x = x[r];
#pragma unroll 1
        for (int r = 0; r < R; ++r) {
            const int g = b * R + r;
            const double corr = sd[g * NN + c] * (double)tb[NN + 1 + r * NN].x;
            x64[g * NN + c] = (sweep == 0) ? corr : x64[g * NN + c] + corr;
        }
        __syncthreads();
        if (broke) break;
    }

    // ---- observation, potential, bookkeeping
    __syncthreads();
    double val = 0.0;
    if (tid < a.n_obs) {
        const int node = a.obs[tid];
        const int jj = node / NP1, ii = node % NP1;
        if (ii >= 1 && ii <= NN - 1 && jj >= 1 && jj <= NN - 1) val = x64[(jj - 1) * NN + ii - 1];
        if (!ok) val = NAN;
        if (a.G) a.G[row * a.n_obs + tid] = val;
    }
    if (tid < 64) {
        const double dlt = (tid < a.n_obs) ? val - a.y[tid] : 0.0;
        const double s = wave_sum(dlt * dlt);
        if (tid == 0) {
            if (a.phi) a.phi[row] = ok ? s * a.inv2s2 : INFINITY;
            if (a.iters) a.iters[row] = ok ? total : -1;
            if (!ok) atomicOr(a.flags, SMC_FLAG_NOCONV);
            if (a.stats) {
                atomicAdd(&a.stats[0], (unsigned long long)total);
                atomicAdd(&a.stats[1], (unsigned long long)(sweeps + 1));
                atomicAdd(&a.stats[2], 1ull);
            }
        }
    }
}

// Same method with every vector in global memory, for grids whose vectors do not fit in one
// workgroup's registers and LDS.  1024 threads stride over the nodes of one particle.
template <typename T>
__global__ __launch_bounds__(1024) void cg_global(SolveArgs a, int NN) {
    constexpr int NW = 16;
    __shared__ double red1[NW], red2[NW];
    const int tid = threadIdx.x;
    const int NP1 = NN + 1;
    const int nodes = NN * NN;
    const int64_t row = blockIdx.x;
    const double* e = a.e + row * a.e_stride;
    double* x64 = a.x64 + row * a.x_stride;
    double* sd = a.sd + row * a.x_stride;
    T* vb = reinterpret_cast<T*>(reinterpret_cast<double*>(a.vec) + row * a.vec_stride);
    T* ae = vb;
    T* an = vb + nodes;
    T* xv = vb + 2 * nodes;
    T* rv = vb + 3 * nodes;
    T* pv = vb + 4 * nodes;
    T* qv = vb + 5 * nodes;
    const double inv_h2 = (double)NN * (double)NN;
    auto interior = [&](int g, int c) { return c < NN - 1 && g < NN - 1; };

    for (int k = tid; k < nodes; k += 1024) {
        const int g = k / NN, c = k % NN, i = c + 1, j = g + 1;
        double v = 1.0;
        if (interior(g, c)) {
            const double d = e[j * NP1 + i] *
                             (e[j * NP1 + i + 1] + e[j * NP1 + i - 1] + e[(j + 1) * NP1 + i] + e[(j - 1) * NP1 + i]) *
                             inv_h2;
            v = 1.0 / sqrt(d);
        }
        sd[k] = v;
    }
    __syncthreads();
    for (int k = tid; k < nodes; k += 1024) {
        const int g = k / NN, c = k % NN, i = c + 1, j = g + 1;
        T vae = T(0), van = T(0);
        if (interior(g, c)) {
            const double eP = e[j * NP1 + i], sP = sd[k];
            if (c + 1 < NN - 1) vae = (T)(eP * e[j * NP1 + i + 1] * inv_h2 * sP * sd[k + 1]);
            if (g + 1 < NN - 1) van = (T)(eP * e[(j + 1) * NP1 + i] * inv_h2 * sP * sd[k + NN]);
        }
        ae[k] = vae;
        an[k] = van;
    }
    __syncthreads();

    const double fnorm = fabs(a.f) * (double)(NN - 1);
    int total = 0, sweeps = 0;
    bool ok = false;
    for (int sweep = 0;; ++sweep) {
        sweeps = sweep;
        double acc = 0.0;
        for (int k = tid; k < nodes; k += 1024) {
            const int g = k / NN, c = k % NN, i = c + 1, j = g + 1;
            T rvk = T(0);
            if (interior(g, c)) {
                double res = a.f;
                if (sweep > 0) {
                    const double xP = x64[k];
                    const double xE = (c + 1 < NN - 1) ? x64[k + 1] : 0.0;
                    const double xW = (c > 0) ? x64[k - 1] : 0.0;
                    const double xN = (g + 1 < NN - 1) ? x64[k + NN] : 0.0;
                    const double xS = (g > 0) ? x64[k - NN] : 0.0;
                    res -= e[j * NP1 + i] * inv_h2 *
                           (e[j * NP1 + i + 1] * (xP - xE) + e[j * NP1 + i - 1] * (xP - xW) +
                            e[(j + 1) * NP1 + i] * (xP - xN) + e[(j - 1) * NP1 + i] * (xP - xS));
                }
                acc += res * res;
                rvk = (T)(sd[k] * res);
            }
            rv[k] = rvk;
            pv[k] = rvk;
            xv[k] = T(0);
        }
        const double rr64 = block_sum<NW>(acc, red2);
        if (sqrt(rr64) <= a.tol64 * fnorm) { ok = true; break; }
        if (!(rr64 < INFINITY) || sweep >= a.max_sweeps || total >= a.max_iter) break;

        double tacc = 0.0;
        for (int k = tid; k < nodes; k += 1024) tacc += (double)rv[k] * (double)rv[k];
        double rr = block_sum<NW>(tacc, red1);
        const double target = a.tol_inner * a.tol_inner * rr;
        bool broke = false;
        while (rr > target) {
            if (total >= a.max_iter) break;
            T pq_acc = T(0);
            for (int k = tid; k < nodes; k += 1024) {
                const int g = k / NN, c = k % NN;
                T qk = T(0);
                const T pk = pv[k];
                if (interior(g, c)) {
                    const T pE = pv[k + 1];
                    const T sW = (c > 0) ? ae[k - 1] * pv[k - 1] : T(0);
                    const T pN = pv[k + NN];
                    const T sS = (g > 0) ? an[k - NN] * pv[k - NN] : T(0);
                    qk = pk - ae[k] * pE - sW - an[k] * pN - sS;
                }
                qv[k] = qk;
                pq_acc += pk * qk;
            }
            const double pq = block_sum<NW>((double)pq_acc, red1);
            if (!(pq > 0.0) || !(pq < INFINITY)) { broke = true; break; }
            const T alpha = (T)(rr / pq);
            T r_acc = T(0);
            for (int k = tid; k < nodes; k += 1024) {
                xv[k] += alpha * pv[k];
                const T rk = rv[k] - alpha * qv[k];
                rv[k] = rk;
                r_acc += rk * rk;
            }
            const double rrn = block_sum<NW>((double)r_acc, red2);
            const T beta = (T)(rrn / rr);
            rr = rrn;
            for (int k = tid; k < nodes; k += 1024) pv[k] = rv[k] + beta * pv[k];
            __syncthreads();
            ++total;
        }
        for (int k = tid; k < nodes; k += 1024) {
            const double corr = sd[k] * (double)xv[k];
            x64[k] = (sweep == 0) ? corr : x64[k] + corr;
        }
        __syncthreads();
        if (broke) break;
    }

    __syncthreads();
    double val = 0.0;
    if (tid < a.n_obs) {
        const int node = a.obs[tid];
        const int jj = node / NP1, ii = node % NP1;
        if (ii >= 1 && ii <= NN - 1 && jj >= 1 && jj <= NN - 1) val = x64[(jj - 1) * NN + ii - 1];
        if (!ok) val = NAN;
        if (a.G) a.G[row * a.n_obs + tid] = val;
    }
    if (tid < 64) {
        const double dlt = (tid < a.n_obs) ? val - a.y[tid] : 0.0;
        const double s = wave_sum(dlt * dlt);
        if (tid == 0) {
            if (a.phi) a.phi[row] = ok ? s * a.inv2s2 : INFINITY;
            if (a.iters) a.iters[row] = ok ? total : -1;
            if (!ok) atomicOr(a.flags, SMC_FLAG_NOCONV);
            if (a.stats) {
                atomicAdd(&a.stats[0], (unsigned long long)total);
                atomicAdd(&a.stats[1], (unsigned long long)(sweeps + 1));
                atomicAdd(&a.stats[2], 1ull);
            }
        }
    }
}

// 1D: the tridiagonal flux-form system has the closed-form solution
//   F_{i+1/2} = F_{1/2} - i h f,  F_{1/2} = sum_i (i h f / a_{i+1/2}) / sum_i (1 / a_{i+1/2}),
//   w_{i+1} = w_i + h F_{i+1/2} / a_{i+1/2},  w_0 = 0,
// from the flux balance (F_{i-1/2} - F_{i+1/2}) / h = f and w_n = 0.  One thread per particle.
__global__ __launch_bounds__(256) void solve1d_kernel(SolveArgs a, int n, int64_t N) {
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (row >= N) return;
    const double* e = a.e + row * a.e_stride;
    double* w = a.x64 + row * a.x_stride;
    const double h = 1.0 / n;
    double s1 = 0.0, s0 = 0.0;
    for (int k = 0; k < n; ++k) {
        const double inv_a = 1.0 / (e[k] * e[k + 1]);   // face coefficient a_{k+1/2} = e_k e_{k+1}
        s1 += k * h * a.f * inv_a;
        s0 += inv_a;
    }
    const double F0 = s1 / s0;
    double wk = 0.0;
    w[0] = 0.0;
    for (int k = 0; k < n; ++k) {
        wk += h * (F0 - k * h * a.f) / (e[k] * e[k + 1]);
        w[k + 1] = (k + 1 == n) ? 0.0 : wk;
    }
    double s = 0.0;
    for (int k = 0; k < a.n_obs; ++k) {
        const double v = w[a.obs[k]];
        if (a.G) a.G[row * a.n_obs + k] = v;
        s += (v - a.y[k]) * (v - a.y[k]);
    }
    if (a.phi) a.phi[row] = s * a.inv2s2;
    if (a.iters) a.iters[row] = 0;
}

template <typename T, int NN, int R>
static hipError_t run_onchip(int64_t N, const SolveArgs& a, hipStream_t s) {
    cg_onchip<T, NN, R><<<dim3((unsigned)N), dim3(NN * NN / R), 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_solve2d(int n, int prec, int64_t N, const SolveArgs& a, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    if (prec == SMC_FP32_REFINE) {
        switch (n) {
            case 16: return run_onchip<float, 16, 4>(N, a, s);
            case 32: return run_onchip<float, 32, 4>(N, a, s);
            case 64: return run_onchip<float, 64, 8>(N, a, s);
            case 128: return run_onchip<float, 128, 16>(N, a, s);
            default:
                cg_global<float><<<dim3((unsigned)N), dim3(1024), 0, s>>>(a, n);
                return hipGetLastError();
        }
    }
    SolveArgs b = a;
    b.tol_inner = 0.1 * a.tol64;
    switch (n) {
        case 16: return run_onchip<double, 16, 4>(N, b, s);
        case 32: return run_onchip<double, 32, 4>(N, b, s);
        case 64: return run_onchip<double, 64, 8>(N, b, s);
        default:
            cg_global<double><<<dim3((unsigned)N), dim3(1024), 0, s>>>(b, n);
            return hipGetLastError();
    }
}

hipError_t launch_solve1d(int n, int64_t N, const SolveArgs& a, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    solve1d_kernel<<<dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s>>>(a, n, N);
    return hipGetLastError();
}

}  // namespace smc
