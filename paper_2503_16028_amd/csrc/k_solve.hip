// Forward solve of the Darcy problem, one workgroup per particle.
//
// Operator (flux form, h = 1/n, geometric-mean faces, Sec. 3.2 eq. (example2:PDE)):
//   (A w)_P = sum_Q a_PQ (w_P - w_Q) / h^2,   a_PQ = e_P e_Q,  e = exp(u/2),
// at interior nodes, w = 0 on the boundary.  Because every face coefficient is a product, the
// symmetrically Jacobi-scaled operator factorises:
//   A^ = D^{-1/2} A D^{-1/2} = I - T N T,   t_P = sqrt(e_P / sum_{Q nbr P} e_Q),
// with N the 0/1 adjacency of interior nodes.  So one coefficient per node suffices and
//   (A^ p)_P = p_P - t_P (y_E + y_W + y_N + y_S),   y = t p.
//
// Method: preconditioned conjugate gradients on A^ y = D^{-1/2} r in precision T, inside an
// FP64 residual refinement: each sweep forms r = f - A x with the FP64 operator, solves the
// scaled correction to a relative reduction, and adds D^{-1/2} y to the FP64 iterate; the
// loop stops on ||f - A x|| <= tol64 ||f||, so the accuracy is the FP64 operator's whatever T.
// Preconditioners: none beyond the Jacobi scaling, or (DST) the inverse of the constant-
// coefficient Dirichlet Laplacian L, which A^ is spectrally close to (its iteration count does
// not grow with the grid).  L^{-1} = S diag(1 / (lam_k + lam_l)) S with the orthonormal
// symmetric sine transform S[a][b] = sqrt(2/n) sin(pi (a+1)(b+1) / n) and
// lam_k = sin^2(pi (k+1) / (2n)) up to a constant factor (CG is blind to it), applied as four
// 16x16x32 FP16 MFMA products with FP32 accumulation, the input scaled by a power of two from
// its norm; operand rounding perturbs only the preconditioner, never the operator or the FP64
// residual.
//
// On-chip layout: thread t owns column c = t % n of the padded n x n block (x-node c + 1) and a
// strip of R rows (y-nodes (t / n) R + 1 ..); nodes with index n are boundary padding with t = 0
// and p = 0.  The CG vectors and t live in registers; each iteration publishes y = t p to one
// zero-padded LDS array, from which the horizontal neighbours (and the strip ends) are read at
// immediate offsets with no branches.  Dot products are wave butterflies plus a fixed-order sum
// of the wave partials: every thread sees the same bits, and a particle's result does not depend
// on the batch it is solved in.
#include <type_traits>
#include <utility>

#include "common.hpp"
#include "move_body.hpp"
#include "synth_body.hpp"

namespace smc {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef _Float16 hf8 __attribute__((ext_vector_type(8)));
typedef _Float16 hf4 __attribute__((ext_vector_type(4)));

// v_mfma_f32_16x16x32_f16 lane layout (the bf16 instruction's too), checked on the device:
//   A[16][32]: lane supplies row lane % 16, k = 8 (lane / 16) + 0..7
//   B[32][16]: lane supplies col lane % 16, k = 8 (lane / 16) + 0..7
//   D[16][16]: lane holds col lane % 16, rows 4 (lane / 16) + 0..3
__device__ __forceinline__ f4 mfma_f16(hf8 a, hf8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// The exponent e of |r| = f 2^e, f in [0.5, 1), from rr = |r|^2; clamped, so that a zero or
// non-finite norm still gives a usable scale.  The transforms take their FP16 input as r 2^-e.
__device__ __forceinline__ int norm_exponent(double rr) {
    int ex = 0;
    (void)frexp(sqrt(rr), &ex);
    return ex < -120 ? -120 : (ex > 120 ? 120 : ex);
}

template <int NN, int NW>
struct DstShape {
    static constexpr int NB = NN / 16;        // 16 x 16 tiles per dimension
    static constexpr int KS = NN / 32;        // k steps of 32
    // strips of S per wave: two when there are no more waves than strips, so that every operand
    // fragment read from LDS feeds two matrix products
    static constexpr int SP = (NW <= NB && NB % 2 == 0) ? 2 : 1;
    static constexpr int NSG = NB / SP;       // strip groups
    static constexpr int TPW = NB * NB / (NW * SP);   // output tiles per wave and strip
    static constexpr int LD = NN + 8;         // 16-bit row stride (16-byte aligned, spreads banks)
    static constexpr int LDZ = NN + 4;        // fp32 row stride of the result
    static constexpr int BYTES = 2 * NN * LD * 2 + NN * LDZ * 4;
    static_assert(NW % NSG == 0 && (NB * NB) % (NW * SP) == 0, "transform tiling");
};

template <typename T, int NN, int R, int NW>
__device__ __forceinline__ void dst_apply(const T (&rin)[R], double rr, unsigned char* smem,
                                          const _Float16* __restrict__ Stab, const float* __restrict__ lamtab, int c,
                                          int b, int wave, int lane) {
    using DS = DstShape<NN, NW>;
    constexpr int LD = DS::LD, LDZ = DS::LDZ, KS = DS::KS, TPW = DS::TPW, SP = DS::SP, NSG = DS::NSG;
    // FP16 operands, FP32 accumulation.  r enters scaled by 2^-e, with |r| = f 2^e and f in
    // [0.5, 1) (rr = |r|^2, the same in every thread); S is orthonormal, so every intermediate
    // is bounded by its Frobenius norm: below 1 before 1 / (lam_k + lam_l) and below
    // 1 / (2 lam_0) < 3400 after it, inside FP16's range with the small high-mode values still
    // normal.  Z is scaled back by 2^e (exact).  With bf16 operands the rounding costs CG
    // iterations (5 instead of 3 to a 1e-3 reduction at 128^2); FP16's 3 more significand bits
    // recover the exact preconditioner's count.
    const int ex = norm_exponent(rr);
    const float sc = ldexpf(1.0f, -ex), unsc = ldexpf(1.0f, ex);
    _Float16* bufA = reinterpret_cast<_Float16*>(smem);   // R^T, later T2^T
    _Float16* bufB = bufA + NN * LD;                      // T1, later T3
    float* Z = reinterpret_cast<float*>(bufB + NN * LD);   // Z[g][c]: lanes of a row read consecutive words
    const int lr = lane & 15, lk = lane >> 4;
    const int sg = wave % NSG, wq = wave / NSG;
    hf8 sfrag[SP][KS];   // rows (sg SP + s) 16.. of S (symmetric: also columns, as a B operand)
    float lam_col[SP];
#pragma unroll
    for (int q = 0; q < SP; ++q) {
        const int sb = sg * SP + q;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
            sfrag[q][ks] = *reinterpret_cast<const hf8*>(Stab + (sb * 16 + lr) * NN + 32 * ks + 8 * lk);
        lam_col[q] = lamtab[sb * 16 + lr];
    }
    {   // stage R^T[c][g] = fp16(r 2^-e): the thread's strip is contiguous
        _Float16* dst = bufA + c * LD + b * R;
        if constexpr (R % 8 == 0) {
#pragma unroll
            for (int r = 0; r < R; r += 8) {
                hf8 v;
#pragma unroll
                for (int q = 0; q < 8; ++q) v[q] = (_Float16)((float)rin[r + q] * sc);
                *reinterpret_cast<hf8*>(dst + r) = v;
            }
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) dst[r] = (_Float16)((float)rin[r] * sc);
        }
    }
    __syncthreads();
    // Each product is ordered so that the four values a lane holds in its 16 x 16 result tile
    // are consecutive in the layout the next product reads (one 8-byte or 16-byte store per tile),
    // while both operands stay contiguous along the contraction index.
#pragma unroll 1
    for (int tt = 0; tt < TPW; ++tt) {   // T1[k][c] = sum_g S[k][g] R[g][c], as (R^T S)[c][k]
        const int cb = wq * TPW + tt;
        f4 acc[SP];
#pragma unroll
        for (int q = 0; q < SP; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const hf8 av = *reinterpret_cast<const hf8*>(bufA + (cb * 16 + lr) * LD + 32 * ks + 8 * lk);
#pragma unroll
            for (int q = 0; q < SP; ++q) acc[q] = mfma_f16(av, sfrag[q][ks], acc[q]);
        }
#pragma unroll
        for (int q = 0; q < SP; ++q) {
            hf4 o;
#pragma unroll
            for (int v = 0; v < 4; ++v) o[v] = (_Float16)acc[q][v];
            *reinterpret_cast<hf4*>(bufB + ((sg * SP + q) * 16 + lr) * LD + cb * 16 + 4 * lk) = o;
        }
    }
    __syncthreads();
#pragma unroll 1
    for (int tt = 0; tt < TPW; ++tt) {   // T2^T[l][k] = (sum_c T1[k][c] S[c][l]) / (lam_k + lam_l)
        const int rb = wq * TPW + tt;
        f4 acc[SP];
#pragma unroll
        for (int q = 0; q < SP; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const hf8 av = *reinterpret_cast<const hf8*>(bufB + (rb * 16 + lr) * LD + 32 * ks + 8 * lk);
#pragma unroll
            for (int q = 0; q < SP; ++q) acc[q] = mfma_f16(av, sfrag[q][ks], acc[q]);
        }
#pragma unroll
        for (int q = 0; q < SP; ++q) {
            hf4 o;
#pragma unroll
            for (int v = 0; v < 4; ++v)
                o[v] = (_Float16)(acc[q][v] * __builtin_amdgcn_rcpf(lamtab[rb * 16 + 4 * lk + v] + lam_col[q]));
            *reinterpret_cast<hf4*>(bufA + ((sg * SP + q) * 16 + lr) * LD + rb * 16 + 4 * lk) = o;
        }
    }
    __syncthreads();
#pragma unroll 1
    for (int tt = 0; tt < TPW; ++tt) {   // T3[g][l] = sum_k S[g][k] T2[k][l], as (T2^T S)[l][g]
        const int cb = wq * TPW + tt;
        f4 acc[SP];
#pragma unroll
        for (int q = 0; q < SP; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const hf8 av = *reinterpret_cast<const hf8*>(bufA + (cb * 16 + lr) * LD + 32 * ks + 8 * lk);
#pragma unroll
            for (int q = 0; q < SP; ++q) acc[q] = mfma_f16(av, sfrag[q][ks], acc[q]);
        }
#pragma unroll
        for (int q = 0; q < SP; ++q) {
            hf4 o;
#pragma unroll
            for (int v = 0; v < 4; ++v) o[v] = (_Float16)acc[q][v];
            *reinterpret_cast<hf4*>(bufB + ((sg * SP + q) * 16 + lr) * LD + cb * 16 + 4 * lk) = o;
        }
    }
    __syncthreads();
#pragma unroll 1
    for (int tt = 0; tt < TPW; ++tt) {   // Z[g][c] = sum_l T3[g][l] S[l][c], as (S T3^T)[c][g]
        const int rb = wq * TPW + tt;
        f4 acc[SP];
#pragma unroll
        for (int q = 0; q < SP; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const hf8 bv = *reinterpret_cast<const hf8*>(bufB + (rb * 16 + lr) * LD + 32 * ks + 8 * lk);
#pragma unroll
            for (int q = 0; q < SP; ++q) acc[q] = mfma_f16(sfrag[q][ks], bv, acc[q]);
        }
#pragma unroll
        for (int q = 0; q < SP; ++q)
            *reinterpret_cast<float4*>(Z + (rb * 16 + lr) * LDZ + (sg * SP + q) * 16 + 4 * lk) =
                make_float4(acc[q][0] * unsc, acc[q][1] * unsc, acc[q][2] * unsc, acc[q][3] * unsc);
    }
    __syncthreads();
}

// The fast-Poisson preconditioner alone: z[g][c] = (L^{-1} r)[g][c] on the padded n x n block of
// each of N grids (row g is y-node g+1, column c is x-node c+1; padding row/column zero).
template <int NN, int R>
__global__ __launch_bounds__(NN * NN / R) void dst_apply_kernel(const float* __restrict__ rin, float* __restrict__ zout,
                                                               const _Float16* __restrict__ Stab,
                                                               const float* __restrict__ lamtab) {
    constexpr int NT = NN * NN / R, NW = NT / 64;
    __shared__ __align__(16) unsigned char smem[DstShape<NN, NW>::BYTES];
    __shared__ double red[16];
    const int tid = threadIdx.x, c = tid % NN, b = tid / NN;
    const int64_t base = (int64_t)blockIdx.x * NN * NN;
    float r[R];
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        r[k] = rin[base + (b * R + k) * NN + c];
        acc += (double)r[k] * (double)r[k];
    }
    const double rr = block_sum<NW>(acc, red);
    dst_apply<float, NN, R, NW>(r, rr, smem, Stab, lamtab, c, b, tid >> 6, tid & 63);
    const float* Z = reinterpret_cast<const float*>(smem + 2 * NN * DstShape<NN, NW>::LD * 2);
#pragma unroll
    for (int k = 0; k < R; ++k) zout[base + (b * R + k) * NN + c] = Z[(b * R + k) * DstShape<NN, NW>::LDZ + c];
}

__global__ __launch_bounds__(1024) void dst256_apply_kernel(const float* __restrict__ rin, float* __restrict__ zout,
                                                            const _Float16* __restrict__ Stab,
                                                            const float* __restrict__ lamtab);

hipError_t launch_dst_apply(int n, int64_t N, const float* r, float* z, const void* S, const float* lam,
                            hipStream_t s) {
    if (N <= 0) return hipSuccess;
    const _Float16* Sh = reinterpret_cast<const _Float16*>(S);
    switch (n) {
        case 256: dst256_apply_kernel<<<dim3((unsigned)N), dim3(1024), 0, s>>>(r, z, Sh, lam); break;
        case 32: dst_apply_kernel<32, 4><<<dim3((unsigned)N), dim3(256), 0, s>>>(r, z, Sh, lam); break;
        case 64: dst_apply_kernel<64, 8><<<dim3((unsigned)N), dim3(512), 0, s>>>(r, z, Sh, lam); break;
        case 128: dst_apply_kernel<128, 16><<<dim3((unsigned)N), dim3(1024), 0, s>>>(r, z, Sh, lam); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

constexpr int cmax(int x, int y) { return x > y ? x : y; }

// LDS bytes of the on-chip solver's big buffer: the exchange array, or the transform buffers.
template <typename T, int NN, int R, bool DST>
constexpr int onchip_smem() {
    constexpr int NW = NN * NN / R / 64;
    constexpr int XBYTES = (2 * (NN + 1) + NN * NN) * (int)sizeof(T);
    return (DST && DstShape<NN, NW>::BYTES > XBYTES) ? DstShape<NN, NW>::BYTES : XBYTES;
}

// Small LDS of one solve: block-reduction slots and the adjoint's point sources.
struct SolveShared {
    double red1[16], red2[16];
    double src_w[MAX_OBS];   // adjoint point sources: weight and unknown index (-1: none)
    int src_at[MAX_OBS];
};

// The FP64 passes over one thread's strip (column c, rows g0 .. g0 + R - 1).  They run outside the
// conjugate-gradient loop and are bound by the latency of their global loads, so each is a separate
// function: register-allocated on its own, it can unroll the strip and keep many loads in flight
// without taking registers from the loop.  Pointers are cast back to their address spaces (the
// call passes them as generic pointers).
typedef const __attribute__((address_space(1))) double* gcdp;
typedef __attribute__((address_space(1))) double* gdp;
template <typename S> using gcp = const __attribute__((address_space(1))) S*;
template <typename S> using gp = __attribute__((address_space(1))) S*;
// Read-only data through the constant address space: wave-uniform loads of it become scalar loads
// into SGPRs, which leaves the vector registers to the strip's own loads.  Only for arrays no
// kernel writes while it runs (the coefficient field, written by the synthesis launch before).
typedef const __attribute__((address_space(4))) double* kcdp;

// The adjoint's point sources (G - y) / sigma^2 of the on-chip solver: weights and interior flat
// indices (-1: not an interior node), written by the forward pass's observation.  Named at module
// level so that the residual pass, a function of its own, reads them with LDS instructions (through a
// pointer argument they would become generic accesses).
__shared__ double g_src_w[MAX_OBS];
__shared__ int g_src_at[MAX_OBS];

// Right-hand side of the pass at interior unknown `flat`: f, or the adjoint's point sources.
__device__ __forceinline__ double strip_rhs(int flat, bool sources, double f, const double* src_w, const int* src_at,
                                            int n_obs) {
    if (!sources) return f;
    double s = 0.0;
    for (int k = 0; k < n_obs; ++k) s += (src_at[k] == flat) ? src_w[k] : 0.0;
    return s;
}


// A pointer every lane holds, made visibly wave-uniform (its loads can then go through the
// scalar unit; used only for data the kernel does not write).
__device__ __forceinline__ const double* wave_uniform(const double* p) {
    const unsigned long long v = (unsigned long long)p;
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v >> 32));
    return (const double*)(((unsigned long long)hi << 32) | lo);
}

// The value `v` of the next lane (lane 63: `edge`) and of the previous lane (lane 0: `edge`), by
// DPP wave shifts: a thread's east and west neighbours are the adjacent lanes of its wave.
__device__ __forceinline__ double from_next_lane(double v, double edge) {
    const long long b = __double_as_longlong(v), be = __double_as_longlong(edge);
    const int lo = __builtin_amdgcn_update_dpp((int)be, (int)b, 0x130, 0xF, 0xF, false);   // wave_shl:1
    const int hi = __builtin_amdgcn_update_dpp((int)(be >> 32), (int)(b >> 32), 0x130, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double from_prev_lane(double v, double edge) {
    const long long b = __double_as_longlong(v), be = __double_as_longlong(edge);
    const int lo = __builtin_amdgcn_update_dpp((int)be, (int)b, 0x138, 0xF, 0xF, false);   // wave_shr:1
    const int hi = __builtin_amdgcn_update_dpp((int)(be >> 32), (int)(b >> 32), 0x138, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Scaled residual D^{-1/2} (f - A x) of the strip into its LDS slots (x = 0 when `zero_x`);
// returns the sum of squares of the unscaled residual.  Every load has a clamped, in-bounds index
// and a select discards what lies outside the domain, so the strip is straight-line code whose
// loads are issued 8 rows at a time.  The east and west values of e and x come from the adjacent
// lanes; only the two wave edges load them (e through the scalar unit when SE: in SGPRs they leave
// the vector registers to the rows' loads).  The scalar cache does not see vector stores, so SE is
// only for a field no store of the same launch has written (the synthesis ran in an earlier one);
// a launch that synthesises the field itself loads the edges as vectors.
// MANY: a strip holding more sources than the list keeps sums over every source at each row (a
// separate instantiation, so that the common one carries no such loop per unrolled row).
template <typename T, int NN, int R, bool SRC, typename SD, bool SE = true, bool MANY = false>
__device__ __noinline__ double strip_residual(const double* __restrict__ e_, const double* __restrict__ xo_,
                                              const SD* __restrict__ sd_, T* __restrict__ tb_, int c, int g0,
                                              bool zero_x, double f, const double* __restrict__ src_w,
                                              const int* __restrict__ src_at, int n_obs) {
    static_assert(NN % 64 == 0, "a wave covers consecutive columns of one row");
    constexpr int NP1 = NN + 1;
    const double inv_h2 = (double)NN * (double)NN;
    gcdp e = (gcdp)e_;
    gcdp xo = (gcdp)xo_;
    gcp<SD> sd = (gcp<SD>)sd_;
    __attribute__((address_space(3))) T* tb = (__attribute__((address_space(3))) T*)tb_;
    const int i = c + 1;
    const bool colin = c < NN - 1;
    double acc = 0.0;
    // SRC: the sources in this thread's strip (column c, rows g0 .. g0 + R - 1), found once; a strip
    // with more than SMAX of them sums over every source at each row instead
    constexpr int SMAX = 4;
    int srow[SMAX];
    double sw[SMAX];
    int ns = 0;
    if constexpr (SRC) {
#pragma unroll
        for (int q = 0; q < SMAX; ++q) {
            srow[q] = -1;
            sw[q] = 0.0;
        }
        for (int k = 0; k < n_obs; ++k) {
            const int at = g_src_at[k];
            const int gr = at / NN, cc = at - gr * NN;
            if (at >= 0 && cc == c && gr >= g0 && gr < g0 + R) {
#pragma unroll
                for (int q = 0; q < SMAX; ++q)
                    if (q == ns) {
                        srow[q] = gr - g0;
                        sw[q] = g_src_w[k];
                    }
                ++ns;
            }
        }
        if constexpr (!MANY) {   // the whole wave together: the pass exchanges values between lanes
            if (__any(ns > SMAX))
                return strip_residual<T, NN, R, true, SD, SE, true>(e_, xo_, sd_, tb_, c, g0, zero_x, f, src_w, src_at,
                                                                    n_obs);
        }
    }
    auto rhs_at = [&](int r) -> double {
        if constexpr (!SRC) {
            return f;
        } else {
            if constexpr (MANY) return strip_rhs((g0 + r) * NN + c, true, f, g_src_w, g_src_at, n_obs);
            double v = 0.0;
#pragma unroll
            for (int q = 0; q < SMAX; ++q) v += (srow[q] == r) ? sw[q] : 0.0;
            return v;
        }
    };
    if (zero_x) {
#pragma unroll 8
        for (int r = 0; r < R; ++r) {
            const int g = g0 + r;
            const bool in = colin && g < NN - 1;
            const double fr = rhs_at(r);
            const double sdv = (double)sd[g * NN + c];
            acc += in ? fr * fr : 0.0;
            tb[NN + 1 + r * NN] = in ? (T)(sdv * fr) : T(0);
        }
        return acc;
    }
    const int lane = threadIdx.x & 63;
    const int c0 = __builtin_amdgcn_readfirstlane(c - lane);       // first column of the wave
    const int ieE = min(c0 + 65, NN), ieW = c0;                     // e columns beyond the wave's edges
    const int cxE = min(c0 + 64, NN - 1), cxW = max(c0 - 1, 0);     // x columns beyond the edges
    const bool xEok = c0 + 64 < NN - 1, xWok = c0 > 0;
    kcdp eu = (kcdp)wave_uniform(e_);
    const int g0u = __builtin_amdgcn_readfirstlane(g0);
    double eS = e[g0 * NP1 + i], eC = e[(g0 + 1) * NP1 + i];
    double xS = xo[max(g0 - 1, 0) * NN + c], xC = xo[g0 * NN + c];
    xS = (g0 > 0 && colin) ? xS : 0.0;
    xC = (g0 < NN - 1 && colin) ? xC : 0.0;
    constexpr int B = R < 8 ? R : 8;   // rows whose loads are issued together
    static_assert(R % B == 0, "strip blocking");
#pragma unroll 1
    for (int r0 = 0; r0 < R; r0 += B) {
        double eN[B], xN[B], sdv[B], eEe[B], eWe[B], xEe[B], xWe[B];
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int g = g0 + r0 + k, j = g + 1;
            eN[k] = e[min(j + 1, NN) * NP1 + i];
            xN[k] = xo[min(g + 1, NN - 1) * NN + c];
            sdv[k] = (double)sd[g * NN + c];
            const int ju = g0u + r0 + k + 1;
            eEe[k] = SE ? eu[ju * NP1 + ieE] : e[ju * NP1 + ieE];
            eWe[k] = SE ? eu[ju * NP1 + ieW] : e[ju * NP1 + ieW];
            xEe[k] = xo[g * NN + cxE];
            xWe[k] = xo[g * NN + cxW];
        }
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int r = r0 + k, g = g0 + r, j = g + 1;
            const double eE = from_next_lane(eC, eEe[k]);
            const double eW = from_prev_lane(eC, eWe[k]);
            const double xe_ = from_next_lane(xC, xEok ? xEe[k] : 0.0);
            const double xw_ = from_prev_lane(xC, xWok ? xWe[k] : 0.0);
            const double xn = (g + 1 < NN - 1 && colin) ? xN[k] : 0.0;
            const double xe = (c + 1 < NN - 1) ? xe_ : 0.0;
            const double xw = (c > 0) ? xw_ : 0.0;
            const bool in = colin && g < NN - 1;
            const double fr = rhs_at(r);
            const double res = fr - eC * inv_h2 * (eE * (xC - xe) + eW * (xC - xw) + eN[k] * (xC - xn) + eS * (xC - xS));
            acc += in ? res * res : 0.0;
            tb[NN + 1 + r * NN] = in ? (T)(sdv[k] * res) : T(0);
            eS = eC;
            eC = (j + 1 <= NN) ? eN[k] : 0.0;
            xS = xC;
            xC = xn;
        }
    }
    return acc;
}

// x += D^{-1/2} y for the strip, y staged in its LDS slots (x = D^{-1/2} y when `first`).
template <typename T, int NN, int R, typename SD>
__device__ __noinline__ void strip_update(double* xo_, const SD* sd_, const T* tb_, int c, int g0, bool first) {
    gdp xo = (gdp)xo_;
    gcp<SD> sd = (gcp<SD>)sd_;
    const __attribute__((address_space(3))) T* tb = (const __attribute__((address_space(3))) T*)tb_;
    constexpr int B = R < 16 ? R : 16;   // rows whose loads are issued together
#pragma unroll 1
    for (int r0 = 0; r0 < R; r0 += B) {
        double sdv[B], xv[B];
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int g = g0 + r0 + k;
            sdv[k] = (double)sd[g * NN + c];
            xv[k] = first ? 0.0 : xo[g * NN + c];
        }
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int g = g0 + r0 + k;
            xo[g * NN + c] = xv[k] + sdv[k] * (double)tb[NN + 1 + (r0 + k) * NN];
        }
    }
}

// dPhi/du at the strip's nodes after the forward solution w and the adjoint solution lam are final
// (App. B's gradient of the discrete potential, the derivative of the face coefficient a_PQ = e_P e_Q
// by u_P being a_PQ / 2):
//   du[P] = -(n^2 / 2) e_P sum_{Q nbr P} e_Q (lam_P - lam_Q)(w_P - w_Q),   w = lam = 0 on the boundary,
// at every node of the (n+1)^2 grid, [j][i]: the thread's nodes are x-node i = c + 1, y-nodes
// j = g0 + 1 .. g0 + R (i = n and j = n are boundary nodes); column 0 is done by the threads of c = 0
// and row 0 by the strips at g0 = 0 (a boundary node's only interior neighbour is beside it).  w and
// lam are in the interior layout [g][c] (index n - 1 holds 0); east and west values come from the
// adjacent lanes, the wave edges load theirs: e's through the scalar unit (no launch writes it while
// it runs), lam's with vector loads (this launch wrote it), w's through the scalar unit when an
// earlier launch wrote it (WS) and with vector loads otherwise.  The scalar edges leave the vector
// registers to the strip's own loads, eight rows in flight without spilling.
template <int NN, int R, bool WS>
__device__ __noinline__ void strip_dphi(const double* __restrict__ e_, const double* __restrict__ w_,
                                        const double* __restrict__ l_, double* __restrict__ du_, int c, int g0) {
    static_assert(NN % 64 == 0, "a wave covers consecutive columns of one row");
    constexpr int NP1 = NN + 1;
    const double scale = -0.5 * (double)NN * (double)NN;
    gcdp e = (gcdp)e_;
    gcdp w = (gcdp)w_;
    gcdp l = (gcdp)l_;
    gdp du = (gdp)du_;
    kcdp eu = (kcdp)wave_uniform(e_);
    kcdp wu = (kcdp)wave_uniform(w_);
    const int i = c + 1;
    const int lane = threadIdx.x & 63;
    const int c0 = __builtin_amdgcn_readfirstlane(c - lane);
    const int ieE = min(c0 + 65, NN), ieW = c0;                     // e columns beyond the wave's edges
    const int cxE = min(c0 + 64, NN - 1), cxW = max(c0 - 1, 0);     // interior columns beyond them
    const bool xEok = c0 + 64 < NN - 1, xWok = c0 > 0;
    const bool colin = c < NN - 1;
    auto wl = [&](gcdp v, int g) -> double {   // interior value at (g, c), 0 outside the interior
        const double x = v[min(max(g, 0), NN - 1) * NN + c];
        return (g >= 0 && g < NN - 1 && colin) ? x : 0.0;
    };
    const int g0u = __builtin_amdgcn_readfirstlane(g0);
    double eS = e[g0 * NP1 + i], eC = e[(g0 + 1) * NP1 + i];
    double wS = wl(w, g0 - 1), wC = wl(w, g0), lS = wl(l, g0 - 1), lC = wl(l, g0);
    constexpr int B = R < 8 ? R : 8;
    static_assert(R % B == 0, "strip blocking");
#pragma unroll 1
    for (int r0 = 0; r0 < R; r0 += B) {
        double eN[B], wN[B], lN[B], eEe[B], eWe[B], wEe[B], wWe[B], lEe[B], lWe[B];
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int g = g0 + r0 + k, j = g + 1;
            const int ju = g0u + r0 + k + 1, gcu = min(ju - 1, NN - 1), gc = min(g, NN - 1);
            eN[k] = e[min(j + 1, NN) * NP1 + i];
            wN[k] = wl(w, g + 1);
            lN[k] = wl(l, g + 1);
            eEe[k] = eu[ju * NP1 + ieE];
            eWe[k] = eu[ju * NP1 + ieW];
            wEe[k] = WS ? wu[gcu * NN + cxE] : w[gc * NN + cxE];
            wWe[k] = WS ? wu[gcu * NN + cxW] : w[gc * NN + cxW];
            lEe[k] = l[gc * NN + cxE];
            lWe[k] = l[gc * NN + cxW];
        }
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int g = g0 + r0 + k, j = g + 1;
            const bool rowin = g < NN - 1;
            const double eE = from_next_lane(eC, eEe[k]);
            const double eW = from_prev_lane(eC, eWe[k]);
            const double wE_ = from_next_lane(wC, (xEok && rowin) ? wEe[k] : 0.0);
            const double wW_ = from_prev_lane(wC, (xWok && rowin) ? wWe[k] : 0.0);
            const double lE_ = from_next_lane(lC, (xEok && rowin) ? lEe[k] : 0.0);
            const double lW_ = from_prev_lane(lC, (xWok && rowin) ? lWe[k] : 0.0);
            const double wE = (c + 1 < NN - 1) ? wE_ : 0.0, lE = (c + 1 < NN - 1) ? lE_ : 0.0;
            const double wW = (c > 0) ? wW_ : 0.0, lW = (c > 0) ? lW_ : 0.0;
            double acc = 0.0;
            acc += eW * (lC - lW) * (wC - wW);
            acc += eE * (lC - lE) * (wC - wE);
            acc += eS * (lC - lS) * (wC - wS);
            acc += eN[k] * (lC - lN[k]) * (wC - wN[k]);
            du[j * NP1 + i] = scale * eC * acc;
            if (c == 0) du[j * NP1] = scale * eW * eC * lC * wC;      // node (0, j): its neighbour is (1, j)
            if (g == 0) {
                du[i] = scale * eS * eC * lC * wC;                     // node (i, 0): its neighbour is (i, 1)
                if (c == 0) du[0] = 0.0;                               // corner: boundary neighbours only
            }
            eS = eC;
            eC = eN[k];
            wS = wC;
            wC = wN[k];
            lS = lC;
            lC = lN[k];
        }
    }
}

// D^{-1/2} into the workspace and t = sqrt(e_P / sum e_Q) into the strip's LDS slots (SE as for
// strip_residual).
template <typename T, int NN, int R, typename SD, bool SE = true>
__device__ __noinline__ void strip_setup(const double* __restrict__ e_, SD* __restrict__ sd_, T* __restrict__ tb_,
                                         int c, int g0) {
    static_assert(NN % 64 == 0, "a wave covers consecutive columns of one row");
    constexpr int NP1 = NN + 1;
    const double h = 1.0 / NN;
    gcdp e = (gcdp)e_;
    gp<SD> sd = (gp<SD>)sd_;
    __attribute__((address_space(3))) T* tb = (__attribute__((address_space(3))) T*)tb_;
    const int i = c + 1;
    const int lane = threadIdx.x & 63;
    const int c0 = __builtin_amdgcn_readfirstlane(c - lane);
    const int ieE = min(c0 + 65, NN), ieW = c0;
    kcdp eu = (kcdp)wave_uniform(e_);
    const int g0u = __builtin_amdgcn_readfirstlane(g0);
    double eS = e[g0 * NP1 + i], eC = e[(g0 + 1) * NP1 + i];
    constexpr int B = R < 16 ? R : 16;
#pragma unroll 1
    for (int r0 = 0; r0 < R; r0 += B) {
        double eN[B], eEe[B], eWe[B];
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int j = g0 + r0 + k + 1, ju = g0u + r0 + k + 1;
            eN[k] = e[min(j + 1, NN) * NP1 + i];
            eEe[k] = SE ? eu[ju * NP1 + ieE] : e[ju * NP1 + ieE];
            eWe[k] = SE ? eu[ju * NP1 + ieW] : e[ju * NP1 + ieW];
        }
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int r = r0 + k, g = g0 + r, j = g + 1;
            const bool in = c < NN - 1 && g < NN - 1;
            const double S = from_next_lane(eC, eEe[k]) + from_prev_lane(eC, eWe[k]) + eN[k] + eS;
            const double rs = 1.0 / sqrt(eC * S);   // h / sqrt(eC S) and sqrt(eC / S) from one root
            sd[g * NN + c] = in ? (SD)(h * rs) : SD(1);
            tb[NN + 1 + r * NN] = in ? (T)(eC * rs) : T(0);
            eS = eC;
            eC = (j + 1 <= NN) ? eN[k] : 0.0;
        }
    }
}

// One particle's solve by the whole workgroup (NN * NN / R threads); `smem` holds at least
// onchip_smem<T, NN, R, DST>() bytes.  Used by the per-grid kernel and by the mixed-grid one.
template <typename T, int NN, int R, bool DST, bool ADJ, bool SE = true, bool AONLY = false>
__device__ __forceinline__ void cg_onchip_body(const SolveArgs& a, const int64_t row, const int32_t* __restrict__ obs,
                                               unsigned char* smem, SolveShared& sh,
                                               const _Float16* __restrict__ Stab, const float* __restrict__ lamtab) {
    // AONLY: the adjoint problem alone, the forward solution already in x64 from an earlier launch
    // (whose iteration count, or -1 for a failed solve, is in iters unless the caller gave w)
    static_assert(!AONLY || ADJ, "adjoint-only needs the adjoint pass");
    int prev_iters = 0;
    if constexpr (AONLY) {
        prev_iters = (a.iters && !a.fwd_given) ? __builtin_amdgcn_readfirstlane(a.iters[row]) : 0;
        if (prev_iters < 0) return;   // no forward solution: the row keeps iters = -1 (gradient NaN)
    }
    constexpr int NT = NN * NN / R;
    constexpr int NW = NT / 64;
    constexpr int NP1 = NN + 1;
    constexpr int PAD = NN + 1;
    using DS = DstShape<NN, NW>;
    static_assert(!DST || NN >= 32, "transform tiling");
    static_assert(NW <= 16, "reduction slots");
    // FP64 passes as separate, unrolled functions (wide strips); inline loops otherwise
    constexpr bool SPLIT = R >= 32;
    double* red1 = sh.red1;
    double* red2 = sh.red2;
    double* src_w = g_src_w;   // module-level: the residual function reads them by name
    int* src_at = g_src_at;
    T* ly = reinterpret_cast<T*>(smem);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c = tid % NN, b = tid / NN;
    const int i = c + 1;
    const double* e = a.e + row * a.e_stride;
    double* x64 = a.x64 + row * a.x_stride;
    // D^{-1/2} is a scaling of the inner system, so with FP32 inner solves it is kept in FP32 (the
    // update applies the same values the residual was scaled by); FP64 inner solves keep FP64.
    // Either way it starts at the particle's own FP64 row: a mixed-grid launch keeps FP64 rows for
    // the global-memory solver in the same workspace.
    using SD = typename std::conditional<std::is_same<T, float>::value, float, double>::type;
    SD* sd = reinterpret_cast<SD*>(a.sd + row * a.sd_stride);
    const double h = 1.0 / NN, inv_h2 = (double)NN * (double)NN;
    // own node of row r: tb[NN + 1 + r * NN]; east +1, west -1, north +NN, south -NN
    T* tb = ly + PAD + b * R * NN + c - NN - 1;

    for (int k = tid; k < PAD; k += NT) {
        ly[k] = T(0);
        ly[PAD + NN * NN + k] = T(0);
    }
    // ---- setup: D^{-1/2} (workspace, in SD) and t (registers), staged through the thread's own LDS slots
    if constexpr (SPLIT) {
        strip_setup<T, NN, R, SD, SE>(e, sd, tb, c, b * R);
    } else {
        // column i of e, rows j-1, j, j+1 carried along the strip (j = g + 1)
        double eS = e[(b * R) * NP1 + i], eC = e[(b * R + 1) * NP1 + i];
#pragma unroll 1
        for (int r = 0; r < R; ++r) {
            const int g = b * R + r, j = g + 1;
            const double eN = (j + 1 <= NN) ? e[(j + 1) * NP1 + i] : 0.0;
            double sdv = 1.0, tv = 0.0;
            if (c < NN - 1 && g < NN - 1) {
                const double S = e[j * NP1 + i + 1] + e[j * NP1 + i - 1] + eN + eS;
                const double rs = 1.0 / sqrt(eC * S);   // h / sqrt(eC S) and sqrt(eC / S) from one root
                sdv = h * rs;
                tv = eC * rs;
            }
            sd[g * NN + c] = (SD)sdv;
            tb[NN + 1 + r * NN] = (T)tv;
            eS = eC;
            eC = eN;
        }
    }
    T t[R];
#pragma unroll
    for (int r = 0; r < R; ++r) t[r] = tb[NN + 1 + r * NN];
    __syncthreads();

    // z = L^{-1} r into Z[g][c] (LDS), with the barriers of the four products
    int napp = 0;   // preconditioner applications (same in every thread)
    auto precondition = [&](const T (&rin)[R], double rrin) __attribute__((always_inline)) {
        if constexpr (DST) {
            dst_apply<T, NN, R, NW>(rin, rrin, smem, Stab, lamtab, c, b, wave, lane);
            ++napp;
        }
    };
    auto zval = [&](int r) __attribute__((always_inline)) -> T {
        if constexpr (DST) {
            const float* Z = reinterpret_cast<const float*>(smem + 2 * NN * DS::LD * 2);
            return (T)Z[(b * R + r) * DS::LDZ + c];
        } else {
            return T(0);
        }
    };
    // observations of the forward solution: G, Phi, and the adjoint's sources (G - y) / sigma^2
    auto observe = [&](bool good) {
        __syncthreads();
        double val = 0.0;
        if (tid < a.n_obs) {
            const int node = obs[tid];
            const int jj = node / NP1, ii = node % NP1;
            const bool in = ii >= 1 && ii <= NN - 1 && jj >= 1 && jj <= NN - 1;
            if (in) val = x64[(jj - 1) * NN + ii - 1];
            if (!good) val = NAN;
            if (a.G) a.G[row * a.n_obs + tid] = val;
            src_w[tid] = 2.0 * a.inv2s2 * (val - a.y[tid]);
            src_at[tid] = in ? (jj - 1) * NN + ii - 1 : -1;
        }
        if (tid < 64) {
            const double dlt = (tid < a.n_obs) ? val - a.y[tid] : 0.0;
            const double s = wave_sum(dlt * dlt);
            if (tid == 0 && a.phi) a.phi[row] = good ? s * a.inv2s2 : INFINITY;
        }
        __syncthreads();
    };

    // ---- pass 0: forward problem A w = f into x64 (skipped when x64 already holds w);
    //      pass 1 (ADJ): adjoint problem A lam = P^T (P w - y) / sigma^2 into a.lam
    const int first = (ADJ && (AONLY || a.fwd_given)) ? 1 : 0, last = ADJ ? 1 : 0;
    int total = 0, sweeps = 0, solves = 0;
    bool ok = true;
    T x[R], rv[R], p[R], q[R];
#pragma unroll 1
    for (int pass_ = first; pass_ <= last && ok; ++pass_) {
        const int pass = AONLY ? 1 : (ADJ ? pass_ : 0);
        if (pass == 1 && first == 1) observe(true);
        double* xo = pass ? a.lam + row * a.lam_stride : x64;
        auto rhs = [&](int flat) __attribute__((always_inline)) -> double {
            if (pass == 0) return a.f;
            double s = 0.0;
            for (int k = 0; k < a.n_obs; ++k) s += (src_at[k] == flat) ? src_w[k] : 0.0;
            return s;
        };
        ok = false;
        double fnorm = 0.0;
        // ---- refinement sweeps
        for (int sweep = 0;; ++sweep) {
            ++sweeps;
            double acc = 0.0;
            if constexpr (SPLIT) {
                acc = (pass == 1) ? strip_residual<T, NN, R, true, SD, SE>(e, xo, sd, tb, c, b * R, sweep == 0, a.f, src_w,
                                                                   src_at, a.n_obs)
                                  : strip_residual<T, NN, R, false, SD, SE>(e, xo, sd, tb, c, b * R, sweep == 0, a.f, src_w,
                                                                    src_at, a.n_obs);
            } else
            if (sweep == 0) {
#pragma unroll 1
                for (int r = 0; r < R; ++r) {
                    const int g = b * R + r;
                    T out = T(0);
                    if (c < NN - 1 && g < NN - 1) {
                        const double f = rhs(g * NN + c);
                        acc += f * f;
                        out = (T)((double)sd[g * NN + c] * f);
                    }
                    tb[NN + 1 + r * NN] = out;
                }
            } else {
                // r = f - A x in FP64; column i of e and x carried along the strip
                const int g0 = b * R;
                double eS = e[g0 * NP1 + i], eC = e[(g0 + 1) * NP1 + i];
                double xS = (g0 > 0 && c < NN - 1) ? xo[(g0 - 1) * NN + c] : 0.0;
                double xC = (g0 < NN - 1 && c < NN - 1) ? xo[g0 * NN + c] : 0.0;
#pragma unroll 1
                for (int r = 0; r < R; ++r) {
                    const int g = g0 + r, j = g + 1;
                    const double eN = (j + 1 <= NN) ? e[(j + 1) * NP1 + i] : 0.0;
                    const double xN = (g + 1 < NN - 1 && c < NN - 1) ? xo[(g + 1) * NN + c] : 0.0;
                    T out = T(0);
                    if (c < NN - 1 && g < NN - 1) {
                        const double xE = (c + 1 < NN - 1) ? xo[g * NN + c + 1] : 0.0;
                        const double xW = (c > 0) ? xo[g * NN + c - 1] : 0.0;
                        const double res = rhs(g * NN + c) -
                                           eC * inv_h2 *
                                               (e[j * NP1 + i + 1] * (xC - xE) + e[j * NP1 + i - 1] * (xC - xW) +
                                                eN * (xC - xN) + eS * (xC - xS));
                        acc += res * res;
                        out = (T)((double)sd[g * NN + c] * res);
                    }
                    tb[NN + 1 + r * NN] = out;
                    eS = eC;
                    eC = eN;
                    xS = xC;
                    xC = xN;
                }
            }
            const double rr64 = block_sum<NW>(acc, red2);
            if (sweep == 0) fnorm = sqrt(rr64);
            if (sqrt(rr64) <= a.tol64 * fnorm) {   // at sweep 0 only for a zero right-hand side
                ok = true;
                if (sweep == 0) {
#pragma unroll 1
                    for (int r = 0; r < R; ++r) xo[(b * R + r) * NN + c] = 0.0;
                }
                break;
            }
            if (!(rr64 < INFINITY) || sweep >= a.max_sweeps || total >= a.max_iter) break;

            double tacc = 0.0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                rv[r] = tb[NN + 1 + r * NN];
                x[r] = T(0);
                tacc += (double)rv[r] * (double)rv[r];
            }
            double rr, rz;
            if constexpr (DST) {
                rr = block_sum<NW>(tacc, red1);   // also the transform's input scale
                __syncthreads();                  // the transform buffers alias the staging slots
                precondition(rv, rr);
                double zacc = 0.0;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    p[r] = zval(r);
                    zacc += (double)rv[r] * (double)p[r];
                }
                rz = block_sum<NW>(zacc, red2);
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) p[r] = rv[r];
                rr = block_sum<NW>(tacc, red1);
                rz = rr;
            }
            // the inner solve reduces its residual by tol_inner, or only as far as the outer tolerance
            // still needs (a margin of 10 for the Jacobi-scaled norm), whichever is less work
            const double red = fmin(0.5, fmax(a.tol_inner, 0.1 * a.tol64 * fnorm / sqrt(rr64)));
            const double target = red * red * rr;
            bool broke = false;
            while (rr > target) {
                if (total >= a.max_iter) break;
#pragma unroll
                for (int r = 0; r < R; ++r) tb[NN + 1 + r * NN] = t[r] * p[r];
                if constexpr (DST) {   // the transform buffers alias the padding: zero it again
                    for (int k = tid; k < PAD; k += NT) {
                        ly[k] = T(0);
                        ly[PAD + NN * NN + k] = T(0);
                    }
                }
                __syncthreads();
                T pq_acc = T(0);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const T yE = tb[NN + 2 + r * NN];
                    const T yW = tb[NN + r * NN];
                    const T yN = (r + 1 < R) ? t[r + 1] * p[r + 1] : tb[NN + 1 + R * NN];
                    const T yS = (r > 0) ? t[r - 1] * p[r - 1] : tb[1];
                    q[r] = p[r] - t[r] * ((yE + yW) + (yN + yS));
                    pq_acc += p[r] * q[r];
                }
                const double pq = block_sum<NW>((double)pq_acc, red1);
                if (!(pq > 0.0) || !(pq < INFINITY)) { broke = true; break; }
                const T alpha = (T)(rz / pq);
                T r_acc = T(0);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    x[r] += alpha * p[r];
                    rv[r] -= alpha * q[r];
                    r_acc += rv[r] * rv[r];
                }
                rr = block_sum<NW>((double)r_acc, red2);
                ++total;
                if (!(rr > target)) break;
                if constexpr (DST) {
                    precondition(rv, rr);
                    T z[R];
                    T rz_acc = T(0);
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        z[r] = zval(r);
                        rz_acc += rv[r] * z[r];
                    }
                    const double rzn = block_sum<NW>((double)rz_acc, red1);
                    const T beta = (T)(rzn / rz);
                    rz = rzn;
#pragma unroll
                    for (int r = 0; r < R; ++r) p[r] = z[r] + beta * p[r];
                } else {
                    const T beta = (T)(rr / rz);
                    rz = rr;
#pragma unroll
                    for (int r = 0; r < R; ++r) p[r] = rv[r] + beta * p[r];
                }
            }
            // xo += D^{-1/2} y, staged through the thread's own LDS slots
            __syncthreads();
#pragma unroll
            for (int r = 0; r < R; ++r) tb[NN + 1 + r * NN] = x[r];
            if constexpr (SPLIT) {
                strip_update<T, NN, R, SD>(xo, sd, tb, c, b * R, sweep == 0);
            } else {
#pragma unroll 1
                for (int r = 0; r < R; ++r) {
                    const int g = b * R + r;
                    const double corr = (double)sd[g * NN + c] * (double)tb[NN + 1 + r * NN];
                    xo[g * NN + c] = (sweep == 0) ? corr : xo[g * NN + c] + corr;
                }
            }
            __syncthreads();
            if (broke) break;
        }
        ++solves;
        if (pass == 0) observe(ok);
    }
    if constexpr (ADJ && NN >= 64) {   // dPhi/du from the final w and lam (the barrier closing the last sweep made them whole)
        if (a.du && ok) strip_dphi<NN, R, AONLY>(e, x64, a.lam + row * a.lam_stride, a.du + row * a.du_stride, c, b * R);
    }

    // ---- bookkeeping
    if (tid == 0) {
        if (a.iters) a.iters[row] = ok ? prev_iters + total : -1;
        if (!ok) atomicOr(a.flags, SMC_FLAG_NOCONV);
        if (a.stats) {
            atomicAdd(&a.stats[0], (unsigned long long)total);
            atomicAdd(&a.stats[1], (unsigned long long)sweeps);
            atomicAdd(&a.stats[2], (unsigned long long)solves);
            atomicAdd(&a.stats[3], (unsigned long long)napp);
        }
    }
    __syncthreads();   // the next body may reuse the LDS
}

template <typename T, int NN, int R, bool DST, bool ADJ, bool AONLY = false>
__global__ __launch_bounds__(NN * NN / R) void cg_onchip(SolveArgs a, const _Float16* __restrict__ Stab,
                                                         const float* __restrict__ lamtab) {
    __shared__ __align__(16) unsigned char smem[onchip_smem<T, NN, R, DST>()];
    __shared__ SolveShared sh;
    cg_onchip_body<T, NN, R, DST, ADJ, true, AONLY>(a, blockIdx.x, a.obs, smem, sh, Stab, lamtab);
}

// Same method (Jacobi-scaled CG, product form) with every vector in global memory, for grids
// whose vectors do not fit in one workgroup's registers and LDS; 1024 threads stride over
// the nodes of one particle.
// The fast-Poisson preconditioner z = L^{-1} r of a 256 x 256 grid whose vectors live in global
// memory (one workgroup of 16 waves).  L^{-1} = S diag(1 / (lam_i + lam_j)) S is applied as four
// passes X <- (X S)^T over a single FP16 copy of the grid in LDS: each pass is a batch of
// independent 1D sine transforms along the rows, and the transposed write-back turns the next pass
// into the transform along the other axis.  Wave w owns output columns 16w..16w+15, keeps its
// 16-column slice of S in registers, holds its 16 result tiles until every wave has read X, then
// writes them transposed.  The second pass applies 1 / (lam_i + lam_j); the fourth writes z (FP32).
constexpr int D256_LD = 256 + 8;
constexpr int D256_BYTES = 256 * D256_LD * 2;

// LDS named at module level: the mixed-grid solve's bodies and the 256^2 transform below are
// functions of their own (register-allocated apart from their callers), and LDS they name directly
// keeps its LDS instructions, where a pointer passed in would turn into generic accesses.
constexpr int MIXED_SMEM = cmax(onchip_smem<float, 128, 16, true>(),
                                cmax(onchip_smem<float, 64, 4, true>(), onchip_smem<double, 64, 4, false>()));
__shared__ __align__(16) unsigned char g_mixed_smem[MIXED_SMEM];

// Four-wide loads and stores of the global solvers' vectors (FP32 or FP64).
template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };
template <typename T> using vec4_t = typename Vec4<T>::type;
template <typename T>
__device__ __forceinline__ vec4_t<T> ld4(const T* p) { return *reinterpret_cast<const vec4_t<T>*>(p); }
template <typename T>
__device__ __forceinline__ void st4(T* p, T a, T b, T c, T d) {
    vec4_t<T> v;
    v.x = a; v.y = b; v.z = c; v.w = d;
    *reinterpret_cast<vec4_t<T>*>(p) = v;
}

// The transform of the global-memory solvers (one workgroup of 16 waves, vectors of type T in
// global memory, grid NN = 128 or 256): X holds fp16(r 2^-ex), z is scaled back by 2^ex.  Wave w
// owns output column tile w mod (NN / 16) and NN / 256 of its row tiles.  With `staged`, X already
// holds the scaled residual (written by the caller's residual update with the same ex); with
// `rz`, the thread's share of sum r z is accumulated while z is stored.
template <int NN, typename T>
__device__ __forceinline__ void dstg_apply(const T* __restrict__ r, T* __restrict__ z, _Float16* X,
                                           const _Float16* __restrict__ S, const float* __restrict__ lam, int ex,
                                           bool staged = false, double* rz = nullptr) {
    constexpr int LD = NN + 8, KS = NN / 32, NBT = NN / 16, WPC = 16 / NBT, RT = NBT / WPC;
    static_assert(NBT * WPC == 16 && RT * WPC == NBT, "16 waves over the output tiles");
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, lk = lane >> 4, cb = wave % NBT, ra0 = (wave / NBT) * RT;
    const float sc = ldexpf(1.0f, -ex), unsc = ldexpf(1.0f, ex);
    hf8 sB[KS];   // B operand: S[k][16 cb + lr] = S[16 cb + lr][k] (S is symmetric)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) sB[ks] = *reinterpret_cast<const hf8*>(S + (16 * cb + lr) * NN + 32 * ks + 8 * lk);
    for (int e = staged ? NN * NN : tid; e < NN * NN / 8; e += 1024) {   // X = fp16(r 2^-ex), row-major
        const int g = e / (NN / 8), c0 = (e % (NN / 8)) * 8;
        const vec4_t<T> u0 = ld4(r + g * NN + c0), u1 = ld4(r + g * NN + c0 + 4);
        const T s = (T)sc;
        hf8 v;
        v[0] = (_Float16)(float)(u0.x * s); v[1] = (_Float16)(float)(u0.y * s); v[2] = (_Float16)(float)(u0.z * s);
        v[3] = (_Float16)(float)(u0.w * s); v[4] = (_Float16)(float)(u1.x * s); v[5] = (_Float16)(float)(u1.y * s);
        v[6] = (_Float16)(float)(u1.z * s); v[7] = (_Float16)(float)(u1.w * s);
        *reinterpret_cast<hf8*>(X + g * LD + c0) = v;
    }
    __syncthreads();
    const float lam_c = lam[16 * cb + lr];
#pragma unroll 1
    for (int step = 0; step < 4; ++step) {
        hf4 out[RT];
#pragma unroll
        for (int i = 0; i < RT; ++i) {   // P[i][j] = sum_k X[i][k] S[k][j], i in row tile ra, j in cb
            const int ra = ra0 + i;
            f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
                acc = mfma_f16(*reinterpret_cast<const hf8*>(X + (16 * ra + lr) * LD + 32 * ks + 8 * lk), sB[ks], acc);
            if (step == 1) {
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[v] *= __builtin_amdgcn_rcpf(lam[16 * ra + 4 * lk + v] + lam_c);
            }
            if (step == 3) {   // z[j][i] = P[i][j]
                const int at = (16 * cb + lr) * NN + 16 * ra + 4 * lk;
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[v] *= unsc;
                st4<T>(z + at, (T)acc[0], (T)acc[1], (T)acc[2], (T)acc[3]);
                if (rz) {
                    const vec4_t<T> rv4 = ld4(r + at);
                    *rz += (double)rv4.x * (double)acc[0] + (double)rv4.y * (double)acc[1] +
                           (double)rv4.z * (double)acc[2] + (double)rv4.w * (double)acc[3];
                }
            } else {
#pragma unroll
                for (int v = 0; v < 4; ++v) out[i][v] = (_Float16)acc[v];
            }
        }
        if (step < 3) {
            __syncthreads();   // every wave has finished reading X
#pragma unroll
            for (int i = 0; i < RT; ++i)
                *reinterpret_cast<hf4*>(X + (16 * cb + lr) * LD + 16 * (ra0 + i) + 4 * lk) = out[i];
            __syncthreads();
        }
    }
    __syncthreads();   // z complete for every thread of the workgroup
}

// The transform as a function of its own, on the module-level buffer the global solvers stage X
// in: inlined into the CG loop it competes for that loop's registers and both spill.  `staged`: r
// is already in X as fp16(r 2^-ex); `want_rz`: returns this thread's share of r.z (else 0).
static_assert(D256_BYTES <= MIXED_SMEM, "256^2 transform LDS");
template <int NN, typename T>
__device__ __noinline__ double dstg_precondition(const T* r, T* z, const _Float16* S, const float* lam, int staged,
                                                 int ex, int want_rz) {
    double rz = 0.0;
    dstg_apply<NN, T>(r, z, reinterpret_cast<_Float16*>(g_mixed_smem), S, lam, ex, staged != 0,
                      want_rz ? &rz : nullptr);
    return rz;
}

// a * b + c with one rounding, for float and double alike
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <typename T>
__device__ __forceinline__ vec4_t<T> fma4(T a, vec4_t<T> b, vec4_t<T> c) {
    vec4_t<T> o;
    o.x = fma_t(a, b.x, c.x); o.y = fma_t(a, b.y, c.y); o.z = fma_t(a, b.z, c.z); o.w = fma_t(a, b.w, c.w);
    return o;
}

__global__ __launch_bounds__(1024) void dst256_apply_kernel(const float* __restrict__ rin, float* __restrict__ zout,
                                                            const _Float16* __restrict__ Stab,
                                                            const float* __restrict__ lamtab) {
    __shared__ __align__(16) _Float16 X[256 * D256_LD];
    __shared__ double red[16];
    const int64_t base = (int64_t)blockIdx.x * 256 * 256;
    double acc = 0.0;
    for (int k = threadIdx.x; k < 256 * 256; k += 1024) acc += (double)rin[base + k] * (double)rin[base + k];
    const double rr = block_sum<16>(acc, red);
    dstg_apply<256, float>(rin + base, zout + base, X, Stab, lamtab, norm_exponent(rr) + 3);
}

// DST: fast-Poisson-preconditioned CG on grid DN (128 or 256; X = its transform's LDS);
// otherwise Jacobi-scaled CG on any grid.  T = float (inside FP64 refinement) or double.
template <typename T, bool ADJ, bool DST = false, int DN = 256>
__device__ __forceinline__ void cg_global_body(const SolveArgs& a, const int64_t row, const int NN,
                                               const int32_t* __restrict__ obs, SolveShared& sh,
                                               _Float16* X = nullptr, const _Float16* __restrict__ Stab = nullptr,
                                               const float* __restrict__ lamtab = nullptr) {
    constexpr int NW = 16;
    using T4 = vec4_t<T>;
    double* red1 = sh.red1;
    double* red2 = sh.red2;
    double* src_w = sh.src_w;
    int* src_at = sh.src_at;
    const int tid = threadIdx.x;
    const int NP1 = NN + 1;
    const int nodes = NN * NN;
    const double* e = a.e + row * a.e_stride;
    double* x64 = a.x64 + row * a.x_stride;
    // D^{-1/2} only scales the inner system: FP32 with FP32 inner solves (the update applies the
    // values the residual was scaled by), inside the particle's own FP64 row
    using SD = typename std::conditional<std::is_same<T, float>::value, float, double>::type;
    SD* sd = reinterpret_cast<SD*>(a.sd + row * a.sd_stride);
    T* vb = reinterpret_cast<T*>(reinterpret_cast<double*>(a.vec) + row * a.vec_stride);
    T* tv = vb;
    T* xv = vb + nodes;
    T* rv = vb + 2 * nodes;
    T* pv = vb + 3 * nodes;
    T* qv = vb + 4 * nodes;
    T* yv = vb + 5 * nodes;   // t p (Jacobi path)
    T* zv = yv;               // preconditioned residual (DST path, which needs no y)
    T* pv2 = vb + 6 * nodes;  // second search-direction buffer (DST path): seven vectors
    const double h = 1.0 / NN, inv_h2 = (double)NN * (double)NN;
    auto interior = [&](int g, int c) { return c < NN - 1 && g < NN - 1; };
    int napp = 0;

    for (int k = tid; k < nodes; k += 1024) {
        const int g = k / NN, c = k % NN, i = c + 1, j = g + 1;
        double sdv = 1.0, tt = 0.0;
        if (interior(g, c)) {
            const double eP = e[j * NP1 + i];
            const double S = e[j * NP1 + i + 1] + e[j * NP1 + i - 1] + e[(j + 1) * NP1 + i] + e[(j - 1) * NP1 + i];
            const double rs = 1.0 / sqrt(eP * S);   // h / sqrt(eP S) and sqrt(eP / S) from one root
            sdv = h * rs;
            tt = eP * rs;
        }
        sd[k] = (SD)sdv;
        tv[k] = (T)tt;
    }
    __syncthreads();

    // observations of the forward solution: G, Phi, and the adjoint's sources (G - y) / sigma^2
    auto observe = [&](bool good) {
        __syncthreads();
        double val = 0.0;
        if (tid < a.n_obs) {
            const int node = obs[tid];
            const int jj = node / NP1, ii = node % NP1;
            const bool in = ii >= 1 && ii <= NN - 1 && jj >= 1 && jj <= NN - 1;
            if (in) val = x64[(jj - 1) * NN + ii - 1];
            if (!good) val = NAN;
            if (a.G) a.G[row * a.n_obs + tid] = val;
            src_w[tid] = 2.0 * a.inv2s2 * (val - a.y[tid]);
            src_at[tid] = in ? (jj - 1) * NN + ii - 1 : -1;
        }
        if (tid < 64) {
            const double dlt = (tid < a.n_obs) ? val - a.y[tid] : 0.0;
            const double s = wave_sum(dlt * dlt);
            if (tid == 0 && a.phi) a.phi[row] = good ? s * a.inv2s2 : INFINITY;
        }
        __syncthreads();
    };

    // pass 0: forward problem into x64 (skipped when given); pass 1 (ADJ): adjoint problem into a.lam
    const int first = (ADJ && a.fwd_given) ? 1 : 0, last = ADJ ? 1 : 0;
    int total = 0, sweeps = 0, solves = 0;
    bool ok = true;
    for (int pass_ = first; pass_ <= last && ok; ++pass_) {
        const int pass = ADJ ? pass_ : 0;
        if (pass == 1 && first == 1) observe(true);
        double* xo = pass ? a.lam + row * a.lam_stride : x64;
        auto rhs = [&](int flat) -> double {
            if (pass == 0) return a.f;
            double s = 0.0;
            for (int k = 0; k < a.n_obs; ++k) s += (src_at[k] == flat) ? src_w[k] : 0.0;
            return s;
        };
        ok = false;
        double fnorm = 0.0;
        for (int sweep = 0;; ++sweep) {
            ++sweeps;
            // residual pass: r = D^{-1/2} (f - A x) in T, with |f - A x|^2 in FP64 and |r|^2 summed on
            // the way (the fast-Poisson path writes r only: its first transform writes p = z, and the
            // first update sets x = alpha p)
            double acc = 0.0, tacc = 0.0;
            for (int k = tid; k < nodes; k += 1024) {
                const int g = k / NN, c = k % NN, i = c + 1, j = g + 1;
                T rk = T(0);
                if (interior(g, c)) {
                    double res = rhs(k);
                    if (sweep > 0) {
                        const double xP = xo[k];
                        const double xE = (c + 1 < NN - 1) ? xo[k + 1] : 0.0;
                        const double xW = (c > 0) ? xo[k - 1] : 0.0;
                        const double xN = (g + 1 < NN - 1) ? xo[k + NN] : 0.0;
                        const double xS = (g > 0) ? xo[k - NN] : 0.0;
                        res -= e[j * NP1 + i] * inv_h2 *
                               (e[j * NP1 + i + 1] * (xP - xE) + e[j * NP1 + i - 1] * (xP - xW) +
                                e[(j + 1) * NP1 + i] * (xP - xN) + e[(j - 1) * NP1 + i] * (xP - xS));
                    }
                    acc += res * res;
                    rk = (T)((double)sd[k] * res);
                    tacc += (double)rk * (double)rk;
                }
                rv[k] = rk;
                if constexpr (!DST) {
                    pv[k] = rk;
                    xv[k] = T(0);
                }
            }
            const double rr64 = block_sum<NW>(acc, red2);
            double rr = block_sum<NW>(tacc, red1);
            if (sweep == 0) fnorm = sqrt(rr64);
            if (sqrt(rr64) <= a.tol64 * fnorm) {   // at sweep 0 only for a zero right-hand side
                ok = true;
                if (sweep == 0)
                    for (int k = tid; k < nodes; k += 1024) xo[k] = 0.0;
                break;
            }
            if (!(rr64 < INFINITY) || sweep >= a.max_sweeps || total >= a.max_iter) break;

            // the inner solve reduces its residual by tol_inner, or only as far as the outer tolerance
            // still needs (a margin of 10 for the Jacobi-scaled norm), whichever is less work
            const double red = fmin(0.5, fmax(a.tol_inner, 0.1 * a.tol64 * fnorm / sqrt(rr64)));
            const double target = red * red * rr;
            bool broke = false;
            bool have_x = true;   // x holds this sweep's correction (else it is zero)
            if constexpr (DST) {
                // p = z = L^{-1} r straight from the transform, with r.z summed as z is stored
                T* pc = pv;    // current search direction
                T* pn = pv2;   // the next one, written while pc is read (neighbours read pc)
                double rz = block_sum<NW>(dstg_precondition<DN, T>(rv, pc, Stab, lamtab, 0, norm_exponent(rr) + 3, 1),
                                          red2);
                ++napp;
                // Per iteration three passes over the global vectors: the stencil, which first forms
                // p <- z + beta p (on the fly at the neighbours too; p is double-buffered because
                // neighbouring rows read the old one), the x/r update (which also stages fp16(r 2^-ex)
                // for the transform in LDS), and the transform (z stored, r.z accumulated).  The
                // staged scale comes from the norm before the update (the new one is summed in the
                // same pass), 2^-3 below unit norm: the residual would have to grow 39-fold in one
                // iteration to overflow FP16 (the largest intermediate is then below
                // 1 / (2 lam_0) / 8 < 1700 times the growth).
                bool first_it = true;   // p = z as stored, x = 0
                T beta = T(0);
                while (rr > target) {
                    if (total >= a.max_iter) break;
                    const int ex = norm_exponent(rr) + 3;
                    const T sc = (T)ldexpf(1.0f, -ex);
                    T pq_acc = T(0);
                    // p at a node: z + beta p_old (the same fused multiply-add wherever it is formed)
                    auto pnew = [&](int k) -> T { return first_it ? pc[k] : fma_t(beta, pc[k], zv[k]); };
                    for (int k = 4 * tid; k < nodes; k += 4096) {   // four consecutive nodes of a row
                        const int g = k / NN, c = k % NN;
                        const int kN = (g < NN - 1) ? k + NN : k, kS = (g > 0) ? k - NN : k;
                        const int kW = (c > 0) ? k - 1 : k, kE = min(k + 4, nodes - 1);
                        T4 p4 = ld4(pc + k), pN = ld4(pc + kN), pS = ld4(pc + kS);
                        const T4 t4 = ld4(tv + k), tN = ld4(tv + kN), tS = ld4(tv + kS);
                        if (!first_it) {
                            const T4 z4 = ld4(zv + k), zN = ld4(zv + kN), zS = ld4(zv + kS);
                            p4 = fma4(beta, p4, z4);
                            pN = fma4(beta, pN, zN);
                            pS = fma4(beta, pS, zS);
                        }
                        const T yW0 = (c > 0) ? tv[kW] * pnew(kW) : T(0), yE3 = tv[kE] * pnew(kE);
                        const T t_[4] = {t4.x, t4.y, t4.z, t4.w};
                        const T pn_[4] = {pN.x, pN.y, pN.z, pN.w}, tn[4] = {tN.x, tN.y, tN.z, tN.w};
                        const T ps[4] = {pS.x, pS.y, pS.z, pS.w}, ts[4] = {tS.x, tS.y, tS.z, tS.w};
                        T p_[4] = {p4.x, p4.y, p4.z, p4.w};
                        T yc[4], q_[4];
#pragma unroll
                        for (int m = 0; m < 4; ++m) {
                            if (!interior(g, c + m)) p_[m] = T(0);
                            yc[m] = t_[m] * p_[m];
                        }
#pragma unroll
                        for (int m = 0; m < 4; ++m) {
                            const T yE = (m < 3) ? yc[m < 3 ? m + 1 : 3] : yE3;
                            const T yW = (m > 0) ? yc[m > 0 ? m - 1 : 0] : yW0;
                            const T yN = tn[m] * pn_[m];
                            const T yS = (g > 0) ? ts[m] * ps[m] : T(0);
                            q_[m] = interior(g, c + m) ? p_[m] - t_[m] * ((yE + yW) + (yN + yS)) : T(0);
                            pq_acc += p_[m] * q_[m];
                        }
                        if (!first_it) st4(pn + k, p_[0], p_[1], p_[2], p_[3]);
                        st4(qv + k, q_[0], q_[1], q_[2], q_[3]);
                    }
                    const double pq = block_sum<NW>((double)pq_acc, red1);   // its barriers publish p and q
                    if (!first_it) {
                        T* sw = pc;
                        pc = pn;
                        pn = sw;
                    }
                    if (!(pq > 0.0) || !(pq < INFINITY)) {
                        have_x = !first_it;
                        broke = true;
                        break;
                    }
                    const T alpha = (T)(rz / pq);
                    T r_acc = T(0);
                    for (int k = 4 * tid; k < nodes; k += 4096) {
                        const T4 p4 = ld4(pc + k);
                        T4 x4;
                        if (first_it) {
                            x4.x = alpha * p4.x; x4.y = alpha * p4.y; x4.z = alpha * p4.z; x4.w = alpha * p4.w;
                        } else {
                            x4 = ld4(xv + k);
                            x4.x += alpha * p4.x; x4.y += alpha * p4.y; x4.z += alpha * p4.z; x4.w += alpha * p4.w;
                        }
                        T4 r4 = ld4(rv + k);
                        const T4 q4 = ld4(qv + k);
                        r4.x -= alpha * q4.x; r4.y -= alpha * q4.y; r4.z -= alpha * q4.z; r4.w -= alpha * q4.w;
                        r_acc += ((r4.x * r4.x + r4.y * r4.y) + (r4.z * r4.z + r4.w * r4.w));
                        st4(xv + k, x4.x, x4.y, x4.z, x4.w);
                        st4(rv + k, r4.x, r4.y, r4.z, r4.w);
                        hf4 b;
                        b[0] = (_Float16)(float)(r4.x * sc); b[1] = (_Float16)(float)(r4.y * sc);
                        b[2] = (_Float16)(float)(r4.z * sc); b[3] = (_Float16)(float)(r4.w * sc);
                        *reinterpret_cast<hf4*>(X + (k / NN) * (DN + 8) + (k % NN)) = b;
                    }
                    rr = block_sum<NW>((double)r_acc, red2);   // its barrier also publishes X
                    ++total;
                    first_it = false;
                    if (!(rr > target)) break;
                    double zacc = dstg_precondition<DN, T>(rv, zv, Stab, lamtab, 1, ex, 1);
                    ++napp;
                    double rzn = block_sum<NW>(zacc, red1);
                    if (!(fabs(rzn) < INFINITY)) {   // the residual outgrew the staged scale: redo from r
                        __syncthreads();
                        zacc = dstg_precondition<DN, T>(rv, zv, Stab, lamtab, 0, norm_exponent(rr) + 3, 1);
                        rzn = block_sum<NW>(zacc, red2);
                        ++napp;
                    }
                    beta = (T)(rzn / rz);
                    rz = rzn;
                }
                if (first_it) have_x = false;   // no update ran: the correction is zero
            } else {
            double rz = rr;
            while (rr > target) {
                if (total >= a.max_iter) break;
                for (int k = tid; k < nodes; k += 1024) yv[k] = tv[k] * pv[k];
                __syncthreads();
                T pq_acc = T(0);
                for (int k = tid; k < nodes; k += 1024) {
                    const int g = k / NN, c = k % NN;
                    T qk = T(0);
                    const T pk = pv[k];
                    if (interior(g, c)) {
                        const T yE = yv[k + 1];
                        const T yW = (c > 0) ? yv[k - 1] : T(0);
                        const T yN = yv[k + NN];
                        const T yS = (g > 0) ? yv[k - NN] : T(0);
                        qk = pk - tv[k] * ((yE + yW) + (yN + yS));
                    }
                    qv[k] = qk;
                    pq_acc += pk * qk;
                }
                const double pq = block_sum<NW>((double)pq_acc, red1);
                if (!(pq > 0.0) || !(pq < INFINITY)) { broke = true; break; }
                const T alpha = (T)(rz / pq);
                T r_acc = T(0);
                for (int k = tid; k < nodes; k += 1024) {
                    xv[k] += alpha * pv[k];
                    const T rk = rv[k] - alpha * qv[k];
                    rv[k] = rk;
                    r_acc += rk * rk;
                }
                const double rrn = block_sum<NW>((double)r_acc, red2);
                ++total;
                const T beta = (T)(rrn / rr);
                rr = rrn;
                rz = rr;
                for (int k = tid; k < nodes; k += 1024) pv[k] = rv[k] + beta * pv[k];
            }
            }
            for (int k = tid; k < nodes; k += 1024) {
                const double corr = have_x ? (double)sd[k] * (double)xv[k] : 0.0;
                xo[k] = (sweep == 0) ? corr : xo[k] + corr;
            }
            __syncthreads();
            if (broke) break;
        }
        ++solves;
        if (pass == 0) observe(ok);
    }

    if (tid == 0) {
        if (a.iters) a.iters[row] = ok ? total : -1;
        if (!ok) atomicOr(a.flags, SMC_FLAG_NOCONV);
        if (a.stats) {
            atomicAdd(&a.stats[0], (unsigned long long)total);
            atomicAdd(&a.stats[1], (unsigned long long)sweeps);
            atomicAdd(&a.stats[2], (unsigned long long)solves);
            if (DST) atomicAdd(&a.stats[3], (unsigned long long)napp);
        }
    }
    __syncthreads();
}

template <typename T, bool ADJ>
__global__ __launch_bounds__(1024) void cg_global(SolveArgs a, int NN) {
    __shared__ SolveShared sh;
    cg_global_body<T, ADJ>(a, blockIdx.x, NN, a.obs, sh);
}

template <typename T, int NN, bool ADJ>
__global__ __launch_bounds__(1024) void cg_global_dst(SolveArgs a, const _Float16* __restrict__ Stab,
                                                      const float* __restrict__ lamtab) {
    __shared__ SolveShared sh;
    cg_global_body<T, ADJ, true, NN>(a, blockIdx.x, NN, a.obs, sh, reinterpret_cast<_Float16*>(g_mixed_smem), Stab,
                                     lamtab);
}

template <typename T, int NN>
static hipError_t run_global_dst(int64_t N, const SolveArgs& a, const void* S, const float* lam, hipStream_t s) {
    const _Float16* Sh = reinterpret_cast<const _Float16*>(S);
    if (a.lam)
        cg_global_dst<T, NN, true><<<dim3((unsigned)N), dim3(1024), 0, s>>>(a, Sh, lam);
    else
        cg_global_dst<T, NN, false><<<dim3((unsigned)N), dim3(1024), 0, s>>>(a, Sh, lam);
    return hipGetLastError();
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

// ------------------------------------------------------------------ several grids in one launch
// Particles on different grids (a per-particle level map) are solved by one persistent launch.
// A work list orders the particles by grid, finest first, so the longest solves start first;
// each workgroup of 1024 threads takes the next list entry from an atomic counter and runs the
// solve body of that particle's grid until the list is exhausted.  The last workgroup to leave
// zeroes the counters for the next launch.

// Work list of a level map: particle ids grouped by grid (largest n first, then the lower level;
// out-of-range levels last, with SMC_FLAG_BADLEVEL); zeroes the two counters.  One workgroup.
__global__ __launch_bounds__(1024) void plan_kernel(int64_t N, const int32_t* __restrict__ level, LevelTable lt,
                                                    int32_t* __restrict__ list, unsigned long long* counters,
                                                    int32_t* flags) {
    __shared__ int wtot[16];
    __shared__ int order[MAX_LEVELS + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) {
        for (int k = 0; k < COUNTER_SEG; ++k) counters[k] = 0;
        bool used[MAX_LEVELS] = {};
        for (int r = 0; r < lt.n_levels; ++r) {
            int best = -1;
            for (int l = 0; l < lt.n_levels; ++l)
                if (!used[l] && (best < 0 || lt.n[l] > lt.n[best])) best = l;
            used[best] = true;
            order[r] = best;
        }
        order[lt.n_levels] = -1;
    }
    __syncthreads();
    int64_t base = 0;
    bool bad = false;
    for (int rank = 0; rank <= lt.n_levels; ++rank) {
        const int target = order[rank];
        const int64_t seg0 = base;
        for (int64_t c0 = 0; c0 < N; c0 += 1024) {
            const int64_t p = c0 + tid;
            bool f = false;
            if (p < N) {
                const int l = level[p];
                f = (target >= 0) ? (l == target) : (l < 0 || l >= lt.n_levels);
                // level -1 parks a particle: listed with the out-of-range ones (no solve) but no error
                bad = bad || (target < 0 && l != -1 && f);
            }
            const unsigned long long m = __ballot(f);
            const int before = __popcll(m & ((1ull << lane) - 1ull));
            if (lane == 0) wtot[wave] = __popcll(m);
            __syncthreads();
            int off = 0, tot = 0;
            for (int w = 0; w < 16; ++w) {
                off += (w < wave) ? wtot[w] : 0;
                tot += wtot[w];
            }
            if (f) list[base + off + before] = (int32_t)p;
            base += tot;
            __syncthreads();
        }
        if (tid == 0) {   // this grid's segment of the list (the last one: no grid)
            const int sl = target >= 0 ? target : MAX_LEVELS;
            counters[COUNTER_SEG + 2 * sl] = (unsigned long long)seg0;
            counters[COUNTER_SEG + 2 * sl + 1] = (unsigned long long)(base - seg0);
        }
    }
    if (tid == 0)   // grids absent from the table hold no particles
        for (int l = lt.n_levels; l < MAX_LEVELS; ++l) counters[COUNTER_SEG + 2 * l + 1] = 0;
    if (__syncthreads_or(bad) && tid == 0 && flags) atomicOr(flags, SMC_FLAG_BADLEVEL);
}

hipError_t launch_plan(int64_t N, const int32_t* level, const LevelTable& lt, int32_t* list,
                       unsigned long long* counters, int32_t* flags, hipStream_t s) {
    plan_kernel<<<dim3(1), dim3(1024), 0, s>>>(N, level, lt, list, counters, flags);
    return hipGetLastError();
}

bool mixed_supported(int n) { return n == 64 || n == 128 || n == 256; }

// Each grid's body as a separate function, so that each is register-allocated on its own (the
// call happens once per particle).  The LDS they share is named directly, not passed by pointer,
// so that the bodies keep their LDS instructions.
__shared__ SolveShared g_mixed_sh;

template <typename T, int NN, int R, bool DST, bool SE = true>
__device__ __noinline__ void mixed_onchip(const SolveArgs& a, int64_t p, const int32_t* obs, const void* S,
                                          const float* lam) {
    static_assert(onchip_smem<T, NN, R, DST>() <= MIXED_SMEM, "mixed-grid LDS");
    cg_onchip_body<T, NN, R, DST, false, SE>(a, p, obs, g_mixed_smem, g_mixed_sh, reinterpret_cast<const _Float16*>(S),
                                         lam);
}

template <typename T>
__device__ __noinline__ void mixed_global(const SolveArgs& a, int64_t p, int n, const int32_t* obs) {
    cg_global_body<T, false>(a, p, n, obs, g_mixed_sh);
}

template <typename T, int NN>
__device__ __noinline__ void mixed_global_dst(const SolveArgs& a, int64_t p, const int32_t* obs, const void* S,
                                              const float* lam) {
    cg_global_body<T, false, true, NN>(a, p, NN, obs, g_mixed_sh, reinterpret_cast<_Float16*>(g_mixed_smem),
                                       reinterpret_cast<const _Float16*>(S), lam);
}

template <int PREC, bool DST>
__global__ __launch_bounds__(1024) void solve_mixed_kernel(SolveArgs a, LevelTable lt,
                                                           const int32_t* __restrict__ level,
                                                           const int32_t* __restrict__ list, int64_t N,
                                                           unsigned long long* counters) {
    __shared__ unsigned long long item_s;
    for (;;) {
        if (threadIdx.x == 0) item_s = atomicAdd(&counters[0], 1ull);
        __syncthreads();
        // the item as a wave-uniform value: the loop exit and the grid dispatch below must compile
        // as uniform branches, or the barriers in the loop would not be met by every lane alike
        const int64_t item = __builtin_amdgcn_readfirstlane((int)(item_s < (unsigned long long)N ? item_s : N));
        __syncthreads();
        if (item >= N) break;
        const int64_t p = __builtin_amdgcn_readfirstlane(list[item]);
        const int l = __builtin_amdgcn_readfirstlane(level[p]);
        const int n = (l >= 0 && l < lt.n_levels) ? lt.n[l] : 0;
        const void* S = n ? lt.S[l] : nullptr;   // FP16 sine table
        if constexpr (PREC == SMC_FP32_REFINE) {
            if (n == 64)
                mixed_onchip<float, 64, 4, DST>(a, p, lt.obs[l], S, lt.lam[l]);
            else if (n == 128)
                mixed_onchip<float, 128, 16, DST>(a, p, lt.obs[l], S, lt.lam[l]);
            else if (n == 256 && DST)
                mixed_global_dst<float, 256>(a, p, lt.obs[l], S, lt.lam[l]);
            else if (n == 256)
                mixed_global<float>(a, p, 256, lt.obs[l]);
        } else {
            if (n == 64)
                mixed_onchip<double, 64, 4, false>(a, p, lt.obs[l], nullptr, nullptr);
            else if (n == 128 && DST)
                mixed_global_dst<double, 128>(a, p, lt.obs[l], S, lt.lam[l]);
            else if (n == 256 && DST)
                mixed_global_dst<double, 256>(a, p, lt.obs[l], S, lt.lam[l]);
            else if (n == 128 || n == 256)
                mixed_global<double>(a, p, n, lt.obs[l]);
        }
        if (n != 64 && n != 128 && n != 256) {   // no such grid: the particle is rejected
            if (threadIdx.x < a.n_obs && a.G) a.G[p * a.n_obs + threadIdx.x] = NAN;
            if (threadIdx.x == 0) {
                if (a.phi) a.phi[p] = INFINITY;
                if (a.iters) a.iters[p] = -1;
            }
        }
        // every lane closes the iteration here, so that no thread-0-only region of this iteration
        // can be merged with the next iteration's fetch by the compiler
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const unsigned long long done = atomicAdd(&counters[1], 1ull);
        if (done == (unsigned long long)gridDim.x - 1ull) {   // every workgroup has stopped fetching
            counters[0] = 0;
            counters[1] = 0;
        }
    }
}

// ------------------------------------------------------------------ persistent move stage
// One launch per stage of n_moves pCN-GM moves (Alg. 2) for particles on one grid solved on chip:
// each workgroup takes the next particle from a counter and runs its whole stage, move after move
// (proposal, synthesis of exp(u/2), forward solve and potential, decision), then the next particle.
// The particles of a stage do not interact, so this is the same computation as one launch per
// step (the same bodies in the same order for each particle: the same bits), without a kernel
// boundary, and its drain, between the steps.  Each phase is a function of its own, register-
// allocated apart, and they share the module-level LDS in turn.
__shared__ int g_stage_acc;

template <int NN, int R>
__device__ __noinline__ void stage_propose(const StageArgs& st, const MoveParams& q, int64_t p) {
    propose_body<NN * NN / R>(p, st.K, st.active, st.slot, q, st.tab, st.xi, st.v, st.logr, st.flags);
}

template <int NN, int R>
__device__ __noinline__ void stage_synth(const StageArgs& st, int64_t p, double* e, int64_t e_stride) {
    static_assert((NN * NN / R) % 64 == 0, "whole waves");
    synth2d_body<true, NN * NN / R / 64>(st.v + p * st.K, st.kl, st.sqrt_lam, st.basis, NN, e + p * e_stride,
                                         reinterpret_cast<double*>(g_mixed_smem));
}

template <int NN, int R>
__device__ __noinline__ void stage_accept(const StageArgs& st, const MoveParams& q, int64_t p, const double* phinew) {
    accept_body<NN * NN / R>(p, st.K, q, st.v, st.logr, phinew, st.xi, st.phi, st.n_acc, g_stage_acc);
}

template <int NN, int R>
__global__ __launch_bounds__(NN * NN / R) void stage_onchip_kernel(SolveArgs a, StageArgs st, MoveParams q,
                                                                   const _Float16* __restrict__ S,
                                                                   const float* __restrict__ lam,
                                                                   unsigned long long* counters) {
    __shared__ unsigned long long item_s;
    for (;;) {
        if (threadIdx.x == 0) item_s = atomicAdd(&counters[0], 1ull);
        __syncthreads();
        // wave-uniform item: the loop exit below must be a uniform branch (see solve_mixed_kernel)
        const int64_t p = __builtin_amdgcn_readfirstlane((int)(item_s < (unsigned long long)st.N ? item_s : st.N));
        __syncthreads();
        if (p >= st.N) break;
        for (int m = 0; m < st.n_moves; ++m) {
            MoveParams qm = q;
            qm.m = m;
            stage_propose<NN, R>(st, qm, p);
            __syncthreads();
            stage_synth<NN, R>(st, p, const_cast<double*>(a.e), a.e_stride);
            __syncthreads();
            mixed_onchip<float, NN, R, true, false>(a, p, a.obs, S, lam);   // phi of the proposal into a.phi
            __syncthreads();
            stage_accept<NN, R>(st, qm, p, a.phi);
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        const unsigned long long done = atomicAdd(&counters[1], 1ull);
        if (done == (unsigned long long)gridDim.x - 1ull) {   // every workgroup has stopped fetching
            counters[0] = 0;
            counters[1] = 0;
        }
    }
}

bool stage_fused_supported(int n, int rows) {
    return (n == 128 && (rows == 32 || rows == 16)) || (n == 64 && rows == 8);
}

hipError_t launch_stage_onchip(int n, int rows, const SolveArgs& a, const StageArgs& st, const MoveParams& q,
                               const void* S, const float* lam, unsigned long long* counters, int grid,
                               hipStream_t s) {
    if (st.N <= 0) return hipSuccess;
    const unsigned g = (unsigned)(st.N < grid ? st.N : grid);
    const _Float16* Sh = reinterpret_cast<const _Float16*>(S);
    const int key = n * 64 + rows;
    switch (key) {
        case 128 * 64 + 32:
            stage_onchip_kernel<128, 32><<<dim3(g), dim3(512), 0, s>>>(a, st, q, Sh, lam, counters);
            break;
        case 128 * 64 + 16:
            stage_onchip_kernel<128, 16><<<dim3(g), dim3(1024), 0, s>>>(a, st, q, Sh, lam, counters);
            break;
        case 64 * 64 + 8:
            stage_onchip_kernel<64, 8><<<dim3(g), dim3(512), 0, s>>>(a, st, q, Sh, lam, counters);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_solve_mixed(int prec, bool dst, int64_t N, const SolveArgs& a, const LevelTable& lt,
                              const int32_t* level, const int32_t* list, unsigned long long* counters, int grid,
                              hipStream_t s) {
    if (N <= 0) return hipSuccess;
    const unsigned g = (unsigned)(N < grid ? N : grid);
    if (prec == SMC_FP32_REFINE) {
        if (dst)
            solve_mixed_kernel<SMC_FP32_REFINE, true><<<dim3(g), dim3(1024), 0, s>>>(a, lt, level, list, N, counters);
        else
            solve_mixed_kernel<SMC_FP32_REFINE, false><<<dim3(g), dim3(1024), 0, s>>>(a, lt, level, list, N, counters);
    } else {
        SolveArgs b = a;
        b.tol_inner = 0.1 * a.tol64;
        if (dst)
            solve_mixed_kernel<SMC_FP64, true><<<dim3(g), dim3(1024), 0, s>>>(b, lt, level, list, N, counters);
        else
            solve_mixed_kernel<SMC_FP64, false><<<dim3(g), dim3(1024), 0, s>>>(b, lt, level, list, N, counters);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ one launch per grid of a level map
// plan_kernel leaves grid l's particles in list[start .. start + count) (start and count at
// COUNTER_SEG + 2 l); each grid is solved by a launch of N workgroups in the shape of its
// single-grid launch, workgroup k taking list entry start + k and the ones beyond the count
// leaving at once.  The body is the single-grid kernel's (the same bits), and without a fetch loop
// around it the compiler allocates its registers as in that kernel (a persistent loop spilled more
// and, at 64^2, held more registers than two workgroups per compute unit leave).
__device__ __forceinline__ int64_t list_item(const unsigned long long* counters, int lvl,
                                             const int32_t* __restrict__ list) {
    const int64_t start = __builtin_amdgcn_readfirstlane((int)counters[COUNTER_SEG + 2 * lvl]);
    const int64_t count = __builtin_amdgcn_readfirstlane((int)counters[COUNTER_SEG + 2 * lvl + 1]);
    if ((int64_t)blockIdx.x >= count) return -1;
    return __builtin_amdgcn_readfirstlane(list[start + blockIdx.x]);
}

template <typename T, int NN, int R>
__global__ __launch_bounds__(NN * NN / R) void solve_list_onchip(SolveArgs a, const int32_t* __restrict__ list,
                                                                 const unsigned long long* counters, int lvl,
                                                                 const int32_t* __restrict__ obs,
                                                                 const _Float16* __restrict__ Stab,
                                                                 const float* __restrict__ lamtab) {
    __shared__ __align__(16) unsigned char smem[onchip_smem<T, NN, R, true>()];
    __shared__ SolveShared sh;
    const int64_t p = list_item(counters, lvl, list);
    if (p < 0) return;
    cg_onchip_body<T, NN, R, true, false>(a, p, obs, smem, sh, Stab, lamtab);
}

template <typename T, int NN>
__global__ __launch_bounds__(1024) void solve_list_global(SolveArgs a, const int32_t* __restrict__ list,
                                                          const unsigned long long* counters, int lvl,
                                                          const int32_t* __restrict__ obs,
                                                          const _Float16* __restrict__ Stab,
                                                          const float* __restrict__ lamtab) {
    __shared__ SolveShared sh;
    const int64_t p = list_item(counters, lvl, list);
    if (p < 0) return;
    cg_global_body<T, false, true, NN>(a, p, NN, obs, sh, reinterpret_cast<_Float16*>(g_mixed_smem), Stab, lamtab);
}

// The particles with no grid (parked or out of range): the outputs of a rejected proposal.
__global__ __launch_bounds__(256) void reject_list_kernel(SolveArgs a, const int32_t* __restrict__ list,
                                                          const unsigned long long* counters) {
    const int64_t start = (int64_t)counters[COUNTER_SEG + 2 * MAX_LEVELS];
    const int64_t count = (int64_t)counters[COUNTER_SEG + 2 * MAX_LEVELS + 1];
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= count) return;
    const int64_t p = list[start + k];
    if (a.G)
        for (int o = 0; o < a.n_obs; ++o) a.G[p * a.n_obs + o] = NAN;
    if (a.phi) a.phi[p] = INFINITY;
    if (a.iters) a.iters[p] = -1;
}

hipError_t launch_solve_levels(int prec, int64_t N, const SolveArgs& a, const LevelTable& lt, const int* rows,
                               const int32_t* list, unsigned long long* counters, int n_cu, hipStream_t s) {
    (void)n_cu;
    if (N <= 0) return hipSuccess;
    int order[MAX_LEVELS];   // finest grid first, as the list is
    for (int l = 0; l < lt.n_levels; ++l) order[l] = l;
    for (int i = 0; i < lt.n_levels; ++i)
        for (int j = i + 1; j < lt.n_levels; ++j)
            if (lt.n[order[j]] > lt.n[order[i]]) std::swap(order[i], order[j]);
    SolveArgs b = a;
    if (prec == SMC_FP64) b.tol_inner = 0.1 * a.tol64;   // FP64 CG to 0.1 tol64 in one sweep, as single-grid
    const dim3 g1((unsigned)N), g4((unsigned)N);   // at most N particles per grid
    for (int k = 0; k < lt.n_levels; ++k) {
        const int l = order[k], n = lt.n[l];
        const _Float16* S = reinterpret_cast<const _Float16*>(lt.S[l]);
        const float* lam = lt.lam[l];
        const int32_t* obs = lt.obs[l];
        if (prec == SMC_FP32_REFINE) {
            if (n == 256)
                solve_list_global<float, 256><<<g1, dim3(1024), 0, s>>>(b, list, counters, l, obs, S, lam);
            else if (n == 128 && rows[l] == 16)
                solve_list_onchip<float, 128, 16><<<g1, dim3(1024), 0, s>>>(b, list, counters, l, obs, S, lam);
            else if (n == 128)
                solve_list_onchip<float, 128, 32><<<g1, dim3(512), 0, s>>>(b, list, counters, l, obs, S, lam);
            else if (n == 64 && rows[l] == 4)
                solve_list_onchip<float, 64, 4><<<g4, dim3(1024), 0, s>>>(b, list, counters, l, obs, S, lam);
            else if (n == 64 && rows[l] == 16)
                solve_list_onchip<float, 64, 16><<<g4, dim3(256), 0, s>>>(b, list, counters, l, obs, S, lam);
            else if (n == 64)
                solve_list_onchip<float, 64, 8><<<g4, dim3(512), 0, s>>>(b, list, counters, l, obs, S, lam);
            else
                return hipErrorInvalidValue;
        } else {
            if (n == 256)
                solve_list_global<double, 256><<<g1, dim3(1024), 0, s>>>(b, list, counters, l, obs, S, lam);
            else if (n == 128)
                solve_list_global<double, 128><<<g1, dim3(1024), 0, s>>>(b, list, counters, l, obs, S, lam);
            else if (n == 64)
                solve_list_onchip<double, 64, 8><<<g4, dim3(512), 0, s>>>(b, list, counters, l, obs, S, lam);
            else
                return hipErrorInvalidValue;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    reject_list_kernel<<<dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s>>>(b, list, counters);
    return hipGetLastError();
}

template <typename T, int NN, int R, bool DST>
static hipError_t run_onchip(int64_t N, const SolveArgs& a, const void* S, const float* lam, hipStream_t s) {
    const _Float16* Sb = reinterpret_cast<const _Float16*>(S);
    if (a.lam)
        cg_onchip<T, NN, R, DST, true><<<dim3((unsigned)N), dim3(NN * NN / R), 0, s>>>(a, Sb, lam);
    else
        cg_onchip<T, NN, R, DST, false><<<dim3((unsigned)N), dim3(NN * NN / R), 0, s>>>(a, Sb, lam);
    return hipGetLastError();
}

// Forward and adjoint solves as two launches of the forward solver's shape (a body with both passes
// needs more registers than the 32-row shape has): the forward problem into x64, then the adjoint
// problem alone from it; the second launch adds its iterations to the first's.
template <typename T, int NN, int R>
static hipError_t run_onchip_two_pass(int64_t N, const SolveArgs& a, const void* S, const float* lam, hipStream_t s) {
    const _Float16* Sb = reinterpret_cast<const _Float16*>(S);
    if (!a.fwd_given) {
        SolveArgs f = a;
        f.lam = nullptr;
        cg_onchip<T, NN, R, true, false><<<dim3((unsigned)N), dim3(NN * NN / R), 0, s>>>(f, Sb, lam);
    }
    cg_onchip<T, NN, R, true, true, true><<<dim3((unsigned)N), dim3(NN * NN / R), 0, s>>>(a, Sb, lam);
    return hipGetLastError();
}

template <typename T>
static hipError_t run_global(int64_t N, const SolveArgs& a, int n, hipStream_t s) {
    if (a.lam)
        cg_global<T, true><<<dim3((unsigned)N), dim3(1024), 0, s>>>(a, n);
    else
        cg_global<T, false><<<dim3((unsigned)N), dim3(1024), 0, s>>>(a, n);
    return hipGetLastError();
}

bool dst_supported(int n) { return n == 32 || n == 64 || n == 128 || n == 256; }

// Tile shapes of the fast-Poisson solver: rows of the grid per thread (the workgroup has n * n / rows
// threads); the first is the default.  The 256 grid runs the global-memory solver (no choice).
int tile_candidates(int n, int* rows) {
    switch (n) {
        case 32: rows[0] = 4; rows[1] = 8; return 2;
        case 64: rows[0] = 8; rows[1] = 4; rows[2] = 16; return 3;
        case 128: rows[0] = 32; rows[1] = 16; return 2;
        case 256: rows[0] = 0; return 1;
        default: return 0;
    }
}

hipError_t launch_solve2d_dst(int n, int rows, int64_t N, const SolveArgs& a, const void* S, const float* lam,
                              hipStream_t s) {
    if (N <= 0) return hipSuccess;
    // forward and adjoint at 128^2 in the 32-row shape: two launches (one body with both passes
    // spills at 32 rows; 16 rows runs both passes in one launch)
    if (a.lam && n == 128 && (rows == 0 || rows == 32)) return run_onchip_two_pass<float, 128, 32>(N, a, S, lam, s);
    const int key = n * 64 + rows;
    switch (key) {
        case 32 * 64 + 0:
        case 32 * 64 + 4: return run_onchip<float, 32, 4, true>(N, a, S, lam, s);
        case 32 * 64 + 8: return run_onchip<float, 32, 8, true>(N, a, S, lam, s);
        case 64 * 64 + 0:
        case 64 * 64 + 8: return run_onchip<float, 64, 8, true>(N, a, S, lam, s);
        case 64 * 64 + 4: return run_onchip<float, 64, 4, true>(N, a, S, lam, s);
        case 64 * 64 + 16: return run_onchip<float, 64, 16, true>(N, a, S, lam, s);
        case 128 * 64 + 16: return run_onchip<float, 128, 16, true>(N, a, S, lam, s);
        case 128 * 64 + 0:
        case 128 * 64 + 32: return run_onchip<float, 128, 32, true>(N, a, S, lam, s);
        case 256 * 64 + 0: return run_global_dst<float, 256>(N, a, S, lam, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_solve2d(int n, int prec, int64_t N, const SolveArgs& a, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    if (prec == SMC_FP32_REFINE) {
        switch (n) {
            case 16: return run_onchip<float, 16, 4, false>(N, a, nullptr, nullptr, s);
            case 32: return run_onchip<float, 32, 4, false>(N, a, nullptr, nullptr, s);
            case 64: return run_onchip<float, 64, 8, false>(N, a, nullptr, nullptr, s);
            case 128: return run_onchip<float, 128, 16, false>(N, a, nullptr, nullptr, s);
            default: return run_global<float>(N, a, n, s);
        }
    }
    SolveArgs b = a;
    b.tol_inner = 0.1 * a.tol64;
    switch (n) {
        case 16: return run_onchip<double, 16, 4, false>(N, b, nullptr, nullptr, s);
        case 32: return run_onchip<double, 32, 4, false>(N, b, nullptr, nullptr, s);
        case 64: return run_onchip<double, 64, 8, false>(N, b, nullptr, nullptr, s);
        default: return run_global<double>(N, b, n, s);
    }
}

// FP64 conjugate gradients on chip with the fast-Poisson preconditioner (FP16 transforms, a
// perturbation of the preconditioner only), to 0.1 tol64 in one sweep: 32^2 and 64^2.
hipError_t launch_solve2d_dst64_onchip(int n, int64_t N, const SolveArgs& a, const void* S, const float* lam,
                                       hipStream_t s) {
    if (N <= 0) return hipSuccess;
    SolveArgs b = a;
    b.tol_inner = 0.1 * a.tol64;
    if (n == 32) return run_onchip<double, 32, 4, true>(N, b, S, lam, s);
    if (n == 64) return run_onchip<double, 64, 8, true>(N, b, S, lam, s);
    return hipErrorInvalidValue;
}

// FP64 conjugate gradients with the fast-Poisson preconditioner (FP16 transforms, a perturbation of
// the preconditioner only) on the 128 and 256 grids, vectors in global memory, to 0.1 tol64 in one
// sweep.
hipError_t launch_solve2d_dst64(int n, int64_t N, const SolveArgs& a, const void* S, const float* lam,
                                hipStream_t s) {
    if (N <= 0) return hipSuccess;
    SolveArgs b = a;
    b.tol_inner = 0.1 * a.tol64;
    if (n == 128) return run_global_dst<double, 128>(N, b, S, lam, s);
    if (n == 256) return run_global_dst<double, 256>(N, b, S, lam, s);
    return hipErrorInvalidValue;
}

hipError_t launch_solve1d(int n, int64_t N, const SolveArgs& a, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    solve1d_kernel<<<dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s>>>(a, n, N);
    return hipGetLastError();
}

}  // namespace smc
