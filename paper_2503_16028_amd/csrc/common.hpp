// Internal definitions shared by the kernels and the C ABI of libsmc.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/smc.h"

namespace smc {

constexpr int MAX_LEVELS = 3;
constexpr int MAX_OBS = 64;
constexpr int MAX_M = 16;
constexpr int MAX_KR = 64;
constexpr int GM_PAR = 2 * MAX_M + 4 * MAX_M * MAX_KR;   // doubles in one mixture-fit parameter block
// Proposal table of one group's mixture: [MAX_M][MAX_KR] 1/s_ji, then [MAX_M] half the sum of
// log s_ji over the active modes, then [MAX_M] the running sums of the weights.
constexpr int MIXTAB = MAX_M * (MAX_KR + 2);
constexpr int MAX_TERMS = 16;        // terms of an L^2 mixture likelihood
constexpr int KIND_DARCY = 0;        // forward map: Darcy solve, observations at nodes
constexpr int KIND_L2MIX = 1;        // no forward map: mixture likelihood in L^2 on the coefficients
constexpr int KLP = 32;          // 2D modes per axis, padded, in the synthesis tiles
constexpr uint32_t UNIFORM_BLOCK = 0x80000000u;

struct Level {
    int n = 0;                   // intervals per axis
    double* basis = nullptr;     // 2D: [(n+1)][KLP] c_k cos(k pi i / n); 1D: [(n+1)][kl] sqrt2 sin(k pi i / n)
    int32_t* obs_node = nullptr; // [n_obs] flat nodal index (2D j*(n+1)+i, 1D i)
    void* dst_S = nullptr;       // [n][n] FP16 sine transform (fast-Poisson preconditioner)
    float* dst_lam = nullptr;    // [n] its 1D eigenvalues sin^2(pi (k+1) / 2n)
    int rows = 0;                // tile of the fast-Poisson solver: grid rows per thread (0 = default)
};

struct Problem {
    int kind = KIND_DARCY;
    int dim = 0, n_levels = 0, kl = 0, K = 0, kr = 0, n_obs = 0;
    int n_terms = 0;             // KIND_L2MIX: likelihood terms
    double* mix_c = nullptr;     // KIND_L2MIX: [n_terms][K] coefficients of the centres f_i
    Level lv[MAX_LEVELS];
    int n_big = 0;               // largest grid
    double sigma = 1, f = 1, tol64 = 1e-10, tol_inner = 1e-5;
    int max_iter = 0, max_sweeps = 0, precond = 0;
    int64_t n_max = 0;
    double* sqrt_lam = nullptr;  // [K]
    int32_t* active = nullptr;   // [kr] active mode ids
    int32_t* slot = nullptr;     // [K] position in the active list or -1
    int32_t active_h[MAX_KR];
    double* y = nullptr;         // [n_obs]
    // workspace, all for n_max particles
    double* ws_v = nullptr;      // [n_max][K]    proposals
    double* ws_logr = nullptr;   // [n_max]       log R of the proposal
    double* ws_phinew = nullptr; // [n_max]       potential of the proposal
    double* ws_e = nullptr;      // [n_max][(n_big+1)^dim]  exp(u/2) at the nodes
    double* ws_x64 = nullptr;    // [n_max][n_big^dim]      FP64 solution
    double* ws_lam = nullptr;    // [n_max][n_big^2]        FP64 adjoint solution (2D)
    double* ws_gnew = nullptr;   // [n_max][K]              gradient at the proposal (2D)
    double* ws_sd = nullptr;     // [n_max][n_big^2]        D^{-1/2} of the Jacobi scaling (FP32 in the first
                                 //                         half of a row for FP32 on-chip solves)
    void* ws_vec = nullptr;      // [n_max][7][n_big^2] doubles: vectors of the global-memory solver
    double* ws_G = nullptr;      // [n_max][n_obs]
    int32_t* ws_iters = nullptr; // [n_max]
    int32_t* ws_list = nullptr;  // [n_max] work list of a level map (particles grouped by grid)
    unsigned long long* ws_counters = nullptr;   // [2] work and exit counters of the persistent solve
    double* ws_fit_d2 = nullptr;      // [n_max]   squared distance to the nearest seeded centre
    double* ws_fit_par = nullptr;     // [2][GM_PAR]  EM parameter blocks (ping-pong)
    double* ws_fit_part = nullptr;    // [workgroups of 128 particles][MAX_M][1 + 2 MAX_KR]  partial sums
    int32_t* ws_fit_centers = nullptr;  // [MAX_M] seeded rows
    double* ws_mixtab = nullptr;      // [MAX_LEVELS][MIXTAB]  mixture tables of the proposal, per group
    int n_cu = 0;                // compute units of the device
    int32_t* flags = nullptr;    // device status word
    unsigned long long* stats = nullptr;  // [4] iterations, sweeps, solves, preconditioner applications
    bool profiling = false;
    void* events = nullptr;      // host-side event list (api.hip)
    int64_t e_stride = 0, x_stride = 0, vec_stride = 0;
};

// ------------------------------------------------------------------ Philox4x32-10
// Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11):
// ten rounds of two 32x32->64 products; the key is bumped by two Weyl constants
// between rounds.
__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    }
    return c;
}

// 53-bit uniform in [0, 1) from two words.
__device__ __forceinline__ double res53(uint32_t a, uint32_t b) {
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * 0x1p-53;
}

// Two standard normals by Box-Muller from the four words of one block.
__device__ __forceinline__ void box_muller(uint4 w, double& z0, double& z1) {
    const double u1 = res53(w.x, w.y), u2 = res53(w.z, w.w);
    const double rad = sqrt(-2.0 * log(1.0 - u1));
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    z0 = rad * c;
    z1 = rad * s;
}

__device__ __forceinline__ uint4 draw(uint64_t seed, uint64_t ctr, uint32_t block, uint32_t particle) {
    return philox(make_uint4(block, particle, (uint32_t)ctr, (uint32_t)(ctr >> 32)), (uint32_t)seed,
                  (uint32_t)(seed >> 32));
}

// ------------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;   // identical in every lane (each butterfly step adds the same two operands)
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// A value every lane of the wave holds (read back from LDS, say) made visibly uniform to the
// compiler: branches and loop exits on it are then compiled as wave-uniform, never as divergent
// control flow around the barriers they enclose.
__device__ __forceinline__ double uniform(double v) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the block in a fixed order; every thread gets the same bits (and the compiler knows).
// `red` holds at least NW doubles of LDS; contains a barrier.
template <int NW>
__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += red[w];
    return uniform(s);
}

// ------------------------------------------------------------------ launchers (defined in k_*.hip)
struct SolveArgs {
    const double* e;     // exp(u/2) nodal, row stride e_stride
    double* x64;         // FP64 solution, row stride x_stride
    double* sd;          // D^{-1/2}, row stride x_stride (doubles; an FP32 row starts at the same place)
    void* vec;           // global-solver vectors, row stride vec_stride (doubles)
    int64_t e_stride, x_stride, sd_stride, vec_stride;
    double* lam;         // adjoint solution [N][lam_stride] (interior layout as x64), or null: no adjoint
    int64_t lam_stride;
    int fwd_given;       // x64 already holds the forward solution: only the adjoint problem is solved
    int64_t row0;        // first particle row
    const int32_t* obs;  // [n_obs] nodal flat index
    int n_obs;
    const double* y;
    double inv2s2;       // 1 / (2 sigma^2)
    double f, tol64, tol_inner;
    int max_iter, max_sweeps;
    double* G;           // [N][n_obs] or null
    double* phi;         // [N] or null
    int32_t* iters;      // [N] or null
    int32_t* flags;
    unsigned long long* stats;   // [4] iterations, sweeps, solves, preconditioner applications; or null
    double* du;          // dPhi/du [N][du_stride] at every node, [j][i] on (n+1)^2, written after the
    int64_t du_stride;   // adjoint solve by the on-chip solvers; null: not formed there
};

// Parameters of the moves of one call.  Either scalars for every particle, or per-group device
// arrays, the group of particle n being group[n]; the counter of move m is ctr (or *ctr_dev) + m.
// Mixture of group g: logw[g][M], mean[g][M][kr], scale[g][M][kr].
struct MoveParams {
    double beta = 0, tau = 0;
    uint64_t seed = 0, ctr = 0;
    const int32_t* group = nullptr;
    const double* beta_g = nullptr;
    const double* tau_g = nullptr;
    const uint64_t* ctr_dev = nullptr;
    int n_groups = 1;
    int M = 1, kr = 0;
    const double* logw = nullptr;
    const double* mean = nullptr;
    const double* scale = nullptr;
    int m = 0;
};

// Group of particle n (-1 if out of range) and its parameters.
__device__ __forceinline__ int mp_group(const MoveParams& q, int64_t n) {
    if (!q.group) return 0;
    const int g = q.group[n];
    return (g >= 0 && g < q.n_groups) ? g : -1;
}
__device__ __forceinline__ double mp_beta(const MoveParams& q, int g) { return q.beta_g ? q.beta_g[g] : q.beta; }
__device__ __forceinline__ double mp_tau(const MoveParams& q, int g) { return q.tau_g ? q.tau_g[g] : q.tau; }
__device__ __forceinline__ uint64_t mp_ctr(const MoveParams& q) {
    return (q.ctr_dev ? *q.ctr_dev : q.ctr) + (uint64_t)q.m;
}
__device__ __forceinline__ bool mp_valid(double beta, double tau) {
    return beta > 0.0 && beta <= 1.0 && tau >= 0.0 && tau <= 1.0;
}

// Per-grid tables handed to the kernels that serve particles of several grids in one launch.
struct LevelTable {
    int n_levels;
    int n[MAX_LEVELS];
    const double* basis[MAX_LEVELS];
    const int32_t* obs[MAX_LEVELS];
    const void* S[MAX_LEVELS];       // FP16 sine transform, or null
    const float* lam[MAX_LEVELS];
};

hipError_t launch_synth2d_levels(const double* xi, int K, int kl, const double* sqrt_lam, const LevelTable& lt,
                                 const int32_t* level, double* out, int64_t out_stride, int64_t N, bool exp_half,
                                 hipStream_t s);
bool mixed_supported(int n);
// The rest of a persistent move-stage launch (the solver's arguments are a SolveArgs): the
// particles' state, the proposal workspace and the tables the proposal and synthesis read.
struct StageArgs {
    int64_t N;
    int K, kl, n_moves;
    const int32_t* active;
    const int32_t* slot;
    const double* tab;        // mixture table of the call (mixtab_kernel)
    const double* sqrt_lam;
    const double* basis;      // cosine basis of the grid
    double* xi;               // [N][K] state, in/out
    double* phi;              // [N] potentials, in/out
    int32_t* n_acc;           // [N] accept counts (zeroed before the launch)
    double* v;                // [N][K] proposal workspace
    double* logr;             // [N] log ratio workspace
    int32_t* flags;
};
// One launch for a whole stage of n_moves pCN-GM moves on one grid solved on chip with the
// fast-Poisson preconditioner (FP32 with FP64 refinement): false if no such launch exists for
// this grid and tile (then the moves run one launch per step).
bool stage_fused_supported(int n, int rows);
hipError_t launch_stage_onchip(int n, int rows, const SolveArgs& a, const StageArgs& st, const MoveParams& q,
                               const void* S, const float* lam, unsigned long long* counters, int grid,
                               hipStream_t s);
// The counters workspace: [0, 2) the persistent launches' fetch and done counters; then per grid
// l of a level map the segment of the work list that holds its particles, start and count, at
// COUNTER_SEG + 2 l (grid MAX_LEVELS: the particles with no grid, parked or out of range, which
// come last).
constexpr int COUNTER_SEG = 2;
constexpr int N_COUNTERS = COUNTER_SEG + 2 * (MAX_LEVELS + 1);
hipError_t launch_plan(int64_t N, const int32_t* level, const LevelTable& lt, int32_t* list,
                       unsigned long long* counters, int32_t* flags, hipStream_t s);
// The solves of a level map as one persistent launch per grid, each in the workgroup shape of that
// grid's single-grid launch (rows[l]: its tile, 0 = default), after launch_plan: FP32 with FP64
// refinement or FP64, fast-Poisson preconditioners on every grid.
hipError_t launch_solve_levels(int prec, int64_t N, const SolveArgs& a, const LevelTable& lt, const int* rows,
                               const int32_t* list, unsigned long long* counters, int n_cu, hipStream_t s);
hipError_t launch_solve_mixed(int prec, bool dst, int64_t N, const SolveArgs& a, const LevelTable& lt,
                              const int32_t* level, const int32_t* list, unsigned long long* counters, int grid,
                              hipStream_t s);
hipError_t launch_synth2d(const double* xi, int K, int kl, const double* sqrt_lam, const double* basis, int n,
                          double* out, int64_t out_stride, int64_t N, bool exp_half, hipStream_t s);
hipError_t launch_synth1d(const double* xi, int kl, const double* sqrt_lam, const double* basis, int n, double* out,
                          int64_t out_stride, int64_t N, bool exp_half, hipStream_t s);
hipError_t launch_gradsynth2d(const double* e, int64_t e_stride, const double* w, int64_t w_stride,
                              const double* lam, int64_t lam_stride, const int32_t* iters, const double* sqrt_lam,
                              const double* basis, int n, int kl, int K, double* grad, int64_t N, const double* du,
                              int64_t du_stride, hipStream_t s);
hipError_t launch_pcnl_propose(int64_t N, int K, double beta, double tau, uint64_t seed, uint64_t ctr,
                               const double* xi, const double* grad, double* v, hipStream_t s);
hipError_t launch_pcnl_accept(int64_t N, int K, double beta, double tau, uint64_t seed, uint64_t ctr, const double* v,
                              const double* gnew, const double* phinew, const int32_t* iters_new, double* xi,
                              double* grad, double* phi, int32_t* n_acc, hipStream_t s);
hipError_t launch_solve2d(int n, int prec, int64_t N, const SolveArgs& a, hipStream_t s);
hipError_t launch_solve1d(int n, int64_t N, const SolveArgs& a, hipStream_t s);
bool dst_supported(int n);
int tile_candidates(int n, int* rows);
hipError_t launch_solve2d_dst(int n, int rows, int64_t N, const SolveArgs& a, const void* S, const float* lam,
                              hipStream_t s);
hipError_t launch_solve2d_dst64(int n, int64_t N, const SolveArgs& a, const void* S, const float* lam,
                                hipStream_t s);
hipError_t launch_solve2d_dst64_onchip(int n, int64_t N, const SolveArgs& a, const void* S, const float* lam,
                                       hipStream_t s);
hipError_t launch_dst_apply(int n, int64_t N, const float* r, float* z, const void* S, const float* lam,
                            hipStream_t s);

hipError_t launch_prior(int64_t N, int K, uint64_t seed, uint64_t ctr, double* xi, hipStream_t s);
hipError_t launch_potential(int64_t N, int n_obs, const double* G, const double* y, double inv2s2, double* phi,
                            hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_mixtab(const MoveParams& q, double* tab, hipStream_t s);
hipError_t launch_propose(int64_t N, int K, const int32_t* active, const int32_t* slot, const MoveParams& q,
                          const double* tab, const double* xi, double* v, double* logr, int32_t* flags,
                          hipStream_t s);
hipError_t launch_accept(int64_t N, int K, const MoveParams& q, const double* v, const double* logr,
                         const double* phinew, double* xi, double* phi, int32_t* n_acc, hipStream_t s);
hipError_t prepare_kernels();
hipError_t launch_l2mix_phi(int64_t N, int K, const double* sqrt_lam, const double* c, int T, double inv2s2,
                            const double* xi, double* phi, int32_t* iters, hipStream_t s);
hipError_t launch_gm_draw(int64_t N, int K, const int32_t* slot, uint64_t seed, uint64_t ctr, int M, int kr,
                          const double* logw, const double* mean, const double* scale, double* v, hipStream_t s);

struct FitWorkspace {
    double* d2;
    double* par;
    double* part;
};
int64_t em_blocks(int64_t N);
// Mixture fit on the library's static scratch array (no allocation), for up to STATIC_FIT_N
// particles; launch_gm_fit_static returns hipErrorInvalidValue beyond that.
constexpr int64_t STATIC_FIT_N = 32768;
size_t static_fit_bytes();
hipError_t launch_gm_fit_static(int64_t N, int K, int kr, const int32_t* active, const double* xi, int M, int iters,
                                double var_floor, uint64_t seed, uint64_t ctr, int32_t* centers, double* logw,
                                double* mean, double* scale, hipStream_t s);
hipError_t prepare_gmfit_kernels();
hipError_t launch_gm_fit(int64_t N, int K, int kr, const int32_t* active, const double* xi, int M, int iters,
                         double var_floor, uint64_t seed, uint64_t ctr, const FitWorkspace& w, int32_t* centers,
                         double* logw, double* mean, double* scale, hipStream_t s);
hipError_t launch_gather(int64_t N, int K, const int32_t* idx, const double* xi_in, const double* phi_in,
                         double* xi_out, double* phi_out, hipStream_t s);
hipError_t launch_temper(int64_t N, const double* phi, const double* tau_in, double ess_frac, double* h,
                         double* tau_new, double* W, double* log_z, int32_t* flags, hipStream_t s);
hipError_t launch_resample(int64_t N, const double* W, uint64_t u53, int32_t* idx, int32_t* flags, hipStream_t s);

}  // namespace smc
