// C ABI of libsmc: argument validation, device tables, workspace and the launch sequence of
// each call.  Every argument is checked before anything is launched.
#include <stdarg.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "common.hpp"
#include "stage_graph.hpp"

using namespace smc;

struct EventPool {
    std::vector<hipEvent_t> ev;   // pairs: ev[2k] before, ev[2k+1] after launch k
    std::vector<int> rounds;      // solve rounds inside launch k (a stage launch holds one per move)
    size_t used = 0;              // events recorded since the last read
};

struct smc_problem_s {
    Problem P;
    int device = 0;
    EventPool pool;
    bool capturing = false;       // launches are being captured into a graph: no profiling events
    bool fuse_stage = false;      // a move stage on one on-chip grid runs as one persistent launch
};

struct smc_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail(SMC_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

static bool pow2_in(int n, int lo, int hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }

template <typename T>
static hipError_t upload(T** dst, const T* src, size_t n) {
    hipError_t e = hipMalloc((void**)dst, n * sizeof(T));
    if (e != hipSuccess) return e;
    return hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice);
}

static void free_problem(Problem& P) {
    auto f = [](void* p) { if (p) (void)hipFree(p); };
    for (int l = 0; l < MAX_LEVELS; ++l) { f(P.lv[l].basis); f(P.lv[l].obs_node); f(P.lv[l].dst_S); f(P.lv[l].dst_lam); }
    f(P.sqrt_lam); f(P.active); f(P.slot); f(P.y);
    f(P.ws_v); f(P.ws_logr); f(P.ws_phinew); f(P.ws_e); f(P.ws_x64); f(P.ws_lam); f(P.ws_gnew); f(P.ws_sd);
    f(P.ws_vec);
    f(P.ws_G); f(P.ws_iters); f(P.ws_list); f(P.ws_counters); f(P.flags); f(P.stats);
    f(P.ws_fit_d2); f(P.ws_fit_par); f(P.ws_fit_part); f(P.ws_fit_centers); f(P.ws_mixtab);
    f(P.mix_c);
}

extern "C" const char* smc_last_error(void) { return g_err.c_str(); }

// Philox4x32-10 on the host (the kernels' generator, for the few draws the host hands to a call).
extern "C" uint64_t smc_philox_u53(uint64_t seed, uint64_t ctr, uint32_t block, uint32_t word) {
    uint32_t c0 = block, c1 = word, c2 = (uint32_t)ctr, c3 = (uint32_t)(ctr >> 32);
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    return ((uint64_t)(c0 >> 5) << 26) | (uint64_t)(c1 >> 6);
}

extern "C" int smc_problem_create(const smc_problem_desc* d, smc_problem* out) {
    if (!d || !out) return fail(SMC_E_INVAL, "desc and out must not be NULL");
    if (d->dim != 1 && d->dim != 2) return fail(SMC_E_INVAL, "dim must be 1 or 2 (got %d)", d->dim);
    if (d->n_levels < 1 || d->n_levels > MAX_LEVELS) return fail(SMC_E_INVAL, "n_levels must be 1..3");
    for (int l = 0; l < d->n_levels; ++l) {
        const bool okn = d->dim == 2 ? pow2_in(d->grid_n[l], 16, 256) : pow2_in(d->grid_n[l], 8, 1024);
        if (!okn) return fail(SMC_E_INVAL, "grid_n[%d] = %d is not a supported power of two", l, d->grid_n[l]);
    }
    if (d->dim == 2 && (d->kl < 1 || d->kl > 32)) return fail(SMC_E_INVAL, "2D kl must be 1..32");
    if (d->dim == 1 && (d->kl < 1 || d->kl > 64)) return fail(SMC_E_INVAL, "1D kl must be 1..64");
    const int K = d->dim == 2 ? d->kl * d->kl : d->kl;
    if (d->kr < 1 || d->kr > MAX_KR || d->kr > K) return fail(SMC_E_INVAL, "kr must be 1..min(64, K)");
    if (d->n_obs < 1 || d->n_obs > MAX_OBS) return fail(SMC_E_INVAL, "n_obs must be 1..64");
    if (d->obs_den < 1 || !d->obs_num || !d->y) return fail(SMC_E_INVAL, "observation arrays missing");
    if (!(d->sigma > 0.0) || !std::isfinite(d->sigma)) return fail(SMC_E_INVAL, "sigma must be positive");
    if (!std::isfinite(d->f)) return fail(SMC_E_INVAL, "f must be finite");
    if (d->n_max < 1 || d->n_max > (1 << 24)) return fail(SMC_E_INVAL, "n_max must be 1..2^24");
    if (!(d->tol64 > 0.0) || !(d->tol_inner > 0.0 && d->tol_inner < 1.0))
        return fail(SMC_E_INVAL, "tolerances must be positive (tol_inner < 1)");
    if (d->max_iter < 1 || d->max_sweeps < 1) return fail(SMC_E_INVAL, "max_iter and max_sweeps must be >= 1");
    if (d->precond != SMC_PRECOND_AUTO && d->precond != SMC_PRECOND_JACOBI)
        return fail(SMC_E_INVAL, "unknown preconditioner %d", d->precond);
    for (int k = 0; k < d->n_obs; ++k) {
        if (!std::isfinite(d->y[k])) return fail(SMC_E_INVAL, "y[%d] is not finite", k);
        for (int a = 0; a < d->dim; ++a) {
            const int num = d->obs_num[k * d->dim + a];
            if (num <= 0 || num >= d->obs_den) return fail(SMC_E_INVAL, "observation %d is not interior", k);
            for (int l = 0; l < d->n_levels; ++l)
                if (((int64_t)num * d->grid_n[l]) % d->obs_den)
                    return fail(SMC_E_INVAL, "observation %d is not a node of grid %d", k, d->grid_n[l]);
        }
    }

    smc_problem_s* ps = new smc_problem_s();
    Problem& P = ps->P;
    (void)hipGetDevice(&ps->device);
    P.dim = d->dim;
    P.n_levels = d->n_levels;
    P.kl = d->kl;
    P.K = K;
    P.kr = d->kr;
    P.n_obs = d->n_obs;
    P.sigma = d->sigma;
    P.f = d->f;
    P.tol64 = d->tol64;
    P.tol_inner = d->tol_inner;
    P.max_iter = d->max_iter;
    P.max_sweeps = d->max_sweeps;
    P.precond = d->precond;
    P.n_max = d->n_max;

    // prior: sqrt(lambda) and the active modes (largest lambda first, ties to the lower index)
    std::vector<double> sl(K);
    std::vector<int> key(K);
    for (int idx = 0; idx < K; ++idx) {
        double mu;
        if (P.dim == 2) {
            const int k = idx / P.kl, l = idx % P.kl;
            key[idx] = k * k + l * l;
            mu = 1.0 + M_PI * M_PI * (double)(k * k + l * l);
        } else {
            key[idx] = idx;
            mu = 1.0 + M_PI * M_PI * (double)((idx + 1) * (idx + 1));
        }
        sl[idx] = 1.0 / mu;   // sqrt of lambda = mu^{-2}
    }
    std::vector<int> order(K);
    for (int idx = 0; idx < K; ++idx) order[idx] = idx;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key[a] < key[b]; });
    std::vector<int32_t> act(order.begin(), order.begin() + P.kr), slot(K, -1);
    for (int a = 0; a < P.kr; ++a) {
        slot[act[a]] = a;
        P.active_h[a] = act[a];
    }

    hipError_t e = hipSuccess;
    auto ck = [&](hipError_t r) { if (e == hipSuccess) e = r; };
    ck(prepare_kernels());
    ck(hipDeviceGetAttribute(&P.n_cu, hipDeviceAttributeMultiprocessorCount, ps->device));
    ck(upload(&P.sqrt_lam, sl.data(), K));
    ck(upload(&P.active, act.data(), act.size()));
    ck(upload(&P.slot, slot.data(), slot.size()));
    ck(upload(&P.y, d->y, P.n_obs));
    P.n_big = 0;
    for (int l = 0; l < P.n_levels; ++l) {
        const int n = d->grid_n[l];
        P.lv[l].n = n;
        P.n_big = std::max(P.n_big, n);
        std::vector<double> B;
        if (P.dim == 2) {
            B.assign((size_t)(n + 1) * KLP, 0.0);
            for (int i = 0; i <= n; ++i)
                for (int k = 0; k < P.kl; ++k)
                    B[(size_t)i * KLP + k] = (k == 0 ? 1.0 : std::sqrt(2.0)) * std::cos(M_PI * k * (double)i / n);
        } else {
            B.assign((size_t)(n + 1) * P.kl, 0.0);
            for (int i = 0; i <= n; ++i)
                for (int k = 0; k < P.kl; ++k)
                    B[(size_t)i * P.kl + k] = std::sqrt(2.0) * std::sin(M_PI * (k + 1) * (double)i / n);
        }
        ck(upload(&P.lv[l].basis, B.data(), B.size()));
        std::vector<int32_t> nodes(P.n_obs);
        for (int k = 0; k < P.n_obs; ++k) {
            const int ii = (int)((int64_t)d->obs_num[k * P.dim] * n / d->obs_den);
            if (P.dim == 2) {
                const int jj = (int)((int64_t)d->obs_num[k * P.dim + 1] * n / d->obs_den);
                nodes[k] = jj * (n + 1) + ii;
            } else {
                nodes[k] = ii;
            }
        }
        ck(upload(&P.lv[l].obs_node, nodes.data(), nodes.size()));
        if (P.dim == 2 && dst_supported(n)) {
            // S[a][b] = sqrt(2/n) sin(pi (a+1)(b+1) / n) for nodes a+1, b+1 = 1..n; the last row and
            // column (the boundary padding node n) are exactly zero.  FP16: the solvers scale their
            // transform operands into FP16's range
            std::vector<double> S((size_t)n * n);
            std::vector<float> lam(n);
            for (int r = 0; r < n; ++r) {
                lam[r] = (float)std::pow(std::sin(M_PI * (r + 1) / (2.0 * n)), 2);
                for (int q = 0; q < n; ++q)
                    S[(size_t)r * n + q] = (r == n - 1 || q == n - 1)
                                               ? 0.0
                                               : std::sqrt(2.0 / n) * std::sin(M_PI * (double)((r + 1) * (q + 1)) / n);
            }
            std::vector<_Float16> Sh(S.size());
            for (size_t k = 0; k < S.size(); ++k) Sh[k] = (_Float16)(float)S[k];
            ck(upload((_Float16**)&P.lv[l].dst_S, Sh.data(), Sh.size()));
            ck(upload(&P.lv[l].dst_lam, lam.data(), lam.size()));
        }
    }
    const int64_t nb = P.n_big;
    P.e_stride = P.dim == 2 ? (nb + 1) * (nb + 1) : nb + 1;
    P.x_stride = P.e_stride;
    P.vec_stride = P.dim == 2 ? 7 * nb * nb : 0;
    const int64_t Nm = P.n_max;
    ck(hipMalloc((void**)&P.ws_v, sizeof(double) * Nm * K));
    ck(hipMalloc((void**)&P.ws_logr, sizeof(double) * Nm));
    ck(hipMalloc((void**)&P.ws_phinew, sizeof(double) * Nm));
    ck(hipMalloc((void**)&P.ws_e, sizeof(double) * Nm * P.e_stride));
    ck(hipMalloc((void**)&P.ws_x64, sizeof(double) * Nm * P.x_stride));
    ck(hipMalloc((void**)&P.ws_sd, sizeof(double) * Nm * P.x_stride));
    if (P.dim == 2) {
        ck(hipMalloc((void**)&P.ws_lam, sizeof(double) * Nm * P.x_stride));
        ck(hipMalloc((void**)&P.ws_gnew, sizeof(double) * Nm * K));
    }
    if (P.dim == 2 && P.n_big >= 128) ck(hipMalloc(&P.ws_vec, sizeof(double) * Nm * P.vec_stride));
    ck(hipMalloc((void**)&P.ws_G, sizeof(double) * Nm * P.n_obs));
    ck(hipMalloc((void**)&P.ws_iters, sizeof(int32_t) * Nm));
    ck(hipMalloc((void**)&P.ws_list, sizeof(int32_t) * Nm));
    ck(hipMalloc((void**)&P.ws_counters, N_COUNTERS * sizeof(unsigned long long)));
    ck(hipMemset(P.ws_counters, 0, N_COUNTERS * sizeof(unsigned long long)));
    {
        const size_t pe = (size_t)MAX_M * (1 + 2 * MAX_KR);
        ck(hipMalloc((void**)&P.ws_fit_d2, sizeof(double) * Nm));
        ck(hipMalloc((void**)&P.ws_fit_par, sizeof(double) * 2 * GM_PAR));
        ck(hipMalloc((void**)&P.ws_fit_part, sizeof(double) * em_blocks(Nm) * pe));
        ck(hipMalloc((void**)&P.ws_fit_centers, sizeof(int32_t) * MAX_M));
        ck(hipMalloc((void**)&P.ws_mixtab, sizeof(double) * MAX_LEVELS * MIXTAB));
    }
    ck(hipMalloc((void**)&P.flags, sizeof(int32_t)));
    ck(hipMalloc((void**)&P.stats, 4 * sizeof(unsigned long long)));
    ck(hipMemset(P.stats, 0, 4 * sizeof(unsigned long long)));
    ck(hipMemset(P.flags, 0, sizeof(int32_t)));
    ck(hipDeviceSynchronize());
    if (e != hipSuccess) {
        free_problem(P);
        delete ps;
        return fail(e == hipErrorOutOfMemory ? SMC_E_NOMEM : SMC_E_HIP, "problem setup: %s", hipGetErrorString(e));
    }
    *out = ps;
    return SMC_OK;
}

extern "C" int smc_problem_create_l2mix(const smc_l2mix_desc* d, smc_problem* out) {
    if (!d || !out) return fail(SMC_E_INVAL, "desc and out must not be NULL");
    if (d->K < 1 || d->K > 1024) return fail(SMC_E_INVAL, "K must be 1..1024");
    if (d->kr < 1 || d->kr > MAX_KR || d->kr > d->K) return fail(SMC_E_INVAL, "kr must be 1..min(64, K)");
    if (!(d->alpha > 0.0) || !std::isfinite(d->alpha)) return fail(SMC_E_INVAL, "alpha must be positive");
    if (d->n_terms < 1 || d->n_terms > MAX_TERMS) return fail(SMC_E_INVAL, "n_terms must be 1..%d", MAX_TERMS);
    if (!d->c) return fail(SMC_E_INVAL, "c must not be NULL");
    for (int64_t i = 0; i < (int64_t)d->n_terms * d->K; ++i)
        if (!std::isfinite(d->c[i])) return fail(SMC_E_INVAL, "c[%lld] is not finite", (long long)i);
    if (!(d->sigma > 0.0) || !std::isfinite(d->sigma)) return fail(SMC_E_INVAL, "sigma must be positive");
    if (d->n_max < 1 || d->n_max > (1 << 24)) return fail(SMC_E_INVAL, "n_max must be 1..2^24");

    smc_problem_s* ps = new smc_problem_s();
    Problem& P = ps->P;
    (void)hipGetDevice(&ps->device);
    P.kind = KIND_L2MIX;
    P.dim = 1;
    P.n_levels = 0;
    P.kl = d->K;
    P.K = d->K;
    P.kr = d->kr;
    P.n_obs = 0;
    P.n_terms = d->n_terms;
    P.sigma = d->sigma;
    P.n_max = d->n_max;
    // lambda_k = (1 + alpha k^2 pi^2)^{-2} decreases with k: the active modes are 0 .. kr-1
    std::vector<double> sl(P.K);
    for (int k = 0; k < P.K; ++k) sl[k] = 1.0 / (1.0 + d->alpha * M_PI * M_PI * (double)k * k);
    std::vector<int32_t> act(P.kr), slot(P.K, -1);
    for (int a = 0; a < P.kr; ++a) {
        act[a] = a;
        slot[a] = a;
        P.active_h[a] = a;
    }
    hipError_t e = hipSuccess;
    auto ck = [&](hipError_t r) { if (e == hipSuccess) e = r; };
    ck(prepare_kernels());
    ck(hipDeviceGetAttribute(&P.n_cu, hipDeviceAttributeMultiprocessorCount, ps->device));
    ck(upload(&P.sqrt_lam, sl.data(), P.K));
    ck(upload(&P.active, act.data(), act.size()));
    ck(upload(&P.slot, slot.data(), slot.size()));
    ck(upload(&P.mix_c, d->c, (size_t)P.n_terms * P.K));
    const int64_t Nm = P.n_max;
    ck(hipMalloc((void**)&P.ws_v, sizeof(double) * Nm * P.K));
    ck(hipMalloc((void**)&P.ws_logr, sizeof(double) * Nm));
    ck(hipMalloc((void**)&P.ws_phinew, sizeof(double) * Nm));
    ck(hipMalloc((void**)&P.ws_iters, sizeof(int32_t) * Nm));
    ck(hipMalloc((void**)&P.ws_fit_d2, sizeof(double) * Nm));
    ck(hipMalloc((void**)&P.ws_fit_par, sizeof(double) * 2 * GM_PAR));
    ck(hipMalloc((void**)&P.ws_fit_part, sizeof(double) * em_blocks(Nm) * MAX_M * (1 + 2 * MAX_KR)));
    ck(hipMalloc((void**)&P.ws_fit_centers, sizeof(int32_t) * MAX_M));
    ck(hipMalloc((void**)&P.ws_mixtab, sizeof(double) * MAX_LEVELS * MIXTAB));
    ck(hipMalloc((void**)&P.flags, sizeof(int32_t)));
    ck(hipMalloc((void**)&P.stats, 4 * sizeof(unsigned long long)));
    ck(hipMemset(P.stats, 0, 4 * sizeof(unsigned long long)));
    ck(hipMemset(P.flags, 0, sizeof(int32_t)));
    ck(hipDeviceSynchronize());
    if (e != hipSuccess) {
        free_problem(P);
        delete ps;
        return fail(e == hipErrorOutOfMemory ? SMC_E_NOMEM : SMC_E_HIP, "problem setup: %s", hipGetErrorString(e));
    }
    *out = ps;
    return SMC_OK;
}

extern "C" void smc_problem_destroy(smc_problem p) {
    if (!p) return;
    (void)hipDeviceSynchronize();
    for (hipEvent_t e : p->pool.ev) (void)hipEventDestroy(e);
    free_problem(p->P);
    delete p;
}

// Record one event of the current solve launch's bracket on stream s; the closing event of a
// launch that holds several solve rounds (a stage launch) gives their number.
static hipError_t record(EventPool& pool, hipStream_t s, int rounds = 1) {
    if (pool.used == pool.ev.size()) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        pool.ev.push_back(e);
    }
    if (pool.used % 2) {
        if (pool.rounds.size() <= pool.used / 2) pool.rounds.resize(pool.used / 2 + 1);
        pool.rounds[pool.used / 2] = rounds;
    }
    return hipEventRecord(pool.ev[pool.used++], s);
}

extern "C" int smc_profile(smc_problem p, int32_t enable) {
    if (!p) return fail(SMC_E_INVAL, "problem is NULL");
    if (enable) {
        HIPCHK(hipDeviceSynchronize());
        HIPCHK(hipMemset(p->P.stats, 0, 4 * sizeof(unsigned long long)));
        HIPCHK(hipDeviceSynchronize());
        p->pool.used = 0;
    }
    p->P.profiling = enable != 0;
    return SMC_OK;
}

extern "C" int smc_profile_read(smc_problem p, smc_stream stream, double* ms, int64_t* launches, int64_t* iters,
                                int64_t* sweeps, int64_t* solves, int64_t* precond_apps) {
    if (!p) return fail(SMC_E_INVAL, "problem is NULL");
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    double tot = 0.0;
    for (size_t k = 0; k + 1 < p->pool.used; k += 2) {
        float t = 0.0f;
        HIPCHK(hipEventElapsedTime(&t, p->pool.ev[k], p->pool.ev[k + 1]));
        tot += t;
    }
    unsigned long long st[4];
    HIPCHK(hipMemcpy(st, p->P.stats, sizeof(st), hipMemcpyDeviceToHost));
    int64_t rounds = 0;
    for (size_t k = 0; k < p->pool.used / 2; ++k) rounds += k < p->pool.rounds.size() ? p->pool.rounds[k] : 1;
    if (ms) *ms = tot;
    if (launches) *launches = rounds;
    if (iters) *iters = (int64_t)st[0];
    if (sweeps) *sweeps = (int64_t)st[1];
    if (solves) *solves = (int64_t)st[2];
    if (precond_apps) *precond_apps = (int64_t)st[3];
    return SMC_OK;
}

extern "C" int smc_problem_info(smc_problem p, int32_t* K, int32_t* active, int32_t* n_obs) {
    if (!p) return fail(SMC_E_INVAL, "problem is NULL");
    if (K) *K = p->P.K;
    if (n_obs) *n_obs = p->P.n_obs;
    if (active) std::copy(p->P.active_h, p->P.active_h + p->P.kr, active);
    return SMC_OK;
}

extern "C" int smc_status_flags(smc_problem p, smc_stream stream, int32_t* flags, int32_t clear) {
    if (!p || !flags) return fail(SMC_E_INVAL, "problem and flags must not be NULL");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipStreamSynchronize(s));
    HIPCHK(hipMemcpy(flags, p->P.flags, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (clear) {
        HIPCHK(launch_fill_i32(p->P.flags, 1, 0, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    return SMC_OK;
}

static int check_n(const Problem& P, int64_t N) {
    if (N < 0 || N > P.n_max) return fail(SMC_E_INVAL, "N = %lld outside 0..n_max (%lld)", (long long)N,
                                          (long long)P.n_max);
    return SMC_OK;
}

extern "C" int smc_prior_sample(smc_problem p, int64_t N, uint64_t seed, uint64_t ctr, double* xi,
                                smc_stream stream) {
    if (!p) return fail(SMC_E_INVAL, "problem is NULL");
    if (int r = check_n(p->P, N)) return r;
    if (N > 0 && !xi) return fail(SMC_E_INVAL, "xi is NULL");
    if (N > 0xFFFFFFFFll) return fail(SMC_E_INVAL, "N exceeds the 32-bit particle counter");
    HIPCHK(launch_prior(N, p->P.K, seed, ctr, xi, (hipStream_t)stream));
    return SMC_OK;
}

// exp(u/2) (or u) of the particles' fields on one grid into `out`.
static hipError_t synth(const Problem& P, int level, int64_t N, const double* xi, double* out, int64_t stride,
                        bool exp_half, hipStream_t s) {
    const Level& L = P.lv[level];
    if (P.dim == 2) return launch_synth2d(xi, P.K, P.kl, P.sqrt_lam, L.basis, L.n, out, stride, N, exp_half, s);
    return launch_synth1d(xi, P.kl, P.sqrt_lam, L.basis, L.n, out, stride, N, exp_half, s);
}

extern "C" int smc_synthesize(smc_problem p, int64_t N, const double* xi, int32_t level, double* u,
                              smc_stream stream) {
    if (!p) return fail(SMC_E_INVAL, "problem is NULL");
    if (int r = check_n(p->P, N)) return r;
    if (level < 0 || level >= p->P.n_levels) return fail(SMC_E_INVAL, "level %d out of range", level);
    if (N > 0 && (!xi || !u)) return fail(SMC_E_INVAL, "xi and u must not be NULL");
    const int n = p->P.lv[level].n;
    const int64_t stride = p->P.dim == 2 ? (int64_t)(n + 1) * (n + 1) : n + 1;
    HIPCHK(synth(p->P, level, N, xi, u, stride, false, (hipStream_t)stream));
    return SMC_OK;
}

static SolveArgs solve_args(const Problem& P, int level) {
    SolveArgs a{};
    a.e = P.ws_e;
    a.x64 = P.ws_x64;
    a.sd = P.ws_sd;
    a.vec = P.ws_vec;
    a.e_stride = P.e_stride;
    a.x_stride = P.x_stride;
    a.sd_stride = P.x_stride;
    a.vec_stride = P.vec_stride;
    a.lam = nullptr;
    a.lam_stride = P.x_stride;
    a.fwd_given = 0;
    a.row0 = 0;
    a.obs = P.lv[level].obs_node;
    a.n_obs = P.n_obs;
    a.y = P.y;
    a.inv2s2 = 0.5 / (P.sigma * P.sigma);
    a.f = P.f;
    a.tol64 = P.tol64;
    a.tol_inner = P.tol_inner;
    a.max_iter = P.max_iter;
    a.max_sweeps = P.max_sweeps;
    a.flags = P.flags;
    a.stats = nullptr;
    return a;
}

// Outputs and options of one batch of forward (and adjoint) solves; every pointer may be NULL.
struct Solve {
    const int32_t* level = nullptr;   // [N] grid of each particle (work list already planned), or null
    double* G = nullptr;
    double* phi = nullptr;
    int32_t* iters = nullptr;
    double* w = nullptr;          // caller's forward-state buffer [N][n*n] (else the workspace)
    bool w_given = false;         // w already holds the forward solutions: solve the adjoint only
    bool adjoint = false;         // also solve A lam = P^T (P w - y) / sigma^2 into the workspace
};

// Synthesis then solve for N particles of one grid.
static LevelTable level_table(const Problem& P) {
    LevelTable t{};
    t.n_levels = P.n_levels;
    for (int l = 0; l < P.n_levels; ++l) {
        t.n[l] = P.lv[l].n;
        t.basis[l] = P.lv[l].basis;
        t.obs[l] = P.lv[l].obs_node;
        t.S[l] = P.lv[l].dst_S;
        t.lam[l] = P.lv[l].dst_lam;
    }
    return t;
}

// Host checks for a per-particle level map: 2D, and every grid served by the mixed-grid solve.
static int check_levels(const Problem& P) {
    if (P.dim != 2) return fail(SMC_E_INVAL, "level maps need the 2D problem");
    for (int l = 0; l < P.n_levels; ++l)
        if (!mixed_supported(P.lv[l].n))
            return fail(SMC_E_INVAL, "grid %d cannot be mixed with others in one launch (64, 128, 256 can)",
                        P.lv[l].n);
    return SMC_OK;
}

static hipError_t forward_levels(smc_problem_s* ps, int prec, int64_t N, const double* xi, const Solve& o,
                                 hipStream_t s) {
    const Problem& P = ps->P;
    const LevelTable lt = level_table(P);
    hipError_t e = launch_synth2d_levels(xi, P.K, P.kl, P.sqrt_lam, lt, o.level, P.ws_e, P.e_stride, N, true, s);
    if (e != hipSuccess) return e;
    SolveArgs a = solve_args(P, 0);
    a.G = o.G;
    a.phi = o.phi;
    a.iters = o.iters;
    a.stats = P.profiling ? P.stats : nullptr;
    const bool rec = P.profiling && !ps->capturing;
    if (rec && (e = record(ps->pool, s)) != hipSuccess) return e;
    const bool dst = P.precond == SMC_PRECOND_AUTO;
    if (dst) {   // one launch per grid, each in its single-grid shape
        int rows[MAX_LEVELS] = {};
        for (int l = 0; l < P.n_levels; ++l) rows[l] = P.lv[l].rows;
        e = launch_solve_levels(prec, N, a, lt, rows, P.ws_list, P.ws_counters, P.n_cu, s);
    } else {
        e = launch_solve_mixed(prec, dst, N, a, lt, o.level, P.ws_list, P.ws_counters, P.n_cu, s);
    }
    if (e != hipSuccess) return e;
    if (rec) e = record(ps->pool, s);
    return e;
}

// Whether the adjoint solve of grid `level` at precision `prec` forms dPhi/du itself: the on-chip
// FP32 solvers with the fast-Poisson preconditioner on grids whose rows span whole waves (64, 128).
static bool du_formed(const Problem& P, int level, int prec) {
    const Level& L = P.lv[level];
    return P.dim == 2 && prec == SMC_FP32_REFINE && P.precond == SMC_PRECOND_AUTO && L.dst_S &&
           (L.n == 64 || L.n == 128);
}

static hipError_t forward(smc_problem_s* ps, int level, int prec, int64_t N, const double* xi, const Solve& o,
                          hipStream_t s) {
    const Problem& P = ps->P;
    if (P.kind == KIND_L2MIX)   // the potential is a closed form of xi: no synthesis, no solve
        return launch_l2mix_phi(N, P.K, P.sqrt_lam, P.mix_c, P.n_terms, 0.5 / (P.sigma * P.sigma), xi, o.phi,
                                o.iters, s);
    if (o.level) return forward_levels(ps, prec, N, xi, o, s);
    hipError_t e = synth(P, level, N, xi, P.ws_e, P.e_stride, true, s);
    if (e != hipSuccess) return e;
    const Level& L = P.lv[level];
    SolveArgs a = solve_args(P, level);
    a.G = o.G;
    a.phi = o.phi;
    a.iters = o.iters;
    if (o.w) {
        a.x64 = o.w;
        a.x_stride = P.dim == 2 ? (int64_t)L.n * L.n : L.n + 1;
    }
    a.fwd_given = o.w_given ? 1 : 0;
    a.lam = o.adjoint ? P.ws_lam : nullptr;
    a.stats = P.profiling ? P.stats : nullptr;
    // the on-chip FP32 solvers form dPhi/du after the adjoint solve, into the scaling rows (free once
    // the solve is done); the gradient then only contracts it (see du_formed)
    if (o.adjoint && du_formed(P, level, prec)) {
        a.du = P.ws_sd;
        a.du_stride = P.x_stride;
    }
    const bool rec = P.profiling && !ps->capturing;
    if (rec && (e = record(ps->pool, s)) != hipSuccess) return e;
    if (P.dim == 1)
        e = launch_solve1d(L.n, N, a, s);
    else if (prec == SMC_FP32_REFINE && P.precond == SMC_PRECOND_AUTO && L.dst_S)
        e = launch_solve2d_dst(L.n, L.rows, N, a, L.dst_S, L.dst_lam, s);
    else if (prec == SMC_FP64 && P.precond == SMC_PRECOND_AUTO && L.dst_S && (L.n == 128 || L.n == 256))
        e = launch_solve2d_dst64(L.n, N, a, L.dst_S, L.dst_lam, s);
    else if (prec == SMC_FP64 && P.precond == SMC_PRECOND_AUTO && L.dst_S && (L.n == 32 || L.n == 64))
        e = launch_solve2d_dst64_onchip(L.n, N, a, L.dst_S, L.dst_lam, s);
    else
        e = launch_solve2d(L.n, prec, N, a, s);
    if (e != hipSuccess) return e;
    if (rec) e = record(ps->pool, s);
    return e;
}

// Gradient of the N particles' potentials after forward(..., adjoint = true, prec).
static hipError_t gradient(const Problem& P, int level, int prec, int64_t N, const double* w, int64_t w_stride,
                           const int32_t* iters, double* grad, hipStream_t s) {
    const Level& L = P.lv[level];
    const bool du = du_formed(P, level, prec);
    return launch_gradsynth2d(P.ws_e, P.e_stride, w, w_stride, P.ws_lam, P.x_stride, iters, P.sqrt_lam, L.basis, L.n,
                              P.kl, P.K, grad, N, du ? P.ws_sd : nullptr, P.x_stride, s);
}

extern "C" int smc_phi_batch(smc_problem p, int64_t N, const double* xi, const int32_t* level, int32_t prec,
                             double* phi, int32_t* iters, smc_stream stream) {
    if (!p) return fail(SMC_E_INVAL, "problem is NULL");
    const Problem& P = p->P;
    if (int r = check_n(P, N)) return r;
    if (N > 0 && (!xi || !phi)) return fail(SMC_E_INVAL, "xi and phi must not be NULL");
    if (prec != SMC_FP64 && prec != SMC_FP32_REFINE) return fail(SMC_E_INVAL, "unknown precision %d", prec);
    if (level) {
        if (int r = check_levels(P)) return r;
        if (N > 0) HIPCHK(launch_plan(N, level, level_table(P), P.ws_list, P.ws_counters, P.flags,
                                      (hipStream_t)stream));
    }
    Solve o;
    o.level = level;
    o.phi = phi;
    o.iters = iters;
    HIPCHK(forward(p, 0, prec, N, xi, o, (hipStream_t)stream));
    return SMC_OK;
}

extern "C" int smc_forward_batch(smc_problem p, int64_t N, const double* xi, const int32_t* level,
                                 int32_t prec, double* G, int32_t* iters, smc_stream stream) {
    if (!p) return fail(SMC_E_INVAL, "problem is NULL");
    if (p->P.kind != KIND_DARCY) return fail(SMC_E_INVAL, "this problem has no observation operator");
    if (int r = check_n(p->P, N)) return r;
    if (N > 0 && (!xi || !G)) return fail(SMC_E_INVAL, "xi and G must not be NULL");
    if (prec != SMC_FP64 && prec != SMC_FP32_REFINE) return fail(SMC_E_INVAL, "unknown precision %d", prec);
    if (level) {
        if (int r = check_levels(p->P)) return r;
        if (N > 0) HIPCHK(launch_plan(N, level, level_table(p->P), p->P.ws_list, p->P.ws_counters, p->P.flags,
                                      (hipStream_t)stream));
    }
    Solve o;
    o.level = level;
    o.G = G;
    o.iters = iters;
    HIPCHK(forward(p, 0, prec, N, xi, o, (hipStream_t)stream));
    return SMC_OK;
}

extern "C" int smc_forward_state(smc_problem p, int64_t N, const double* xi, int32_t prec, double* G, double* w,
                                 int32_t* iters, smc_stream stream) {
    if (!p) return fail(SMC_E_INVAL, "problem is NULL");
    if (p->P.dim != 2) return fail(SMC_E_INVAL, "forward states are kept for the 2D problem only");
    if (int r = check_n(p->P, N)) return r;
    if (N > 0 && (!xi || !w)) return fail(SMC_E_INVAL, "xi and w must not be NULL");
    if (prec != SMC_FP64 && prec != SMC_FP32_REFINE) return fail(SMC_E_INVAL, "unknown precision %d", prec);
    Solve o;
    o.G = G;
    o.iters = iters;
    o.w = w;
    HIPCHK(forward(p, 0, prec, N, xi, o, (hipStream_t)stream));
    return SMC_OK;
}

extern "C" int smc_value_and_grad(smc_problem p, int64_t N, const double* xi, int32_t prec, const double* w,
                                  double* phi, double* grad, int32_t* iters, smc_stream stream) {
    if (!p) return fail(SMC_E_INVAL, "problem is NULL");
    const Problem& P = p->P;
    if (P.dim != 2) return fail(SMC_E_INVAL, "the adjoint gradient is implemented for the 2D problem");
    if (int r = check_n(P, N)) return r;
    if (N > 0 && (!xi || !grad)) return fail(SMC_E_INVAL, "xi and grad must not be NULL");
    if (prec != SMC_FP64 && prec != SMC_FP32_REFINE) return fail(SMC_E_INVAL, "unknown precision %d", prec);
    hipStream_t s = (hipStream_t)stream;
    Solve o;
    o.phi = phi;
    o.iters = iters ? iters : P.ws_iters;
    o.adjoint = true;
    if (w) {
        o.w = const_cast<double*>(w);   // read only: the forward pass is skipped
        o.w_given = true;
    }
    HIPCHK(forward(p, 0, prec, N, xi, o, s));
    const int n = P.lv[0].n;
    HIPCHK(gradient(P, 0, prec, N, w ? w : P.ws_x64, w ? (int64_t)n * n : P.x_stride, o.iters, grad, s));
    return SMC_OK;
}

extern "C" int smc_potential(smc_problem p, int64_t N, const double* G, double* phi, smc_stream stream) {
    if (!p) return fail(SMC_E_INVAL, "problem is NULL");
    if (p->P.kind != KIND_DARCY) return fail(SMC_E_INVAL, "this problem has no observations (use smc_phi_batch)");
    if (int r = check_n(p->P, N)) return r;
    if (N > 0 && (!G || !phi)) return fail(SMC_E_INVAL, "G and phi must not be NULL");
    HIPCHK(launch_potential(N, p->P.n_obs, G, p->P.y, 0.5 / (p->P.sigma * p->P.sigma), phi, (hipStream_t)stream));
    return SMC_OK;
}

// Tile of the fast-Poisson solver of grid `level` (the set one, else the default).
static int tile_rows(const Problem& P, int level) {
    int c[8];
    tile_candidates(P.lv[level].n, c);
    return P.lv[level].rows ? P.lv[level].rows : c[0];
}

// A whole stage of moves in one persistent launch (single grid, FP32 with refinement, on-chip
// fast-Poisson solver with a tile that has a stage kernel).
static bool stage_fusable(const smc_problem_s* p, const int32_t* level, int32_t prec) {
    const Problem& P = p->P;
    if (!p->fuse_stage || level || P.kind != KIND_DARCY || P.dim != 2 || prec != SMC_FP32_REFINE ||
        P.precond != SMC_PRECOND_AUTO || !P.lv[0].dst_S)
        return false;
    return stage_fused_supported(P.lv[0].n, tile_rows(P, 0));
}

static hipError_t stage_launch(smc_problem_s* ps, int64_t N, const MoveParams& q, int32_t n_moves, double* xi,
                               double* phi, int32_t* n_acc, hipStream_t s) {
    const Problem& P = ps->P;
    const Level& L = P.lv[0];
    SolveArgs a = solve_args(P, 0);
    a.phi = P.ws_phinew;
    a.iters = P.ws_iters;
    a.stats = P.profiling ? P.stats : nullptr;
    StageArgs st{};
    st.N = N;
    st.K = P.K;
    st.kl = P.kl;
    st.n_moves = n_moves;
    st.active = P.active;
    st.slot = P.slot;
    st.tab = P.ws_mixtab;
    st.sqrt_lam = P.sqrt_lam;
    st.basis = L.basis;
    st.xi = xi;
    st.phi = phi;
    st.n_acc = n_acc;
    st.v = P.ws_v;
    st.logr = P.ws_logr;
    st.flags = P.flags;
    const bool rec = P.profiling && !ps->capturing;
    hipError_t e;
    if (rec && (e = record(ps->pool, s)) != hipSuccess) return e;
    e = launch_stage_onchip(L.n, tile_rows(P, 0), a, st, q, L.dst_S, L.dst_lam, P.ws_counters, P.n_cu, s);
    if (e != hipSuccess) return e;
    if (rec) e = record(ps->pool, s, n_moves);
    return e;
}

// The move loop shared by smc_gmpcn_move and smc_gmpcn_stage (arguments already checked).
static int move_loop(smc_problem_s* p, int64_t N, MoveParams q, int32_t n_moves, const int32_t* level, int32_t prec,
                     double* xi, double* phi, int32_t* n_acc, hipStream_t s) {
    const Problem& P = p->P;
    if (N <= 0) return SMC_OK;
    HIPCHK(launch_fill_i32(n_acc, N, 0, s));
    if (level) HIPCHK(launch_plan(N, level, level_table(P), P.ws_list, P.ws_counters, P.flags, s));
    if (n_moves > 0) HIPCHK(launch_mixtab(q, P.ws_mixtab, s));
    if (n_moves > 0 && stage_fusable(p, level, prec)) {
        HIPCHK(stage_launch(p, N, q, n_moves, xi, phi, n_acc, s));
        return SMC_OK;
    }
    for (int m = 0; m < n_moves; ++m) {
        q.m = m;
        HIPCHK(launch_propose(N, P.K, P.active, P.slot, q, P.ws_mixtab, xi, P.ws_v, P.ws_logr, P.flags, s));
        Solve o;
        o.level = level;
        o.phi = P.ws_phinew;
        o.iters = P.ws_iters;
        HIPCHK(forward(p, 0, prec, N, P.ws_v, o, s));
        HIPCHK(launch_accept(N, P.K, q, P.ws_v, P.ws_logr, P.ws_phinew, xi, phi, n_acc, s));
    }
    return SMC_OK;
}

static int check_move_common(const Problem& P, int64_t N, int32_t n_moves, const int32_t* level, int32_t prec,
                             double* xi, double* phi, int32_t* n_acc) {
    if (int r = check_n(P, N)) return r;
    if (n_moves < 0) return fail(SMC_E_INVAL, "n_moves must be >= 0");
    if (prec != SMC_FP64 && prec != SMC_FP32_REFINE) return fail(SMC_E_INVAL, "unknown precision %d", prec);
    if (level)
        if (int r = check_levels(P)) return r;
    if (N > 0 && (!xi || !phi || !n_acc)) return fail(SMC_E_INVAL, "xi, phi and n_acc must not be NULL");
    if (N > 0xFFFFFFFFll) return fail(SMC_E_INVAL, "N exceeds the 32-bit particle counter");
    return SMC_OK;
}

static int check_gm(const Problem& P, const smc_gm* gm) {
    if (!gm) return fail(SMC_E_INVAL, "gm is NULL");
    if (gm->M < 1 || gm->M > MAX_M) return fail(SMC_E_INVAL, "M must be 1..%d", MAX_M);
    if (gm->kr != P.kr) return fail(SMC_E_INVAL, "gm.kr (%d) differs from the problem's kr (%d)", gm->kr, P.kr);
    if (!gm->logw || !gm->mean || !gm->scale) return fail(SMC_E_INVAL, "mixture arrays must not be NULL");
    return SMC_OK;
}

extern "C" int smc_gm_draw(smc_problem p, int64_t N, const smc_gm* gm, uint64_t seed, uint64_t ctr,
                           const int32_t* level, int32_t prec, double* xi, double* phi, int32_t* iters,
                           smc_stream stream) {
    if (!p) return fail(SMC_E_INVAL, "problem is NULL");
    const Problem& P = p->P;
    if (int r = check_gm(P, gm)) return r;
    if (int r = check_n(P, N)) return r;
    if (prec != SMC_FP64 && prec != SMC_FP32_REFINE) return fail(SMC_E_INVAL, "unknown precision %d", prec);
    if (level)
        if (int r = check_levels(P)) return r;
    if (N > 0 && (!xi || !phi)) return fail(SMC_E_INVAL, "xi and phi must not be NULL");
    if (N > 0xFFFFFFFFll) return fail(SMC_E_INVAL, "N exceeds the 32-bit particle counter");
    if (N == 0) return SMC_OK;
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(launch_gm_draw(N, P.K, P.slot, seed, ctr, gm->M, gm->kr, gm->logw, gm->mean, gm->scale, xi, s));
    if (level) HIPCHK(launch_plan(N, level, level_table(P), P.ws_list, P.ws_counters, P.flags, s));
    Solve o;
    o.level = level;
    o.phi = phi;
    o.iters = iters ? iters : P.ws_iters;
    HIPCHK(forward(p, 0, prec, N, xi, o, s));
    return SMC_OK;
}

extern "C" int smc_gm_fit(smc_problem p, int64_t N, const double* xi, int32_t M, int32_t iters, double var_floor,
                          uint64_t seed, uint64_t ctr, double* logw, double* mean, double* scale, int32_t* centers,
                          smc_stream stream) {
    if (!p) return fail(SMC_E_INVAL, "problem is NULL");
    const Problem& P = p->P;
    if (int r = check_n(P, N)) return r;
    if (N < 1) return fail(SMC_E_INVAL, "the fit needs at least one particle");
    if (N > (1ll << 24)) return fail(SMC_E_INVAL, "the fit takes at most 2^24 particles");
    if (M < 1 || M > MAX_M) return fail(SMC_E_INVAL, "M must be 1..%d", MAX_M);
    if (iters < 0 || iters > 100000) return fail(SMC_E_INVAL, "iters must be 0..100000");
    if (!(var_floor > 0.0) || !std::isfinite(var_floor)) return fail(SMC_E_INVAL, "var_floor must be positive");
    if (!xi || !logw || !mean || !scale) return fail(SMC_E_INVAL, "xi, logw, mean and scale must not be NULL");
    FitWorkspace w{P.ws_fit_d2, P.ws_fit_par, P.ws_fit_part};
    HIPCHK(launch_gm_fit(N, P.K, P.kr, P.active, xi, M, iters, var_floor, seed, ctr, w,
                         centers ? centers : P.ws_fit_centers, logw, mean, scale, (hipStream_t)stream));
    return SMC_OK;
}

extern "C" int smc_gmpcn_propose(smc_problem p, int64_t N, const smc_gm* gm, double beta, uint64_t seed, uint64_t ctr,
                                 const double* xi, double* v, double* logr, smc_stream stream) {
    if (!p) return fail(SMC_E_INVAL, "problem is NULL");
    const Problem& P = p->P;
    if (int r = check_gm(P, gm)) return r;
    if (!(beta > 0.0 && beta <= 1.0)) return fail(SMC_E_INVAL, "beta must be in (0, 1]");
    if (int r = check_n(P, N)) return r;
    if (N > 0 && (!xi || !v || !logr)) return fail(SMC_E_INVAL, "xi, v and logr must not be NULL");
    if (xi == v) return fail(SMC_E_INVAL, "v must not alias xi");
    if (N > 0xFFFFFFFFll) return fail(SMC_E_INVAL, "N exceeds the 32-bit particle counter");
    if (N == 0) return SMC_OK;
    MoveParams q;
    q.beta = beta;
    q.tau = 0.0;
    q.seed = seed;
    q.ctr = ctr;
    q.M = gm->M;
    q.kr = gm->kr;
    q.logw = gm->logw;
    q.mean = gm->mean;
    q.scale = gm->scale;
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(launch_mixtab(q, P.ws_mixtab, s));
    HIPCHK(launch_propose(N, P.K, P.active, P.slot, q, P.ws_mixtab, xi, v, logr, P.flags, s));
    return SMC_OK;
}

extern "C" int64_t smc_gm_fit_noalloc_max(void) { return STATIC_FIT_N; }

extern "C" int smc_gm_fit_noalloc(int64_t N, int32_t K, int32_t kr, const int32_t* active, const double* xi, int32_t M,
                                  int32_t iters, double var_floor, uint64_t seed, uint64_t ctr, double* logw,
                                  double* mean, double* scale, int32_t* centers, smc_stream stream) {
    if (N < 1 || N > STATIC_FIT_N)
        return fail(SMC_E_INVAL, "N = %lld outside 1..%lld (the static workspace's size)", (long long)N,
                    (long long)STATIC_FIT_N);
    if (K < 1 || K > 1024) return fail(SMC_E_INVAL, "K must be 1..1024");
    if (kr < 1 || kr > MAX_KR || kr > K) return fail(SMC_E_INVAL, "kr must be 1..min(64, K)");
    if (M < 1 || M > MAX_M) return fail(SMC_E_INVAL, "M must be 1..%d", MAX_M);
    if (iters < 0 || iters > 100000) return fail(SMC_E_INVAL, "iters must be 0..100000");
    if (!(var_floor > 0.0) || !std::isfinite(var_floor)) return fail(SMC_E_INVAL, "var_floor must be positive");
    if (!active || !xi || !logw || !mean || !scale)
        return fail(SMC_E_INVAL, "active, xi, logw, mean and scale must not be NULL");
    HIPCHK(launch_gm_fit_static(N, K, kr, active, xi, M, iters, var_floor, seed, ctr, centers, logw, mean, scale,
                                (hipStream_t)stream));
    return SMC_OK;
}

extern "C" int smc_gmpcn_move(smc_problem p, int64_t N, const smc_gm* gm, double beta, double tau,
                              int32_t n_moves, uint64_t seed, uint64_t ctr, const int32_t* level, int32_t prec,
                              double* xi, double* phi, int32_t* n_acc, smc_stream stream) {
    if (!p) return fail(SMC_E_INVAL, "problem is NULL");
    const Problem& P = p->P;
    if (int r = check_gm(P, gm)) return r;
    if (!(beta > 0.0 && beta <= 1.0)) return fail(SMC_E_INVAL, "beta must be in (0, 1]");
    if (!(tau >= 0.0 && tau <= 1.0)) return fail(SMC_E_INVAL, "tau must be in [0, 1]");
    if (int r = check_move_common(P, N, n_moves, level, prec, xi, phi, n_acc)) return r;
    MoveParams q;
    q.beta = beta;
    q.tau = tau;
    q.seed = seed;
    q.ctr = ctr;
    q.M = gm->M;
    q.kr = gm->kr;
    q.logw = gm->logw;
    q.mean = gm->mean;
    q.scale = gm->scale;
    return move_loop(p, N, q, n_moves, level, prec, xi, phi, n_acc, (hipStream_t)stream);
}

static int stage_params(const Problem& P, const smc_stage* st, const int32_t* level, MoveParams& q) {
    if (!st) return fail(SMC_E_INVAL, "stage is NULL");
    const int G = level ? P.n_levels : 1;
    if (st->n_groups != G)
        return fail(SMC_E_INVAL, "n_groups (%d) must be %d (%s)", st->n_groups, G,
                    level ? "the problem's grid count with a level map" : "1 without a level map");
    if (st->M < 1 || st->M > MAX_M) return fail(SMC_E_INVAL, "M must be 1..%d", MAX_M);
    if (st->kr != P.kr) return fail(SMC_E_INVAL, "kr (%d) differs from the problem's kr (%d)", st->kr, P.kr);
    if (!st->logw || !st->mean || !st->scale || !st->beta || !st->tau || !st->ctr)
        return fail(SMC_E_INVAL, "stage arrays must not be NULL");
    q = MoveParams{};
    q.seed = st->seed;
    q.group = level;
    q.beta_g = st->beta;
    q.tau_g = st->tau;
    q.ctr_dev = st->ctr;
    q.n_groups = G;
    q.M = st->M;
    q.kr = st->kr;
    q.logw = st->logw;
    q.mean = st->mean;
    q.scale = st->scale;
    return SMC_OK;
}

extern "C" int smc_gmpcn_stage(smc_problem p, int64_t N, const int32_t* level, const smc_stage* st, int32_t n_moves,
                               int32_t prec, double* xi, double* phi, int32_t* n_acc, smc_stream stream) {
    if (!p) return fail(SMC_E_INVAL, "problem is NULL");
    MoveParams q;
    if (int r = stage_params(p->P, st, level, q)) return r;
    if (int r = check_move_common(p->P, N, n_moves, level, prec, xi, phi, n_acc)) return r;
    return move_loop(p, N, q, n_moves, level, prec, xi, phi, n_acc, (hipStream_t)stream);
}

extern "C" int smc_stage_graph_create(smc_problem p, int64_t N, const int32_t* level, const smc_stage* st,
                                      int32_t n_moves, int32_t prec, double* xi, double* phi, int32_t* n_acc,
                                      smc_stream stream, smc_graph* out) {
    if (!p || !out) return fail(SMC_E_INVAL, "problem and out must not be NULL");
    if (!stream) return fail(SMC_E_INVAL, "graph capture needs a created stream, not the null stream");
    MoveParams q;
    if (int r = stage_params(p->P, st, level, q)) return r;
    if (int r = check_move_common(p->P, N, n_moves, level, prec, xi, phi, n_acc)) return r;
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    p->capturing = true;
    const int r = move_loop(p, N, q, n_moves, level, prec, xi, phi, n_acc, s);
    p->capturing = false;
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(s, &g);
    if (r != SMC_OK) {
        if (g) (void)hipGraphDestroy(g);
        return r;
    }
    if (ec != hipSuccess) return fail(SMC_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(ec));
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(SMC_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ei));
    }
    smc_graph_s* gr = new smc_graph_s();
    gr->graph = g;
    gr->exec = ex;
    *out = gr;
    return SMC_OK;
}

extern "C" int smc_stage_graph_launch(smc_graph g, smc_stream stream) {
    if (!g) return fail(SMC_E_INVAL, "graph is NULL");
    HIPCHK(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return SMC_OK;
}

extern "C" void smc_stage_graph_destroy(smc_graph g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

// The launches of one whole tempering stage (arguments already checked), in the order the
// samplers make the same calls one by one.
static int sampler_stage(smc_problem_s* p, const smc_sampler_graph_desc* d, int32_t prec, const int64_t* off,
                         int64_t N, hipStream_t s) {
    const Problem& P = p->P;
    const int G = d->n_groups, K = P.K, M = d->M, kr = d->kr;
    const uint64_t* ctr = d->ctr;
    for (int g = 0; g < G; ++g) {
        const int64_t o = off[g], n = d->counts[g];
        HIPCHK(launch_temper(n, d->phi + o, d->tau + g, d->ess_frac, d->h + g, d->tau_new + g, d->W + o,
                             d->log_z + g, d->flags, s));
        HIPCHK(launch_resample_ctr(n, d->W + o, d->seed, ctr, (uint64_t)g, d->idx + o, d->flags, s));
        HIPCHK(launch_gather(n, K, d->idx + o, d->xi + o * K, d->phi + o, d->xi2 + o * K, d->phi2 + o, s));
        HIPCHK(hipMemcpyAsync(d->xi + o * K, d->xi2 + o * K, sizeof(double) * n * K, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(d->phi + o, d->phi2 + o, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(d->tau + g, d->tau_new + g, sizeof(double), hipMemcpyDeviceToDevice, s));
        if (M > 1) {
            FitWorkspace w{P.ws_fit_d2, P.ws_fit_par, P.ws_fit_part};
            HIPCHK(launch_gm_fit_ctr(n, K, kr, P.active, d->xi + o * K, M, d->fit_iters, d->var_floor, d->seed, ctr,
                                     (uint64_t)g, w, P.ws_fit_centers, d->logw + (int64_t)g * M,
                                     d->mean + (int64_t)g * M * kr, d->scale + (int64_t)g * M * kr, s));
        }
    }
    smc_stage st{};
    st.n_groups = G;
    st.M = M;
    st.kr = kr;
    st.logw = d->logw;
    st.mean = d->mean;
    st.scale = d->scale;
    st.beta = d->beta;
    st.tau = d->tau;
    st.ctr = ctr;
    st.seed = d->seed;
    MoveParams q;
    if (int r = stage_params(P, &st, d->level, q)) return r;
    if (int r = move_loop(p, N, q, d->n_moves, d->level, prec, d->xi, d->phi, d->n_acc, s)) return r;
    StageRule rule;
    rule.G = G;
    for (int g = 0; g < G; ++g) {
        rule.off[g] = off[g];
        rule.count[g] = d->counts[g];
    }
    rule.n_moves = d->n_moves;
    rule.n_acc = d->n_acc;
    rule.tau = d->tau;
    rule.h = d->h;
    rule.log_z = d->log_z;
    rule.beta = d->beta;
    rule.level = d->level;
    rule.ctr = d->ctr;
    rule.stride = d->stride;
    rule.record = d->record;
    rule.max_stages = d->max_stages;
    HIPCHK(launch_stage_rule(rule, s));
    return SMC_OK;
}

extern "C" int smc_sampler_graph_create(smc_problem p, const smc_sampler_graph_desc* d, int32_t prec,
                                        smc_stream stream, smc_graph* out) {
    if (!p || !d || !out) return fail(SMC_E_INVAL, "problem, desc and out must not be NULL");
    if (!stream) return fail(SMC_E_INVAL, "graph capture needs a created stream, not the null stream");
    const Problem& P = p->P;
    const int G = d->n_groups;
    if (G != (d->level ? P.n_levels : 1))
        return fail(SMC_E_INVAL, "n_groups (%d) must be %d (%s)", G, d->level ? P.n_levels : 1,
                    d->level ? "the problem's grid count with a level map" : "1 without a level map");
    int64_t off[MAX_LEVELS] = {}, N = 0;
    for (int g = 0; g < G; ++g) {
        if (d->counts[g] < 1 || d->counts[g] > (1 << 20))
            return fail(SMC_E_INVAL, "counts[%d] must be 1..2^20 (the tempering step's batch)", g);
        off[g] = N;
        N += d->counts[g];
    }
    if (int r = check_n(P, N)) return r;
    if (N > (1ll << 24)) return fail(SMC_E_INVAL, "at most 2^24 particles");
    if (d->M < 1 || d->M > MAX_M) return fail(SMC_E_INVAL, "M must be 1..%d", MAX_M);
    if (d->kr != P.kr) return fail(SMC_E_INVAL, "kr (%d) differs from the problem's kr (%d)", d->kr, P.kr);
    if (d->M > 1 && (d->fit_iters < 0 || d->fit_iters > 100000))
        return fail(SMC_E_INVAL, "fit_iters must be 0..100000");
    if (d->M > 1 && (!(d->var_floor > 0.0) || !std::isfinite(d->var_floor)))
        return fail(SMC_E_INVAL, "var_floor must be positive");
    if (!(d->ess_frac > 0.0 && d->ess_frac <= 1.0)) return fail(SMC_E_INVAL, "ess_frac must be in (0, 1]");
    if (d->stride < 1 || d->max_stages < 0) return fail(SMC_E_INVAL, "stride must be >= 1 and max_stages >= 0");
    if (!d->xi || !d->phi || !d->xi2 || !d->phi2 || !d->W || !d->idx || !d->tau || !d->tau_new || !d->h ||
        !d->log_z || !d->beta || !d->logw || !d->mean || !d->scale || !d->ctr || !d->n_acc ||
        (d->max_stages > 0 && !d->record))
        return fail(SMC_E_INVAL, "device arrays must not be NULL (level and flags may be)");
    if (d->xi == d->xi2 || d->phi == d->phi2) return fail(SMC_E_INVAL, "the gather scratch must not alias xi or phi");
    if (int r = check_move_common(P, N, d->n_moves, d->level, prec, d->xi, d->phi, d->n_acc)) return r;
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    p->capturing = true;
    const int r = sampler_stage(p, d, prec, off, N, s);
    p->capturing = false;
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(s, &g);
    if (r != SMC_OK) {
        if (g) (void)hipGraphDestroy(g);
        return r;
    }
    if (ec != hipSuccess) return fail(SMC_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(ec));
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(SMC_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ei));
    }
    smc_graph_s* gr = new smc_graph_s();
    gr->graph = g;
    gr->exec = ex;
    *out = gr;
    return SMC_OK;
}

extern "C" int smc_pcnl_move(smc_problem p, int64_t N, double beta, double tau, int32_t n_moves, uint64_t seed,
                             uint64_t ctr, int32_t prec, double* xi, double* phi, double* grad, int32_t* n_acc,
                             smc_stream stream) {
    if (!p) return fail(SMC_E_INVAL, "problem is NULL");
    const Problem& P = p->P;
    if (P.dim != 2) return fail(SMC_E_INVAL, "the pCN-Langevin move needs the 2D adjoint gradient");
    if (int r = check_n(P, N)) return r;
    if (!(beta > 0.0 && beta <= 1.0)) return fail(SMC_E_INVAL, "beta must be in (0, 1]");
    if (!(tau >= 0.0 && tau <= 1.0)) return fail(SMC_E_INVAL, "tau must be in [0, 1]");
    if (n_moves < 0) return fail(SMC_E_INVAL, "n_moves must be >= 0");
    if (prec != SMC_FP64 && prec != SMC_FP32_REFINE) return fail(SMC_E_INVAL, "unknown precision %d", prec);
    if (N > 0 && (!xi || !phi || !grad || !n_acc)) return fail(SMC_E_INVAL, "xi, phi, grad and n_acc must not be NULL");
    if (N > 0xFFFFFFFFll) return fail(SMC_E_INVAL, "N exceeds the 32-bit particle counter");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(launch_fill_i32(n_acc, N, 0, s));
    for (int m = 0; m < n_moves; ++m) {
        const uint64_t c = ctr + (uint64_t)m;
        HIPCHK(launch_pcnl_propose(N, P.K, beta, tau, seed, c, xi, grad, P.ws_v, s));
        Solve o;
        o.phi = P.ws_phinew;
        o.iters = P.ws_iters;
        o.adjoint = true;
        HIPCHK(forward(p, 0, prec, N, P.ws_v, o, s));
        HIPCHK(gradient(P, 0, prec, N, P.ws_x64, P.x_stride, P.ws_iters, P.ws_gnew, s));
        HIPCHK(launch_pcnl_accept(N, P.K, beta, tau, seed, c, P.ws_v, P.ws_gnew, P.ws_phinew, P.ws_iters, xi, grad,
                                  phi, n_acc, s));
    }
    return SMC_OK;
}

// ------------------------------------------------------------------ tile choice and autotuning
extern "C" int smc_tile_candidates(int32_t n, int32_t* rows, int32_t* count) {
    if (!rows || !count) return fail(SMC_E_INVAL, "rows and count must not be NULL");
    int r[8];
    const int c = tile_candidates(n, r);
    if (c == 0) return fail(SMC_E_INVAL, "grid %d has no fast-Poisson solver", n);
    std::copy(r, r + c, rows);
    *count = c;
    return SMC_OK;
}

static int check_tile(const Problem& P, int32_t level, int32_t rows) {
    if (level < 0 || level >= P.n_levels) return fail(SMC_E_INVAL, "level %d out of range", level);
    if (P.dim != 2 || !P.lv[level].dst_S) return fail(SMC_E_INVAL, "grid %d has no fast-Poisson solver", P.lv[level].n);
    if (rows == 0) return SMC_OK;
    int r[8];
    const int c = tile_candidates(P.lv[level].n, r);
    for (int k = 0; k < c; ++k)
        if (r[k] == rows) return SMC_OK;
    return fail(SMC_E_INVAL, "grid %d has no tile of %d rows per thread", P.lv[level].n, rows);
}

extern "C" int smc_set_tile(smc_problem p, int32_t level, int32_t rows) {
    if (!p) return fail(SMC_E_INVAL, "problem is NULL");
    if (int r = check_tile(p->P, level, rows)) return r;
    p->P.lv[level].rows = rows;
    return SMC_OK;
}

extern "C" int smc_set_stage_fusion(smc_problem p, int32_t enable) {
    if (!p) return fail(SMC_E_INVAL, "problem is NULL");
    p->fuse_stage = enable != 0;
    return SMC_OK;
}

extern "C" int smc_get_tile(smc_problem p, int32_t level, int32_t* rows) {
    if (!p || !rows) return fail(SMC_E_INVAL, "problem and rows must not be NULL");
    if (int r = check_tile(p->P, level, 0)) return r;
    int c[8];
    tile_candidates(p->P.lv[level].n, c);
    *rows = p->P.lv[level].rows ? p->P.lv[level].rows : c[0];
    return SMC_OK;
}

extern "C" int smc_autotune(smc_problem p, int32_t level, int64_t N, int32_t reps, smc_stream stream, int32_t* rows,
                            double* ms) {
    if (!p) return fail(SMC_E_INVAL, "problem is NULL");
    Problem& P = p->P;
    if (int r = check_tile(P, level, 0)) return r;
    if (N < 1 || N > P.n_max) return fail(SMC_E_INVAL, "N must be 1..n_max");
    if (reps < 1 || reps > 100) return fail(SMC_E_INVAL, "reps must be 1..100");
    if (N > 0xFFFFFFFFll) return fail(SMC_E_INVAL, "N exceeds the 32-bit particle counter");
    hipStream_t s = (hipStream_t)stream;
    int cand[8];
    const int nc = tile_candidates(P.lv[level].n, cand);
    const int saved = P.lv[level].rows;
    const bool prof = P.profiling;
    P.profiling = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        P.profiling = prof;
    };
    auto run = [&](hipError_t e) -> bool {
        if (e == hipSuccess) return true;
        P.lv[level].rows = saved;
        cleanup();
        fail(SMC_E_HIP, "autotune: %s", hipGetErrorString(e));
        return false;
    };
    if (!run(hipEventCreate(&e0)) || !run(hipEventCreate(&e1))) return SMC_E_HIP;
    // synthetic particles: prior draws of the library's own generator, in the proposal workspace
    if (!run(launch_prior(N, P.K, 0x5EED, 0, P.ws_v, s))) return SMC_E_HIP;
    int best = cand[0];
    double best_ms = INFINITY;
    for (int k = 0; k < nc; ++k) {
        P.lv[level].rows = cand[k];
        Solve o;
        o.phi = P.ws_phinew;
        o.iters = P.ws_iters;
        if (!run(forward(p, level, SMC_FP32_REFINE, N, P.ws_v, o, s))) return SMC_E_HIP;   // warm-up
        if (!run(hipEventRecord(e0, s))) return SMC_E_HIP;
        for (int r = 0; r < reps; ++r)
            if (!run(forward(p, level, SMC_FP32_REFINE, N, P.ws_v, o, s))) return SMC_E_HIP;
        if (!run(hipEventRecord(e1, s)) || !run(hipEventSynchronize(e1))) return SMC_E_HIP;
        float t = 0.0f;
        if (!run(hipEventElapsedTime(&t, e0, e1))) return SMC_E_HIP;
        const double per = (double)t / reps;
        if (ms) ms[k] = per;
        if (per < best_ms) {
            best_ms = per;
            best = cand[k];
        }
    }
    P.lv[level].rows = best;
    if (rows) *rows = best;
    cleanup();
    return SMC_OK;
}

extern "C" int smc_precond_apply(smc_problem p, int32_t level, int64_t N, const float* r, float* z,
                                 smc_stream stream) {
    if (!p) return fail(SMC_E_INVAL, "problem is NULL");
    if (int rc = check_n(p->P, N)) return rc;
    if (level < 0 || level >= p->P.n_levels) return fail(SMC_E_INVAL, "level %d out of range", level);
    const Level& L = p->P.lv[level];
    if (!L.dst_S) return fail(SMC_E_INVAL, "grid %d has no fast-Poisson preconditioner", L.n);
    if (N > 0 && (!r || !z)) return fail(SMC_E_INVAL, "r and z must not be NULL");
    HIPCHK(launch_dst_apply(L.n, N, r, z, L.dst_S, L.dst_lam, (hipStream_t)stream));
    return SMC_OK;
}

extern "C" int smc_temper(int64_t N, const double* phi, const double* tau_in, double ess_frac, double* h,
                          double* tau_new, double* W, double* log_z_inc, int32_t* flags, smc_stream stream) {
    if (N < 1 || N > (1 << 20)) return fail(SMC_E_INVAL, "N must be 1..2^20");
    if (!phi || !tau_in || !h || !tau_new || !W || !log_z_inc)
        return fail(SMC_E_INVAL, "temper arrays must not be NULL");
    if (!(ess_frac > 0.0 && ess_frac < 1.0)) return fail(SMC_E_INVAL, "ess_frac must be in (0, 1)");
    HIPCHK(launch_temper(N, phi, tau_in, ess_frac, h, tau_new, W, log_z_inc, flags, (hipStream_t)stream));
    return SMC_OK;
}

extern "C" int smc_resample(int64_t N, const double* W, uint64_t u53, int32_t* idx, int32_t* flags,
                            smc_stream stream) {
    if (N < 1 || N > (1ll << 24)) return fail(SMC_E_INVAL, "N must be 1..2^24");
    if (!W || !idx) return fail(SMC_E_INVAL, "W and idx must not be NULL");
    if (u53 >= (1ull << 53)) return fail(SMC_E_INVAL, "u53 must be below 2^53");
    HIPCHK(launch_resample(N, W, u53, idx, flags, (hipStream_t)stream));
    return SMC_OK;
}

extern "C" int smc_gather(int64_t N, int32_t K, const int32_t* idx, const double* xi_in, const double* phi_in,
                          double* xi_out, double* phi_out, smc_stream stream) {
    if (N < 0 || K < 1) return fail(SMC_E_INVAL, "N must be >= 0 and K >= 1");
    if (N > 0 && (!idx || !xi_in || !xi_out)) return fail(SMC_E_INVAL, "idx, xi_in and xi_out must not be NULL");
    if (xi_in == xi_out || (phi_in && phi_in == phi_out)) return fail(SMC_E_INVAL, "outputs must not alias inputs");
    HIPCHK(launch_gather(N, K, idx, xi_in, phi_in, xi_out, phi_out, (hipStream_t)stream));
    return SMC_OK;
}
