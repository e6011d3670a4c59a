"""Python binding of libsmc: the C ABI of include/smc.h under the same names.

Argument marshalling only: every function checks that its tensors are contiguous device
tensors of the right dtype and size, passes their addresses and the current HIP stream to
the library, and raises SMCError on a non-OK status.  All computation runs in the library's
kernels; there is no fallback when the library is missing.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libsmc.so")

SMC_OK = 0
SMC_E_INVAL, SMC_E_HIP, SMC_E_NOCONV, SMC_E_STALL, SMC_E_NONFINITE, SMC_E_NOMEM = -1, -2, -3, -4, -5, -6
SMC_FP64 = 0
SMC_FP32_REFINE = 1
FLAG_NOCONV, FLAG_STALL, FLAG_NONFINITE, FLAG_BADWEIGHTS, FLAG_BADLEVEL, FLAG_BADPARAM = 1, 2, 4, 8, 16, 32
LEVEL_PARKED = -1
PRECISIONS = {"fp64": SMC_FP64, "fp32_refine": SMC_FP32_REFINE}
PRECOND_AUTO, PRECOND_JACOBI = 0, 1

c_i32, c_i64, c_u64, c_dbl, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p


class SMCError(RuntimeError):
    def __init__(self, status, text):
        super().__init__("libsmc status %d: %s" % (status, text))
        self.status = status


class ProblemDesc(ctypes.Structure):
    _fields_ = [("dim", c_i32), ("n_levels", c_i32), ("grid_n", c_i32 * 3), ("kl", c_i32), ("kr", c_i32),
                ("n_obs", c_i32), ("obs_den", c_i32), ("obs_num", ctypes.POINTER(c_i32)),
                ("y", ctypes.POINTER(c_dbl)), ("sigma", c_dbl), ("f", c_dbl), ("n_max", c_i64),
                ("tol64", c_dbl), ("tol_inner", c_dbl), ("max_iter", c_i32), ("max_sweeps", c_i32),
                ("precond", c_i32)]


class GMDesc(ctypes.Structure):
    _fields_ = [("M", c_i32), ("kr", c_i32), ("logw", c_vp), ("mean", c_vp), ("scale", c_vp)]


class L2MixDesc(ctypes.Structure):
    _fields_ = [("K", c_i32), ("kr", c_i32), ("alpha", c_dbl), ("n_terms", c_i32), ("c", ctypes.POINTER(c_dbl)),
                ("sigma", c_dbl), ("n_max", c_i64)]


class StageDesc(ctypes.Structure):
    _fields_ = [("n_groups", c_i32), ("M", c_i32), ("kr", c_i32), ("logw", c_vp), ("mean", c_vp), ("scale", c_vp),
                ("beta", c_vp), ("tau", c_vp), ("ctr", c_vp), ("seed", c_u64)]


class SamplerGraphDesc(ctypes.Structure):
    _fields_ = [("n_groups", c_i32), ("counts", c_i64 * 4), ("M", c_i32), ("kr", c_i32), ("fit_iters", c_i32),
                ("n_moves", c_i32), ("max_stages", c_i32), ("ess_frac", c_dbl), ("var_floor", c_dbl),
                ("seed", c_u64), ("stride", c_u64),
                ("xi", c_vp), ("phi", c_vp), ("xi2", c_vp), ("phi2", c_vp), ("W", c_vp), ("idx", c_vp),
                ("tau", c_vp), ("tau_new", c_vp), ("h", c_vp), ("log_z", c_vp), ("beta", c_vp),
                ("logw", c_vp), ("mean", c_vp), ("scale", c_vp), ("ctr", c_vp), ("level", c_vp), ("n_acc", c_vp),
                ("record", c_vp), ("flags", c_vp)]


_SIGS = {
    "smc_problem_create": (c_i32, [ctypes.POINTER(ProblemDesc), ctypes.POINTER(c_vp)]),
    "smc_problem_create_l2mix": (c_i32, [ctypes.POINTER(L2MixDesc), ctypes.POINTER(c_vp)]),
    "smc_problem_destroy": (None, [c_vp]),
    "smc_phi_batch": (c_i32, [c_vp, c_i64, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp]),
    "smc_last_error": (ctypes.c_char_p, []),
    "smc_philox_u53": (c_u64, [c_u64, c_u64, ctypes.c_uint32, ctypes.c_uint32]),
    "smc_problem_info": (c_i32, [c_vp, ctypes.POINTER(c_i32), ctypes.POINTER(c_i32), ctypes.POINTER(c_i32)]),
    "smc_status_flags": (c_i32, [c_vp, c_vp, ctypes.POINTER(c_i32), c_i32]),
    "smc_prior_sample": (c_i32, [c_vp, c_i64, c_u64, c_u64, c_vp, c_vp]),
    "smc_synthesize": (c_i32, [c_vp, c_i64, c_vp, c_i32, c_vp, c_vp]),
    "smc_forward_batch": (c_i32, [c_vp, c_i64, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp]),
    "smc_potential": (c_i32, [c_vp, c_i64, c_vp, c_vp, c_vp]),
    "smc_gmpcn_move": (c_i32, [c_vp, c_i64, ctypes.POINTER(GMDesc), c_dbl, c_dbl, c_i32, c_u64, c_u64, c_vp, c_i32,
                               c_vp, c_vp, c_vp, c_vp]),
    "smc_gmpcn_propose": (c_i32, [c_vp, c_i64, ctypes.POINTER(GMDesc), c_dbl, c_u64, c_u64, c_vp, c_vp, c_vp, c_vp]),
    "smc_gm_draw": (c_i32, [c_vp, c_i64, ctypes.POINTER(GMDesc), c_u64, c_u64, c_vp, c_i32, c_vp, c_vp, c_vp, c_vp]),
    "smc_gm_fit": (c_i32, [c_vp, c_i64, c_vp, c_i32, c_i32, c_dbl, c_u64, c_u64, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "smc_gm_fit_noalloc": (c_i32, [c_i64, c_i32, c_i32, c_vp, c_vp, c_i32, c_i32, c_dbl, c_u64, c_u64, c_vp, c_vp,
                                   c_vp, c_vp, c_vp]),
    "smc_gm_fit_noalloc_max": (c_i64, []),
    "smc_forward_state": (c_i32, [c_vp, c_i64, c_vp, c_i32, c_vp, c_vp, c_vp, c_vp]),
    "smc_value_and_grad": (c_i32, [c_vp, c_i64, c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "smc_pcnl_move": (c_i32, [c_vp, c_i64, c_dbl, c_dbl, c_i32, c_u64, c_u64, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "smc_gmpcn_stage": (c_i32, [c_vp, c_i64, c_vp, ctypes.POINTER(StageDesc), c_i32, c_i32, c_vp, c_vp, c_vp, c_vp]),
    "smc_stage_graph_create": (c_i32, [c_vp, c_i64, c_vp, ctypes.POINTER(StageDesc), c_i32, c_i32, c_vp, c_vp, c_vp,
                                       c_vp, ctypes.POINTER(c_vp)]),
    "smc_sampler_graph_create": (c_i32, [c_vp, ctypes.POINTER(SamplerGraphDesc), c_i32, c_vp, ctypes.POINTER(c_vp)]),
    "smc_stage_graph_launch": (c_i32, [c_vp, c_vp]),
    "smc_stage_graph_destroy": (None, [c_vp]),
    "smc_tile_candidates": (c_i32, [c_i32, ctypes.POINTER(c_i32), ctypes.POINTER(c_i32)]),
    "smc_set_tile": (c_i32, [c_vp, c_i32, c_i32]),
    "smc_set_stage_fusion": (c_i32, [c_vp, c_i32]),
    "smc_get_tile": (c_i32, [c_vp, c_i32, ctypes.POINTER(c_i32)]),
    "smc_autotune": (c_i32, [c_vp, c_i32, c_i64, c_i32, c_vp, ctypes.POINTER(c_i32), ctypes.POINTER(c_dbl)]),
    "smc_temper": (c_i32, [c_i64, c_vp, c_vp, c_dbl, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "smc_resample": (c_i32, [c_i64, c_vp, c_u64, c_vp, c_vp, c_vp]),
    "smc_gather": (c_i32, [c_i64, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "smc_precond_apply": (c_i32, [c_vp, c_i32, c_i64, c_vp, c_vp, c_vp]),
    "smc_profile": (c_i32, [c_vp, c_i32]),
    "smc_profile_read": (c_i32, [c_vp, c_vp, ctypes.POINTER(c_dbl), ctypes.POINTER(c_i64), ctypes.POINTER(c_i64),
                                 ctypes.POINTER(c_i64), ctypes.POINTER(c_i64), ctypes.POINTER(c_i64)]),
}
EXPORTED = sorted(_SIGS)

_lib = None


def lib():
    """Load libsmc.so (built in-tree); raise if it is not there."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsmc.so is not built (python -m paper_2503_16028_amd.build)")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def _check(status):
    if status != SMC_OK:
        raise SMCError(status, lib().smc_last_error().decode())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return c_vp(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _ptr(t, dtype, numel=None, name="tensor", optional=False):
    if t is None:
        if optional:
            return None
        raise ValueError("%s is required" % name)
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a device tensor" % name)
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError("%s must be a contiguous %s tensor" % (name, dtype))
    if numel is not None and t.numel() < numel:
        raise ValueError("%s has %d elements, needs %d" % (name, t.numel(), numel))
    return c_vp(t.data_ptr())


class Problem:
    """An smc_problem built from a problem definition (dict with the JSON fields)."""

    def __init__(self, d, n_max, grids=None, tol64=1e-10, tol_inner=1e-3, max_iter=None, max_sweeps=8,
                 precond=PRECOND_AUTO):
        L = lib()
        grids = list(grids if grids is not None else d["grids"])
        self.dim = int(d["dim"])
        self.grids = grids
        obs = [int(v) for o in d["obs"] for v in o]
        self._obs = (c_i32 * len(obs))(*obs)
        self._y = (c_dbl * len(d["y"]))(*[float(v) for v in d["y"]])
        desc = ProblemDesc()
        desc.dim = self.dim
        desc.n_levels = len(grids)
        for k, n in enumerate(grids):
            desc.grid_n[k] = int(n)
        desc.kl = int(d["kl_per_axis"])
        desc.kr = int(d.get("kr", 1))
        desc.n_obs = len(d["obs"])
        desc.obs_den = int(d["obs_den"])
        desc.obs_num = self._obs
        desc.y = self._y
        desc.sigma = float(d["sigma"])
        desc.f = float(d.get("f", 1.0))
        desc.n_max = int(n_max)
        desc.tol64 = float(tol64)
        desc.tol_inner = float(tol_inner)
        desc.max_iter = int(max_iter if max_iter is not None else 40 * max(grids))
        desc.max_sweeps = int(max_sweeps)
        desc.precond = int(precond)
        handle = c_vp()
        _check(L.smc_problem_create(ctypes.byref(desc), ctypes.byref(handle)))
        self.handle = handle
        self.n_max = int(n_max)
        self._info(desc.kr)

    def _info(self, kr):
        K, n_obs = c_i32(), c_i32()
        act = (c_i32 * 64)()
        _check(lib().smc_problem_info(self.handle, ctypes.byref(K), act, ctypes.byref(n_obs)))
        self.K, self.n_obs, self.kr = K.value, n_obs.value, kr
        self.active = [act[k] for k in range(self.kr)]

    def close(self):
        if getattr(self, "handle", None):
            lib().smc_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class L2MixProblem(Problem):
    """An smc_problem of the L^2 mixture kind (no PDE): c is [n_terms][K] (numpy or list)."""

    def __init__(self, K, kr, alpha, c, sigma, n_max):
        import numpy as np
        c = np.ascontiguousarray(np.asarray(c, dtype=np.float64).reshape(-1, int(K)))
        self._c = (c_dbl * c.size)(*c.ravel().tolist())
        desc = L2MixDesc()
        desc.K, desc.kr, desc.alpha = int(K), int(kr), float(alpha)
        desc.n_terms, desc.c, desc.sigma, desc.n_max = c.shape[0], self._c, float(sigma), int(n_max)
        handle = c_vp()
        _check(lib().smc_problem_create_l2mix(ctypes.byref(desc), ctypes.byref(handle)))
        self.handle = handle
        self.dim, self.grids, self.n_max = 1, [], int(n_max)
        self._info(int(kr))


RESAMPLE_BLOCK = 0x80000001


def smc_philox_u53(seed, ctr, block=RESAMPLE_BLOCK, word=0):
    """53-bit integer uniform of the library's generator (host arithmetic)."""
    return int(lib().smc_philox_u53(int(seed), int(ctr), int(block), int(word)))


def smc_status_flags(problem, stream=None, clear=True):
    out = c_i32()
    _check(lib().smc_status_flags(problem.handle, _stream(stream), ctypes.byref(out), int(bool(clear))))
    return out.value


def smc_prior_sample(problem, N, seed, ctr, xi, stream=None):
    _check(lib().smc_prior_sample(problem.handle, N, seed, ctr, _ptr(xi, torch.float64, N * problem.K, "xi"),
                                  _stream(stream)))


def smc_synthesize(problem, N, xi, level, u, stream=None):
    n = problem.grids[level]
    per = (n + 1) ** problem.dim
    _check(lib().smc_synthesize(problem.handle, N, _ptr(xi, torch.float64, N * problem.K, "xi"), level,
                                _ptr(u, torch.float64, N * per, "u"), _stream(stream)))


def smc_forward_batch(problem, N, xi, level, prec, G, iters=None, stream=None):
    _check(lib().smc_forward_batch(problem.handle, N, _ptr(xi, torch.float64, N * problem.K, "xi"),
                                   _ptr(level, torch.int32, N, "level", optional=True), prec,
                                   _ptr(G, torch.float64, N * problem.n_obs, "G"),
                                   _ptr(iters, torch.int32, N, "iters", optional=True), _stream(stream)))


def smc_phi_batch(problem, N, xi, level, prec, phi, iters=None, stream=None):
    """Potential of each particle (forward map and Phi, or the closed form of an L^2 mixture)."""
    _check(lib().smc_phi_batch(problem.handle, N, _ptr(xi, torch.float64, N * problem.K, "xi"),
                               _ptr(level, torch.int32, N, "level", optional=True), prec,
                               _ptr(phi, torch.float64, N, "phi"), _ptr(iters, torch.int32, N, "iters", optional=True),
                               _stream(stream)))


def smc_potential(problem, N, G, phi, stream=None):
    _check(lib().smc_potential(problem.handle, N, _ptr(G, torch.float64, N * problem.n_obs, "G"),
                               _ptr(phi, torch.float64, N, "phi"), _stream(stream)))


def gm_desc(logw, mean, scale):
    M = logw.numel()
    kr = mean.shape[-1]
    d = GMDesc()
    d.M, d.kr = M, kr
    d.logw = _ptr(logw, torch.float64, M, "logw")
    d.mean = _ptr(mean, torch.float64, M * kr, "mean")
    d.scale = _ptr(scale, torch.float64, M * kr, "scale")
    d._tensors = (logw, mean, scale)
    return d


def smc_gmpcn_move(problem, N, gm, beta, tau, n_moves, seed, ctr, level, prec, xi, phi, n_acc, stream=None):
    """gm is (logw[M], mean[M][kr], scale[M][kr]) device tensors."""
    d = gm_desc(*gm)
    _check(lib().smc_gmpcn_move(problem.handle, N, ctypes.byref(d), float(beta), float(tau), int(n_moves), seed,
                                ctr, _ptr(level, torch.int32, N, "level", optional=True), prec,
                                _ptr(xi, torch.float64, N * problem.K, "xi"), _ptr(phi, torch.float64, N, "phi"),
                                _ptr(n_acc, torch.int32, N, "n_acc"), _stream(stream)))


def smc_gmpcn_propose(problem, N, gm, beta, seed, ctr, xi, v, logr, stream=None):
    """The pCN-GM proposal v[N][K] of move counter ctr and its log ratio logr[N] (no potential)."""
    d = gm_desc(*gm)
    _check(lib().smc_gmpcn_propose(problem.handle, N, ctypes.byref(d), float(beta), seed, ctr,
                                   _ptr(xi, torch.float64, N * problem.K, "xi"), _ptr(v, torch.float64, N * problem.K, "v"),
                                   _ptr(logr, torch.float64, N, "logr"), _stream(stream)))


def smc_gm_draw(problem, N, gm, seed, ctr, level, prec, xi, phi, iters=None, stream=None):
    """SMC-GM mutation: xi[N][K] <- independent mixture draws, phi[N] <- their potentials."""
    d = gm_desc(*gm)
    _check(lib().smc_gm_draw(problem.handle, N, ctypes.byref(d), seed, ctr,
                             _ptr(level, torch.int32, N, "level", optional=True), prec,
                             _ptr(xi, torch.float64, N * problem.K, "xi"), _ptr(phi, torch.float64, N, "phi"),
                             _ptr(iters, torch.int32, N, "iters", optional=True), _stream(stream)))


def smc_gm_fit(problem, N, xi, M, iters, var_floor, seed, ctr, logw, mean, scale, centers=None, stream=None):
    """Mixture fit of xi[0..N) on the active modes into logw[M], mean[M][kr], scale[M][kr]."""
    kr = problem.kr
    _check(lib().smc_gm_fit(problem.handle, N, _ptr(xi, torch.float64, N * problem.K, "xi"), int(M), int(iters),
                            float(var_floor), seed, ctr, _ptr(logw, torch.float64, M, "logw"),
                            _ptr(mean, torch.float64, M * kr, "mean"), _ptr(scale, torch.float64, M * kr, "scale"),
                            _ptr(centers, torch.int32, M, "centers", optional=True), _stream(stream)))


def smc_gm_fit_noalloc(N, K, active, xi, M, iters, var_floor, seed, ctr, logw, mean, scale, centers=None,
                       stream=None):
    """The same fit without a problem and without allocating: active[kr] (int32, device) lists the
    coordinates of xi[N][K] to fit; the workspace is the library's static array (N up to
    smc_gm_fit_noalloc_max())."""
    kr = int(active.numel())
    _check(lib().smc_gm_fit_noalloc(N, int(K), kr, _ptr(active, torch.int32, kr, "active"),
                                    _ptr(xi, torch.float64, N * K, "xi"), int(M), int(iters), float(var_floor), seed,
                                    ctr, _ptr(logw, torch.float64, M, "logw"), _ptr(mean, torch.float64, M * kr, "mean"),
                                    _ptr(scale, torch.float64, M * kr, "scale"),
                                    _ptr(centers, torch.int32, M, "centers", optional=True), _stream(stream)))


def smc_gm_fit_noalloc_max():
    return int(lib().smc_gm_fit_noalloc_max())


def smc_forward_state(problem, N, xi, prec, G, w, iters=None, stream=None):
    """w: [N][n][n] FP64 forward solutions of grid 0 (the checkpointed forward state)."""
    n = problem.grids[0]
    _check(lib().smc_forward_state(problem.handle, N, _ptr(xi, torch.float64, N * problem.K, "xi"), prec,
                                   _ptr(G, torch.float64, N * problem.n_obs, "G", optional=True),
                                   _ptr(w, torch.float64, N * n * n, "w"),
                                   _ptr(iters, torch.int32, N, "iters", optional=True), _stream(stream)))


def smc_value_and_grad(problem, N, xi, prec, w, phi, grad, iters=None, stream=None):
    """Potential and dPhi/dxi by an adjoint solve; w = forward states from smc_forward_state or None."""
    n = problem.grids[0]
    _check(lib().smc_value_and_grad(problem.handle, N, _ptr(xi, torch.float64, N * problem.K, "xi"), prec,
                                    _ptr(w, torch.float64, N * n * n, "w", optional=True),
                                    _ptr(phi, torch.float64, N, "phi", optional=True),
                                    _ptr(grad, torch.float64, N * problem.K, "grad"),
                                    _ptr(iters, torch.int32, N, "iters", optional=True), _stream(stream)))


def smc_pcnl_move(problem, N, beta, tau, n_moves, seed, ctr, prec, xi, phi, grad, n_acc, stream=None):
    _check(lib().smc_pcnl_move(problem.handle, N, float(beta), float(tau), int(n_moves), seed, ctr, prec,
                               _ptr(xi, torch.float64, N * problem.K, "xi"), _ptr(phi, torch.float64, N, "phi"),
                               _ptr(grad, torch.float64, N * problem.K, "grad"), _ptr(n_acc, torch.int32, N, "n_acc"),
                               _stream(stream)))


def stage_desc(n_groups, logw, mean, scale, beta, tau, ctr, seed):
    """Device tensors: logw [G][M], mean and scale [G][M][kr], beta [G], tau [G], ctr [1] (int64)."""
    M = logw.shape[-1]
    kr = mean.shape[-1]
    d = StageDesc()
    d.n_groups, d.M, d.kr, d.seed = int(n_groups), M, kr, int(seed)
    d.logw = _ptr(logw, torch.float64, n_groups * M, "logw")
    d.mean = _ptr(mean, torch.float64, n_groups * M * kr, "mean")
    d.scale = _ptr(scale, torch.float64, n_groups * M * kr, "scale")
    d.beta = _ptr(beta, torch.float64, n_groups, "beta")
    d.tau = _ptr(tau, torch.float64, n_groups, "tau")
    d.ctr = _ptr(ctr, torch.int64, 1, "ctr")
    # the descriptor holds device addresses: keep the tensors alive as long as it (and any graph
    # captured from it) exists, or their memory could be reused before the kernels read it
    d._tensors = (logw, mean, scale, beta, tau, ctr)
    return d


def smc_gmpcn_stage(problem, N, level, stage, n_moves, prec, xi, phi, n_acc, stream=None):
    """stage: a StageDesc from stage_desc(...)."""
    _check(lib().smc_gmpcn_stage(problem.handle, N, _ptr(level, torch.int32, N, "level", optional=True),
                                 ctypes.byref(stage), int(n_moves), prec, _ptr(xi, torch.float64, N * problem.K, "xi"),
                                 _ptr(phi, torch.float64, N, "phi"), _ptr(n_acc, torch.int32, N, "n_acc"),
                                 _stream(stream)))


class StageGraph:
    """smc_gmpcn_stage captured once into a HIP graph; launch() replays it."""

    def __init__(self, problem, N, level, stage, n_moves, prec, xi, phi, n_acc, stream):
        self.handle = c_vp()
        self._keep = (problem, level, stage, xi, phi, n_acc)
        _check(lib().smc_stage_graph_create(problem.handle, N, _ptr(level, torch.int32, N, "level", optional=True),
                                            ctypes.byref(stage), int(n_moves), prec,
                                            _ptr(xi, torch.float64, N * problem.K, "xi"),
                                            _ptr(phi, torch.float64, N, "phi"), _ptr(n_acc, torch.int32, N, "n_acc"),
                                            _stream(stream), ctypes.byref(self.handle)))

    def launch(self, stream=None):
        _check(lib().smc_stage_graph_launch(self.handle, _stream(stream)))

    def close(self):
        if getattr(self, "handle", None):
            lib().smc_stage_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SamplerGraph:
    """A whole tempering stage of G samplers (smc_sampler_graph_create) captured once; launch()
    runs the next stage.  The tensors are the samplers' device state, read and written in place:
    xi [N][K], phi [N], xi2 [N][K], phi2 [N], W [N], idx [N] (int32), tau, tau_new, h, log_z and
    beta [G], logw [G][M], mean and scale [G][M][kr], ctr [1] (int64; stage s runs at s * stride),
    level [N] (int32, or None for one group), n_acc [N] (int32), record [max_stages][G][5], flags
    [1] (int32, or None)."""

    def __init__(self, problem, counts, M, n_moves, fit_iters, ess_frac, var_floor, seed, stride, prec, t, stream,
                 max_stages):
        G = len(counts)
        N = sum(int(c) for c in counts)
        K, kr = problem.K, problem.kr
        d = SamplerGraphDesc()
        d.n_groups, d.M, d.kr, d.fit_iters = G, int(M), kr, int(fit_iters)
        for g, c in enumerate(counts):
            d.counts[g] = int(c)
        d.n_moves, d.max_stages = int(n_moves), int(max_stages)
        d.ess_frac, d.var_floor, d.seed, d.stride = float(ess_frac), float(var_floor), int(seed), int(stride)
        d.xi = _ptr(t["xi"], torch.float64, N * K, "xi")
        d.phi = _ptr(t["phi"], torch.float64, N, "phi")
        d.xi2 = _ptr(t["xi2"], torch.float64, N * K, "xi2")
        d.phi2 = _ptr(t["phi2"], torch.float64, N, "phi2")
        d.W = _ptr(t["W"], torch.float64, N, "W")
        d.idx = _ptr(t["idx"], torch.int32, N, "idx")
        for name in ("tau", "tau_new", "h", "log_z", "beta"):
            setattr(d, name, _ptr(t[name], torch.float64, G, name))
        d.logw = _ptr(t["logw"], torch.float64, G * M, "logw")
        d.mean = _ptr(t["mean"], torch.float64, G * M * kr, "mean")
        d.scale = _ptr(t["scale"], torch.float64, G * M * kr, "scale")
        d.ctr = _ptr(t["ctr"], torch.int64, 1, "ctr")
        d.level = _ptr(t.get("level"), torch.int32, N, "level", optional=True)
        d.n_acc = _ptr(t["n_acc"], torch.int32, N, "n_acc")
        d.record = _ptr(t["record"], torch.float64, max_stages * G * 5, "record")
        d.flags = _ptr(t.get("flags"), torch.int32, 1, "flags", optional=True)
        self.handle = c_vp()
        # the graph holds device addresses: keep every tensor alive as long as it exists
        self._keep = (problem, dict(t), d)
        _check(lib().smc_sampler_graph_create(problem.handle, ctypes.byref(d), prec, _stream(stream),
                                              ctypes.byref(self.handle)))

    def launch(self, stream=None):
        _check(lib().smc_stage_graph_launch(self.handle, _stream(stream)))

    def close(self):
        if getattr(self, "handle", None):
            lib().smc_stage_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def smc_tile_candidates(n):
    rows = (c_i32 * 8)()
    count = c_i32()
    _check(lib().smc_tile_candidates(int(n), rows, ctypes.byref(count)))
    return [rows[k] for k in range(count.value)]


def smc_set_stage_fusion(problem, enable):
    """One persistent launch per move stage (True, where supported) or one launch per step (False, the
    default)."""
    _check(lib().smc_set_stage_fusion(problem.handle, 1 if enable else 0))


def smc_set_tile(problem, level, rows):
    _check(lib().smc_set_tile(problem.handle, int(level), int(rows)))


def smc_get_tile(problem, level):
    out = c_i32()
    _check(lib().smc_get_tile(problem.handle, int(level), ctypes.byref(out)))
    return out.value


def smc_autotune(problem, level, N, reps=2, stream=None):
    """Time every tile candidate of grid `level`; keep the fastest.  Returns (rows, {rows: ms})."""
    cands = smc_tile_candidates(problem.grids[level])
    ms = (c_dbl * 8)()
    out = c_i32()
    _check(lib().smc_autotune(problem.handle, int(level), int(N), int(reps), _stream(stream), ctypes.byref(out), ms))
    return out.value, {c: ms[k] for k, c in enumerate(cands)}


def smc_temper(N, phi, tau_in, ess_frac, h, tau_new, W, log_z_inc, flags=None, stream=None):
    _check(lib().smc_temper(N, _ptr(phi, torch.float64, N, "phi"), _ptr(tau_in, torch.float64, 1, "tau_in"),
                            float(ess_frac), _ptr(h, torch.float64, 1, "h"), _ptr(tau_new, torch.float64, 1, "tau_new"),
                            _ptr(W, torch.float64, N, "W"), _ptr(log_z_inc, torch.float64, 1, "log_z_inc"),
                            _ptr(flags, torch.int32, 1, "flags", optional=True), _stream(stream)))


def smc_resample(N, W, u53, idx, flags=None, stream=None):
    _check(lib().smc_resample(N, _ptr(W, torch.float64, N, "W"), int(u53), _ptr(idx, torch.int32, N, "idx"),
                              _ptr(flags, torch.int32, 1, "flags", optional=True), _stream(stream)))


def smc_gather(N, K, idx, xi_in, phi_in, xi_out, phi_out, stream=None):
    _check(lib().smc_gather(N, K, _ptr(idx, torch.int32, N, "idx"), _ptr(xi_in, torch.float64, N * K, "xi_in"),
                            _ptr(phi_in, torch.float64, N, "phi_in", optional=True),
                            _ptr(xi_out, torch.float64, N * K, "xi_out"),
                            _ptr(phi_out, torch.float64, N, "phi_out", optional=True), _stream(stream)))


def smc_profile(problem, enable):
    _check(lib().smc_profile(problem.handle, int(bool(enable))))


def smc_profile_read(problem, stream=None):
    """dict(ms, launches, iters, sweeps, solves, precond_apps) for the solve launches since smc_profile(p, 1)."""
    ms = c_dbl()
    vals = [c_i64() for _ in range(5)]
    _check(lib().smc_profile_read(problem.handle, _stream(stream), ctypes.byref(ms), *[ctypes.byref(v) for v in vals]))
    return dict(ms=ms.value, launches=vals[0].value, iters=vals[1].value, sweeps=vals[2].value, solves=vals[3].value,
                precond_apps=vals[4].value)


def smc_precond_apply(problem, level, N, r, z, stream=None):
    n = problem.grids[level]
    _check(lib().smc_precond_apply(problem.handle, int(level), N, _ptr(r, torch.float32, N * n * n, "r"),
                                   _ptr(z, torch.float32, N * n * n, "z"), _stream(stream)))
