"""The SMC loop of Alg. 1 with a pCN-GM mutation (SMC-pCN-GM), and SMC-GM (Alg. 3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Per stage, in the order of the operator form S^N P_{j+1} L_{j+1} (Sec. 2.2,
eq. (decidemuJN)): re-weight with the next increment h (Alg. 1, App. C), resample
(every stage, since Alg. 1 resets the weights to 1/N), fit the mixture to the
resampled cloud, then n_moves pCN-GM steps (Alg. 2) at the new temperature, and
finally the App. C step-size rule
    beta <- 2 beta if mean acceptance > 0.3, beta / 2 if < 0.15, else unchanged,
capped at beta <= 1 since the proposal needs beta in (0, 1] (Sec. 2.3).
The loop stops when the cumulative temperature reaches 1 (sum_j h_j = 1).

SMC-GM (Alg. 3, Sec. 2.4) keeps the re-weighting and resampling and replaces the
mutation by the mixture itself: fit the mixture to the resampled cloud, replace every
particle by an independent draw from it (accepted without a test), and evaluate the
potential of the draws, which the next stage re-weights.  The loop stops after the
stage whose temperature reaches 1 (Alg. 3 runs its loop one step further than Alg. 1;
both stop at the same final temperature here).

Random numbers: the prior draw uses counter 0; stage s uses counters
s * 2^20 + m for its moves, draws its resampling uniform from block
RESAMPLE_BLOCK at counter s * 2^20, and seeds its mixture fit (gmfit.fit_philox)
at counter s * 2^20.  SMC-GM's fit and draw at stage s both use counter s * 2^20
(different blocks).  A run is therefore a function of its seed alone, and the GPU
drivers, which follow the same layout, replay it.
"""
import numpy as np

from . import gmfit, philox
from .moves import GM, gm_draw, gmpcn_moves, pcn_gm, prior_sample
from .resample import systematic
from .temper import temper

RESAMPLE_BLOCK = 0x80000001
STAGE_STRIDE = 1 << 20


def resample_u53(seed, ctr):
    c = np.array([RESAMPLE_BLOCK, 0, ctr & philox.MASK32, (ctr >> 32) & philox.MASK32], dtype=np.uint64)
    w = philox.philox4x32_10(c, philox._key(seed))
    return (int(w[0]) >> 5) * (1 << 26) + (int(w[1]) >> 6)


def adapt_beta(beta, rate):
    if rate > 0.3:
        return min(1.0, 2.0 * beta)
    if rate < 0.15:
        return 0.5 * beta
    return beta


def _pde_potentials(args):
    from .forward import phi as phi_pde
    prob, n, xi = args
    return np.array([phi_pde(prob, x, n) for x in xi])


def _pde_moves(args):
    prob, n, xi, phi, gm, beta, tau, n_moves, seed, ctr, ids = args
    return gmpcn_moves(prob, n, xi, phi, gm, beta, tau, n_moves, seed, ctr, ids=ids)


def run(prob, n, N, M, n_moves, rho, beta0, seed, phi_fn=None, kr=None, max_stages=500, xi0=None, ids=None,
        ctr_off=0, pmap=None, chunks=1):
    """Returns dict(xi, phi, taus, log_Z, betas, rates, n_acc).

    A sampler that shares its random streams with others (several samplers in one batch) passes
    its starting cloud xi0, its particles' ids (the words of their streams) and ctr_off, added to
    the counter of its resampling uniform and its mixture seeding.

    pmap (a map over a list, e.g. a process pool's; PDE potentials only) spreads the potentials
    of the initial cloud and each stage's moves over `chunks` contiguous blocks of particles.
    Particles never interact inside a stage's moves and every random number is keyed by the
    particle's id, so the result is the same as with pmap=None."""
    from .forward import phi as phi_pde
    K = prob.K
    f = phi_fn if phi_fn is not None else (lambda x: phi_pde(prob, x, n))
    active = prob.active() if kr is None else np.arange(kr)
    xi = prior_sample(K, N, seed, 0) if xi0 is None else np.array(xi0, dtype=np.float64)
    par = pmap is not None and phi_fn is None
    blocks = np.array_split(np.arange(N), max(1, chunks))
    row_ids = np.arange(N) if ids is None else np.asarray(ids)
    if par:
        phi = np.concatenate(list(pmap(_pde_potentials, [(prob, n, xi[b]) for b in blocks])))
    else:
        phi = np.array([f(x) for x in xi])
    tau, beta, log_Z = 0.0, float(beta0), 0.0
    taus, betas, rates, accepts = [0.0], [], [], []
    for s in range(1, max_stages + 1):
        h, tau, W, lz, stalled = temper(phi, tau, rho)
        if stalled:
            raise RuntimeError("temperature bisection stalled")
        log_Z += lz
        taus.append(tau)
        idx = systematic(W, resample_u53(seed, s * STAGE_STRIDE + ctr_off))
        xi, phi = xi[idx], phi[idx]
        if M == 1:
            gm = pcn_gm(K, active)
        else:
            logw, mean, var, _ = gmfit.fit_philox(xi[:, active], M, seed, s * STAGE_STRIDE + ctr_off)
            gm = GM(logw, mean, var, active, K)
        if par:
            out = list(pmap(_pde_moves, [(prob, n, xi[b], phi[b], gm, beta, tau, n_moves, seed, s * STAGE_STRIDE,
                                          row_ids[b]) for b in blocks]))
            xi = np.concatenate([o[0] for o in out])
            phi = np.concatenate([o[1] for o in out])
            n_acc = np.concatenate([o[2] for o in out])
        else:
            xi, phi, n_acc = gmpcn_moves(prob, n, xi, phi, gm, beta, tau, n_moves, seed, s * STAGE_STRIDE,
                                         phi_fn=f, ids=ids)
        rate = n_acc.sum() / (N * n_moves)
        betas.append(beta)
        rates.append(rate)
        accepts.append(int(n_acc.sum()))
        beta = adapt_beta(beta, rate)
        if tau >= 1.0:
            break
    return dict(xi=xi, phi=phi, taus=np.array(taus), log_Z=log_Z, betas=betas, rates=rates, n_acc=accepts)


def run_gm(prob, n, N, M, rho, seed, phi_fn=None, kr=None, iters=50, var_floor=1e-3, max_stages=500):
    """SMC-GM (Alg. 3).  Returns dict(xi, phi, taus, log_Z, mixtures)."""
    from .forward import phi as phi_pde
    K = prob.K
    f = phi_fn if phi_fn is not None else (lambda x: phi_pde(prob, x, n))
    active = prob.active() if kr is None else np.arange(kr)
    xi = prior_sample(K, N, seed, 0)
    phi = np.array([f(x) for x in xi])
    tau, log_Z = 0.0, 0.0
    taus, mixtures = [0.0], []
    for s in range(1, max_stages + 1):
        h, tau, W, lz, stalled = temper(phi, tau, rho)
        if stalled:
            raise RuntimeError("temperature bisection stalled")
        log_Z += lz
        taus.append(tau)
        ctr = s * STAGE_STRIDE
        idx = systematic(W, resample_u53(seed, ctr))
        logw, mean, var, _ = gmfit.fit_philox(xi[idx][:, active], M, seed, ctr, iters, var_floor)
        gm = GM(logw, mean, var, active, K)
        mixtures.append((logw, mean, var))
        xi = gm_draw(gm, seed, ctr, np.arange(N))
        phi = np.array([f(x) for x in xi])
        if tau >= 1.0:
            break
    return dict(xi=xi, phi=phi, taus=np.array(taus), log_Z=log_Z, mixtures=mixtures)
