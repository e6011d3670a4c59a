"""End-to-end posterior study of finished SMC runs: the quantities Sec. 3.3 reports.

  * modes: the final cloud clustered by k-means in function space (the L^2 metric, which in
    the orthonormal KL basis is the Euclidean metric of the coefficients u_k = sqrt(lambda_k) xi_k);
    the number of clusters is the k in 2..k_max with the largest mean silhouette, or 1 when no
    k reaches a silhouette of 0.25 (below that, clusters carry no substantial structure);
  * average data misfit of the cluster means, (1/N_modal) sum_i ||F(u_i) - d||_2, with F
    evaluated by the library's forward solve (Sec. 3.3, sparse-measurement table);
  * relative L^2 error of the posterior mean against the truth, ||u_mean - u_true|| / ||u_true||,
    exact in function space by Parseval (Sec. 3.3, posterior mean);
  * total-variation distance between two runs' marginal densities of the first coefficients,
    with Gaussian kernel density estimates (Sec. 3.3, marginal densities);
  * temperature curves of samplers on nested grids (Sec. 3.3, mesh independence).

This is post-processing of a finished run on the host (the final cloud is a few MB); the
sampling itself runs in the library.  Run as `python -m paper_2503_16028_amd.study PROBLEM.json`.
"""
import argparse
import json
import math
import time

import numpy as np


# ------------------------------------------------------------------ clustering

def kmeans(X, k, seed=0, iters=100):
    """Lloyd's k-means from a k-means++ seeding (numpy generator `seed`).  Returns
    (labels[N], centers[k][D], inertia)."""
    X = np.asarray(X, dtype=np.float64)
    N = X.shape[0]
    rng = np.random.default_rng(seed)
    centers = [X[rng.integers(N)]]
    d2 = np.sum((X - centers[0]) ** 2, axis=1)
    for _ in range(1, k):
        tot = d2.sum()
        c = X[rng.choice(N, p=d2 / tot)] if tot > 0 else X[rng.integers(N)]
        centers.append(c)
        d2 = np.minimum(d2, np.sum((X - c) ** 2, axis=1))
    C = np.array(centers)
    labels = np.full(N, -1)
    for _ in range(iters):
        D = _sqdist(X, C)
        new = np.argmin(D, axis=1)
        if np.array_equal(new, labels):
            break
        labels = new
        for j in range(k):
            sel = labels == j
            if sel.any():
                C[j] = X[sel].mean(axis=0)
    D = _sqdist(X, C)
    labels = np.argmin(D, axis=1)
    return labels, C, float(D[np.arange(N), labels].sum())


def _sqdist(X, C):
    return np.maximum(np.sum(X * X, axis=1)[:, None] - 2.0 * X @ C.T + np.sum(C * C, axis=1)[None, :], 0.0)


def silhouette(X, labels):
    """Mean silhouette (b - a) / max(a, b) over all points; a point alone in its cluster scores 0."""
    X = np.asarray(X, dtype=np.float64)
    ks = np.unique(labels)
    if ks.size < 2:
        return 0.0
    N = X.shape[0]
    sums = np.zeros((N, ks.size))
    for j0 in range(0, N, 1024):
        D = np.sqrt(_sqdist(X[j0:j0 + 1024], X))
        for c, kk in enumerate(ks):
            sums[j0:j0 + 1024, c] = D[:, labels == kk].sum(axis=1)
    sizes = np.array([(labels == kk).sum() for kk in ks])
    own = np.searchsorted(ks, labels)
    a = sums[np.arange(N), own] / np.maximum(sizes[own] - 1, 1)
    other = sums / sizes[None, :]
    other[np.arange(N), own] = np.inf
    b = other.min(axis=1)
    s = np.where(sizes[own] > 1, (b - a) / np.maximum(np.maximum(a, b), 1e-300), 0.0)
    return float(s.mean())


def count_modes(X, k_max=8, seed=0, threshold=0.25, sample=4096):
    """Number of clusters of the cloud X (rows): the k in 2..k_max with the largest mean
    silhouette (scored on at most `sample` rows), 1 if none reaches `threshold`.
    Returns (k, labels, centers, scores{k: silhouette})."""
    X = np.asarray(X, dtype=np.float64)
    rng = np.random.default_rng(seed)
    sub = X if X.shape[0] <= sample else X[rng.choice(X.shape[0], sample, replace=False)]
    scores, fits = {}, {}
    for k in range(2, k_max + 1):
        if k >= sub.shape[0]:
            break
        lab, C, _ = kmeans(X, k, seed)
        fits[k] = (lab, C)
        sub_lab = np.argmin(_sqdist(sub, C), axis=1)
        scores[k] = silhouette(sub, sub_lab)
    best = max(scores, key=scores.get) if scores else 1
    if not scores or scores[best] < threshold:
        return 1, np.zeros(X.shape[0], dtype=np.int64), X.mean(axis=0, keepdims=True), scores
    lab, C = fits[best]
    return best, lab, C, scores


# ------------------------------------------------------------------ errors and distances

def rel_l2_error(lam, xi_mean, xi_true):
    """||u_mean - u_true||_L2 / ||u_true||_L2 with u = sum sqrt(lambda_k) xi_k phi_k and an
    orthonormal basis (Parseval)."""
    lam = np.asarray(lam, dtype=np.float64)
    d = np.asarray(xi_mean) - np.asarray(xi_true)
    return float(math.sqrt(np.sum(lam * d * d) / np.sum(lam * np.asarray(xi_true) ** 2)))


def kde(x, grid):
    """Gaussian kernel density estimate of the sample x on the uniform `grid`, Scott's bandwidth:
    the sample is linearly binned onto the grid, then convolved with the kernel sampled at the
    grid spacing (binning moves each point by under one spacing)."""
    x = np.asarray(x, dtype=np.float64)
    P = grid.size
    bw = max(x.std(ddof=1), 1e-12) * x.size ** (-0.2)
    dx = grid[1] - grid[0]
    pos = np.clip((x - grid[0]) / dx, 0.0, P - 1.0)
    i = np.minimum(np.floor(pos).astype(np.int64), P - 2)
    f = pos - i
    w = np.bincount(i, 1.0 - f, P) + np.bincount(i + 1, f, P)
    half = int(math.ceil(5.0 * bw / dx))
    t = np.arange(-half, half + 1) * dx / bw
    kern = np.exp(-0.5 * t * t) / (x.size * bw * math.sqrt(2.0 * math.pi))
    return np.convolve(w, kern, mode="full")[half:half + P]


def tv_distance(a, b, points=2001):
    """(1/2) int |p_a - p_b| for kernel density estimates of two 1D samples (trapezoid rule on a
    grid covering both samples and four bandwidths beyond them)."""
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    s = max(a.std(), b.std(), 1e-12)
    grid = np.linspace(min(a.min(), b.min()) - 4 * s, max(a.max(), b.max()) + 4 * s, points)
    return float(0.5 * np.trapezoid(np.abs(kde(a, grid) - kde(b, grid)), grid))


def mean_tv(U1, U2, n_coef=20):
    """Average TV distance of the marginals of the first n_coef coefficients (columns)."""
    return float(np.mean([tv_distance(U1[:, k], U2[:, k]) for k in range(n_coef)]))


# ------------------------------------------------------------------ a study of one problem

def sqrt_lambda(d):
    """sqrt(lambda_k) of the 2D cosine prior in the library's mode order (index k * kl + l)."""
    kl = int(d["kl_per_axis"])
    k = np.arange(kl)
    lam = (1.0 + np.pi ** 2 * (k[:, None] ** 2 + k[None, :] ** 2)) ** -2.0
    return np.sqrt(lam.ravel())


def modes_and_misfit(problem, d, xi, k_max=8, seed=0, prec=None):
    """Cluster a final cloud (device tensor [N][K]) in function space, solve the forward problem
    at each cluster mean (library) and return the mode count, masses, the average l2 misfit
    ||F(u_i) - d|| of the cluster means and their whitened coefficients."""
    import torch
    from . import smc
    prec = smc.SMC_FP32_REFINE if prec is None else prec
    X = xi.detach().cpu().numpy()
    sl = sqrt_lambda(d)
    k, lab, C, scores = count_modes(X * sl, k_max=k_max, seed=seed)
    means = np.array([X[lab == j].mean(axis=0) for j in range(k)])
    G = torch.empty(k, problem.n_obs, dtype=torch.float64, device=xi.device)
    smc.smc_forward_batch(problem, k, torch.tensor(means, device=xi.device), None, prec, G)
    y = np.asarray(d["y"], dtype=np.float64)
    mis = np.linalg.norm(G.cpu().numpy() - y[None, :], axis=1)
    masses = np.array([(lab == j).mean() for j in range(k)])
    return dict(n_modal=int(k), masses=masses.tolist(), misfits=mis.tolist(), avg_error=float(mis.mean()),
                silhouettes={int(a): float(b) for a, b in scores.items()}, means=means)


def study(d, N, M=8, n_moves=20, seed=0, methods=("smc-pcn-gm", "smc-gm", "smc-pcn"), k_max=8, n_gm=None,
          device="cuda"):
    """Run each method to temperature 1 on problem `d` (one grid) and report, per method: wall
    time, stages, temperatures, log Z, modes and the average misfit of the cluster means, the
    relative L^2 error of the posterior mean, and the mean TV distance of the first 20
    coefficients' marginals against the first method."""
    import torch
    from . import smc
    from .sampler import SMCGMSampler, SMCSampler
    sl = sqrt_lambda(d)
    xi_true = np.asarray(d["xi_true"], dtype=np.float64) if "xi_true" in d else None
    out, clouds = {}, {}
    for name in methods:
        n = n_gm if (name == "smc-gm" and n_gm) else N
        p = smc.Problem(d, n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if name == "smc-gm":
            r = SMCGMSampler(p, n, M=M, seed=seed, device=device).run()
        else:
            r = SMCSampler(p, n, M=(M if name == "smc-pcn-gm" else 1), n_moves=n_moves, seed=seed,
                           device=device).run()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rep = modes_and_misfit(p, d, r["xi"], k_max=k_max, seed=seed)
        X = r["xi"].cpu().numpy()
        clouds[name] = X * sl
        res = dict(particles=n, seconds=dt, stages=len(r["history"]), log_Z=r["log_Z"],
                   taus=[h["tau"] for h in r["history"]], n_modal=rep["n_modal"], masses=rep["masses"],
                   misfits=rep["misfits"], avg_error=rep["avg_error"], silhouettes=rep["silhouettes"])
        if xi_true is not None:
            res["rel_l2_error_of_mean"] = rel_l2_error(sl ** 2, X.mean(axis=0), xi_true)
            # a symmetric posterior's mean lies between its mirror modes: also the nearest mode's mean
            res["rel_l2_error_of_nearest_mode"] = min(rel_l2_error(sl ** 2, m, xi_true) for m in rep["means"])
        out[name] = res
        p.close()
    first = methods[0]
    for name in methods[1:]:
        out[name]["mean_tv_first20_vs_" + first] = mean_tv(clouds[first], clouds[name], 20)
    return out


def mesh_study(d, counts=(4096, 3072, 1024), M=8, n_moves=20, seed=0, device="cuda"):
    """Samplers on the problem's nested grids run together (MixedSampler): temperature curves,
    stage counts and log Z per grid."""
    import torch
    from . import smc
    from .sampler import MixedSampler
    p = smc.Problem(d, sum(counts))
    ms = MixedSampler(p, counts, M, n_moves, seed=seed, device=device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = ms.run()
    dt = time.perf_counter() - t0
    ms.close()
    grids = list(p.grids)
    p.close()
    return dict(seconds=dt, grids=grids, counts=list(counts),
                taus=[[h["tau"] for h in r["history"]] for r in res],
                stages=[len(r["history"]) for r in res], log_Z=[r["log_Z"] for r in res])


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("problem", help="problem definition (JSON)")
    ap.add_argument("--particles", type=int, default=4096)
    ap.add_argument("--gm-particles", type=int, default=None, help="particles of the SMC-GM run")
    ap.add_argument("--mixture", type=int, default=8)
    ap.add_argument("--moves", type=int, default=20)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--mesh", action="store_true", help="temperature curves on the problem's nested grids")
    ap.add_argument("--counts", type=str, default="4096,3072,1024")
    args = ap.parse_args()
    d = json.load(open(args.problem))
    if args.mesh:
        out = mesh_study(d, tuple(int(c) for c in args.counts.split(",")), args.mixture, args.moves, args.seed)
    else:
        out = study(d, args.particles, args.mixture, args.moves, args.seed, n_gm=args.gm_particles)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
