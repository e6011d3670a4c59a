"""Problem definition: grids, prior eigenpairs, observation nodes and data.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Prior.  The prior is mu_0 = N(0, C) with C positive, self-adjoint and trace class
(Sec. 2.1); the Darcy example uses C_0 = (I - Delta)^{-2} (Sec. 3.2).  It is
represented through its Karhunen-Loeve eigenpairs (lambda_i, phi_i), the same
eigenbasis the mixture covariances share (Sec. 2.3, C_j phi_i = lambda_ji phi_i).
A particle is the vector xi of whitened coefficients, u = sum_i sqrt(lambda_i)
xi_i phi_i, so xi ~ N(0, I) under the prior.

  2D, on (0,1)^2 with Neumann eigenfunctions of -Delta:
      phi_kl(x, y) = c_k c_l cos(k pi x) cos(l pi y),  c_0 = 1, c_k = sqrt(2)
      lambda_kl    = (1 + pi^2 (k^2 + l^2))^{-2},       k, l = 0 .. kl-1
      flat index   = k * kl + l   (k goes with x, l with y)
  1D, on (0,1) with Dirichlet eigenfunctions of -d^2/dx^2:
      phi_k(x) = sqrt(2) sin(k pi x),  lambda_k = (1 + k^2 pi^2)^{-2},  k = 1 .. kl
      flat index = k - 1

Grid.  n intervals per axis, h = 1/n, nodes x_i = i/n, i = 0..n; the unknowns are
the interior nodes.  Grids with n = 64, 128, 256 nest, so an observation point on
a multiple of 1/64 is a node of each of them.

Active modes.  The mixture moves the K_r modes with the largest lambda (ties go to
the smaller flat index); the other modes keep the prior's law (mean 0, scale 1),
which keeps every mixture component equivalent to mu_0 (assumption of Thm. on the
well-definedness of mu_0(dv)Q(v,du), Sec. 2.3).

Data (Sec. 2.1, eq. for d; Sec. 3.2 for the noise rule).  d = F(u_true) + eps with
eps ~ N(0, sigma^2 I), sigma = noise_frac * max_k |F(u_true)_k|, F evaluated on a
finer grid than the inference grids.  Optionally observation points come in
mirror pairs about x = 1/2 and each pair gets the pair-averaged noise-free value
plus one shared noise draw, which makes the potential exactly invariant under
x -> 1 - x.
"""
import json
import numpy as np


class Problem:
    """A problem read from a JSON definition (see tests/golden/problem_*.json)."""

    def __init__(self, d):
        self.d = d
        self.name = d["name"]
        self.dim = int(d["dim"])
        self.grids = [int(n) for n in d["grids"]]
        self.kl = int(d["kl_per_axis"])
        self.K = self.kl ** self.dim
        self.kr = int(d.get("kr", 0))
        self.obs_den = int(d["obs_den"])
        self.obs = [tuple(int(v) for v in o) for o in d["obs"]]
        self.f = float(d.get("f", 1.0))
        self.y = np.array(d["y"], dtype=np.float64) if "y" in d else None
        self.sigma = float(d["sigma"]) if "sigma" in d else None
        self.lam = eigenvalues(self.dim, self.kl)
        self.sqrt_lam = np.sqrt(self.lam)

    @classmethod
    def load(cls, path):
        with open(path) as fh:
            return cls(json.load(fh))

    @property
    def n_obs(self):
        return len(self.obs)

    def obs_nodes(self, n):
        """Node indices of the observation points on the grid with n intervals."""
        out = []
        for o in self.obs:
            idx = []
            for num in o:
                if (num * n) % self.obs_den:
                    raise ValueError("observation point is not a node of grid %d" % n)
                idx.append(num * n // self.obs_den)
            out.append(tuple(idx))
        return out

    def active(self):
        return active_modes(self.lam, self.kr)


def eigenvalues(dim, kl):
    if dim == 2:
        k = np.arange(kl, dtype=np.float64)
        kk = k[:, None] ** 2 + k[None, :] ** 2
        return ((1.0 + np.pi ** 2 * kk) ** -2).reshape(-1)
    if dim == 1:
        k = np.arange(1, kl + 1, dtype=np.float64)
        return (1.0 + np.pi ** 2 * k ** 2) ** -2
    raise ValueError("dim must be 1 or 2")


def basis_matrix(dim, kl, n):
    """Per-axis basis values at the nodes x_i = i/n: B[i, k]."""
    x = np.arange(n + 1, dtype=np.float64) / n
    if dim == 2:
        k = np.arange(kl)
        c = np.where(k == 0, 1.0, np.sqrt(2.0))
        return c[None, :] * np.cos(np.pi * np.outer(x, k))
    k = np.arange(1, kl + 1)
    return np.sqrt(2.0) * np.sin(np.pi * np.outer(x, k))


def synthesize(prob, xi, n):
    """Nodal field u = sum_i sqrt(lambda_i) xi_i phi_i on the grid with n intervals.

    2D returns U[i, j] = u(x_i, y_j), shape (n+1, n+1); 1D returns U[i], shape (n+1).
    """
    xi = np.asarray(xi, dtype=np.float64)
    B = basis_matrix(prob.dim, prob.kl, n)
    coef = prob.sqrt_lam * xi
    if prob.dim == 2:
        Xs = coef.reshape(prob.kl, prob.kl)          # [k (x-mode), l (y-mode)]
        return B @ Xs @ B.T                          # sum_k sum_l B[i,k] Xs[k,l] B[j,l]
    return B @ coef


def active_modes(lam, kr):
    order = sorted(range(lam.size), key=lambda i: (-lam[i], i))
    return np.array(order[:kr], dtype=np.int64)


def reflect_x(prob, xi):
    """Coefficients of u(1 - x, y): cos(k pi (1-x)) = (-1)^k cos(k pi x)."""
    if prob.dim != 2:
        raise ValueError("reflection is defined for the 2D cosine basis")
    k = np.repeat(np.arange(prob.kl), prob.kl)
    return np.where(k % 2 == 1, -1.0, 1.0) * np.asarray(xi)
