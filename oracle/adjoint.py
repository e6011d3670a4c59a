"""Gradient of the potential with respect to the whitened coefficients.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper counts one extra (adjoint) PDE solve for gradient-informed moves such as
pCN-Langevin (Sec. 2.4).  With A(u) w = f the discrete flux-form operator (see
`forward`) and Phi = |P w - d|^2 / (2 sigma^2):
    A lam = P^T (P w - d) / sigma^2             (A is symmetric)
    dPhi/du_P = -(1/2) sum_{faces (P,Q)} a_PQ (lam_P - lam_Q)(w_P - w_Q) / h^2
for every node P (lam = w = 0 on the boundary), because lam^T A w is the sum over
faces of a_PQ (lam_P - lam_Q)(w_P - w_Q)/h^2 and d a_PQ / d u_P = a_PQ / 2.
Finally grad_xi Phi = sqrt(lambda) * (B^T (dPhi/du) B), the transpose of the KL
synthesis.
"""
import numpy as np
import scipy.sparse.linalg

from .forward import darcy_matrix_2d, observe, potential
from .problem import basis_matrix, synthesize


def value_and_grad(prob, xi, n):
    if prob.dim != 2:
        raise ValueError("the adjoint gradient is implemented for the 2D problem")
    U = synthesize(prob, xi, n)
    A = darcy_matrix_2d(U, n)
    m = n - 1
    w = scipy.sparse.linalg.spsolve(A, np.full(m * m, prob.f))
    W = np.zeros((n + 1, n + 1))
    W[1:n, 1:n] = w.reshape(m, m)
    G = observe(prob, W, n)
    phi = float(potential(G, prob.y, prob.sigma))
    rhs = np.zeros((n + 1, n + 1))
    for (i, j), r in zip(prob.obs_nodes(n), (G - prob.y) / prob.sigma ** 2):
        rhs[i, j] += r
    lam = scipy.sparse.linalg.spsolve(A, rhs[1:n, 1:n].reshape(-1))
    L = np.zeros((n + 1, n + 1))
    L[1:n, 1:n] = lam.reshape(m, m)
    h2 = 1.0 / n ** 2
    dU = np.zeros((n + 1, n + 1))
    # x-faces between (i, j) and (i+1, j); y-faces between (i, j) and (i, j+1)
    ax = np.exp(0.5 * (U[:-1, :] + U[1:, :]))
    tx = -0.5 * ax * (L[:-1, :] - L[1:, :]) * (W[:-1, :] - W[1:, :]) / h2
    ay = np.exp(0.5 * (U[:, :-1] + U[:, 1:]))
    ty = -0.5 * ay * (L[:, :-1] - L[:, 1:]) * (W[:, :-1] - W[:, 1:]) / h2
    dU[:-1, :] += tx
    dU[1:, :] += tx
    dU[:, :-1] += ty
    dU[:, 1:] += ty
    B = basis_matrix(2, prob.kl, n)
    g = prob.sqrt_lam * (B.T @ dU @ B).reshape(-1)
    return phi, g
