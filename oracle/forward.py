"""Forward map F and potential Phi by direct solves.

TEST INFRASTRUCTURE ONLY (see the package docstring).

PDE (Sec. 3.2, eq. (example2:PDE), read with the gradient on the state):
    -div(e^u grad w) = f  on (0,1)^d,   w = 0 on the boundary.
Finite differences in flux form on the grid with n intervals (h = 1/n): at an
interior node P with neighbours Q (4 in 2D, 2 in 1D)
    sum_Q a_PQ (w_P - w_Q) / h^2 = f_P,    a_PQ = exp((u_P + u_Q) / 2),
with w_Q = 0 on the boundary.  The face coefficient is the geometric mean of
e^u at the two nodes (the paper uses finite elements and does not fix one).

Observation (Sec. 3.2): F(u) = (w(x_1), ..., w(x_Nd)), point values at nodes.
Potential (Sec. 2.1): Phi(u) = |F(u) - d|^2 / (2 sigma^2).
"""
import numpy as np
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg


def darcy_matrix_2d(U, n):
    """Sparse matrix of the 2D flux-form operator on the (n-1)^2 interior nodes.

    U[i, j] is the nodal field at (i/n, j/n); unknown (i, j) has row
    (i-1)*(n-1) + (j-1).
    """
    m = n - 1
    h2 = 1.0 / n ** 2
    rows, cols, vals = [], [], []
    diag = np.zeros((m, m))
    idx = np.arange(m * m).reshape(m, m)
    for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        # face between interior P = (i, j) and Q = (i+di, j+dj)
        i = np.arange(1, n)[:, None]
        j = np.arange(1, n)[None, :]
        a = np.exp(0.5 * (U[1:n, 1:n] + U[1 + di:n + di, 1 + dj:n + dj])) / h2
        diag += a
        qi, qj = i + di + 0 * j, j + dj + 0 * i
        inner = (qi >= 1) & (qi <= m) & (qj >= 1) & (qj <= m)
        rows.append(idx[inner])
        cols.append(idx[(qi[inner] - 1), (qj[inner] - 1)])
        vals.append(-a[inner])
    rows.append(idx.reshape(-1))
    cols.append(idx.reshape(-1))
    vals.append(diag.reshape(-1))
    return scipy.sparse.csc_matrix(
        (np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(m * m, m * m))


def solve_2d(U, n, f=1.0):
    """State W[i, j] on all nodes (zeros on the boundary) for nodal field U."""
    m = n - 1
    A = darcy_matrix_2d(U, n)
    rhs = np.full(m * m, float(f)) if np.isscalar(f) else np.asarray(f, dtype=np.float64)[1:n, 1:n].reshape(-1)
    w = scipy.sparse.linalg.spsolve(A, rhs)
    W = np.zeros((n + 1, n + 1))
    W[1:n, 1:n] = w.reshape(m, m)
    return W


def solve_1d(U, n, f=1.0):
    """State W[i] (zeros at both ends) for nodal field U on the 1D grid."""
    h2 = 1.0 / n ** 2
    a = np.exp(0.5 * (U[:-1] + U[1:])) / h2       # a[i] is the face between nodes i, i+1
    m = n - 1
    ab = np.zeros((3, m))
    ab[1] = a[:-1] + a[1:]                         # node i (1..n-1): faces i-1 and i
    ab[0, 1:] = -a[1:m]                            # super-diagonal
    ab[2, :-1] = -a[1:m]                           # sub-diagonal
    rhs = np.full(m, float(f)) if np.isscalar(f) else np.asarray(f, dtype=np.float64)[1:n]
    w = scipy.linalg.solve_banded((1, 1), ab, rhs)
    W = np.zeros(n + 1)
    W[1:n] = w
    return W


def solve(prob, U, n):
    return solve_2d(U, n, prob.f) if prob.dim == 2 else solve_1d(U, n, prob.f)


def observe(prob, W, n):
    nodes = prob.obs_nodes(n)
    if prob.dim == 2:
        return np.array([W[i, j] for i, j in nodes])
    return np.array([W[i] for (i,) in nodes])


def forward(prob, xi, n):
    """F(u(xi)) on the grid with n intervals."""
    from .problem import synthesize
    U = synthesize(prob, xi, n)
    return observe(prob, solve(prob, U, n), n)


def potential(G, y, sigma):
    """Phi = |G - y|^2 / (2 sigma^2); +inf when G is not finite."""
    G = np.asarray(G, dtype=np.float64)
    r = G - np.asarray(y, dtype=np.float64)
    out = np.sum(r * r, axis=-1) / (2.0 * sigma ** 2)
    return np.where(np.all(np.isfinite(G), axis=-1), out, np.inf)


def phi(prob, xi, n):
    return float(potential(forward(prob, xi, n), prob.y, prob.sigma))
