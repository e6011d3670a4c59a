"""The potential Phi(xi) as a differentiable torch function, backed by the library's adjoint solves.

    phi = potential(problem, xi, prec=SMC_FP32_REFINE, checkpoint="auto")
    phi.sum().backward()      # xi.grad = dPhi/dxi by one adjoint solve per particle

Forward runs one PDE solve per particle (smc_forward_state or smc_forward_batch); backward runs
the adjoint solve and the transposed synthesis (smc_value_and_grad), the extra solve per
particle that gradient-informed moves cost (Sec. 2.4).  What forward keeps for backward:

  "state"      the FP64 forward solutions w, N * n^2 doubles (at 128^2 and N = 2048: 256 MiB);
               backward then solves only the adjoint problems.
  "recompute"  only xi (the checkpoint); backward solves the forward problems again.
  "auto"       "state" when the states fit in `budget_bytes` (default: a quarter of the free
               device memory), else "recompute".

Batches larger than the problem's n_max run in chunks of n_max particles.  All arithmetic runs
in the library; this module only allocates tensors and sequences calls.
"""
import torch

from . import smc


def choose_checkpoint(mode, N, n, budget_bytes):
    """Resolve "auto" to "state" or "recompute" for N particles on an n x n grid."""
    if mode not in ("auto", "state", "recompute"):
        raise ValueError("checkpoint must be 'auto', 'state' or 'recompute' (got %r)" % (mode,))
    if mode != "auto":
        return mode
    return "state" if 8 * N * n * n <= budget_bytes else "recompute"


def _chunks(N, size):
    for a in range(0, N, size):
        yield a, min(N, a + size)


class _Potential(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xi, problem, prec, mode):
        N, K = xi.shape
        n = problem.grids[0]
        dev = xi.device
        xi = xi.detach().contiguous()
        phi = torch.empty(N, dtype=torch.float64, device=dev)
        G = torch.empty(N, problem.n_obs, dtype=torch.float64, device=dev)
        w = torch.empty(N, n * n, dtype=torch.float64, device=dev) if mode == "state" else None
        for a, b in _chunks(N, problem.n_max):
            if w is not None:
                smc.smc_forward_state(problem, b - a, xi[a:b], prec, G[a:b], w[a:b])
            else:
                smc.smc_forward_batch(problem, b - a, xi[a:b], None, prec, G[a:b])
            smc.smc_potential(problem, b - a, G[a:b], phi[a:b])
        ctx.problem, ctx.prec = problem, prec
        if w is not None:
            ctx.save_for_backward(xi, w)
        else:
            ctx.save_for_backward(xi)
        return phi

    @staticmethod
    def backward(ctx, gphi):
        saved = ctx.saved_tensors
        xi = saved[0]
        w = saved[1] if len(saved) > 1 else None
        problem = ctx.problem
        N = xi.shape[0]
        grad = torch.empty_like(xi)
        for a, b in _chunks(N, problem.n_max):
            smc.smc_value_and_grad(problem, b - a, xi[a:b], ctx.prec, None if w is None else w[a:b], None,
                                   grad[a:b])
        return gphi.to(grad.dtype)[:, None] * grad, None, None, None


def potential(problem, xi, prec=smc.SMC_FP32_REFINE, checkpoint="auto", budget_bytes=None):
    """Phi for each row of xi ([N][K] float64 on the device), differentiable in xi."""
    if xi.dim() != 2 or xi.shape[1] != problem.K or xi.dtype != torch.float64 or not xi.is_cuda:
        raise TypeError("xi must be a float64 device tensor of shape [N][%d]" % problem.K)
    if problem.dim != 2:
        raise ValueError("the adjoint gradient is implemented for the 2D problem")
    n = problem.grids[0]
    if budget_bytes is None and checkpoint == "auto":
        free, _ = torch.cuda.mem_get_info(xi.device)
        budget_bytes = free // 4
    mode = choose_checkpoint(checkpoint, xi.shape[0], n, budget_bytes or 0)
    return _Potential.apply(xi, problem, int(prec), mode)
