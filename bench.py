"""Benchmark: particle GM-pCN moves per second (forward solve + potential) on one MI355X.

Workload: the 2D Darcy problem on a 128 x 128 grid, N = 4096 particles, an 8-component
mixture over 64 active modes, 20 pCN-GM moves per tempering stage, 10 observations mirrored
about x = 1/2 (synthetic data from tests/golden/problem_c3.json).  A step is one tempering
stage of the move phase: re-weighting and ESS bisection, systematic resampling, the row
gather and 20 pCN-GM moves of every particle (proposal, KL synthesis, forward solve,
potential, Metropolis decision).  The mixture fit between resampling and the moves is the
stage's input and is not timed.  Inputs are resident on the device before timing starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-variants]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
PROBLEM = os.path.join(ROOT, "tests", "golden", "problem_c3.json")
N, M, N_MOVES, GRID = 4096, 8, 20, 128
FLOPS_PER_UNKNOWN_ITER = 18     # one scaled-CG iteration per interior unknown, product-form stencil
FLOPS_PER_UNKNOWN_SWEEP = 16    # one FP64 residual evaluation per interior unknown
FP32_VECTOR_PEAK = 157.3e12     # MI355X published FP32 vector peak
F16_MFMA_PEAK = 2.5e15          # MI355X published dense fp16 and bf16 matrix peak
HBM_PEAK = 8.0e12               # MI355X HBM3E peak, bytes/s
LDS_PEAK = 256 * 128 * 2.4e9    # LDS bandwidth: 256 compute units x 128 bytes per clock x 2.4 GHz
L2_PEAK = 8 * 16 * 128 * 2.4e9  # L2: 8 XCDs x 16 channels x 128 bytes per clock x 2.4 GHz


def lds_bytes_per_solve(iters, apps, sweeps, n=GRID):
    """LDS bytes one 128^2 on-chip solve moves (32 rows per thread), from the kernel's access pattern:
    per preconditioner application the FP16 staging of r (2 n^2 bytes), four products that each read
    their FP16 operand once per strip group (4 groups: 8 n^2), three FP16 results (2 n^2 each), the
    FP32 result (4 n^2) and the solver reading it back (4 n^2); per CG iteration the published t p
    (4 n^2) and its four neighbour reads (16 n^2); per FP64 sweep the residual and the update through
    the strip's FP32 LDS slots (16 n^2)."""
    n2 = float(n * n)
    per_app = 2 * n2 + 4 * 8 * n2 + 3 * 2 * n2 + 4 * n2 + 4 * n2
    per_iter = 4 * n2 + 16 * n2
    per_sweep = 16 * n2
    return apps * per_app + iters * per_iter + sweeps * per_sweep


COUNTERS = os.path.join(ROOT, "profiles", "cg_onchip_128x32_fastpoisson_c3_counters.md")
SOLVER_SOURCES = [os.path.join(ROOT, "paper_2503_16028_amd", "csrc", f) for f in ("k_solve.hip", "common.hpp")]


def measured_traffic(tile, field="traffic_bytes_per_launch"):
    """Bytes per solve launch from the committed counter summary: HBM (FETCH_SIZE and WRITE_SIZE,
    each calibrated against a copy of known size), or with `field` the L2 request bytes
    (TCP_TCC_READ_REQ and TCP_TCC_WRITE_REQ times the request sizes a copy shows); None once the
    solver sources or the tile shape differ from what was profiled."""
    import hashlib
    try:
        fields = dict(l.strip().split(" = ", 1) for l in open(COUNTERS) if " = " in l and l.startswith("    "))
        h = hashlib.sha256()
        for f in SOLVER_SOURCES:
            h.update(open(f, "rb").read())
        if h.hexdigest() != fields.get("source_sha256") or int(fields.get("tile_rows", -1)) != tile:
            return None
        return float(fields[field])
    except (OSError, ValueError, KeyError):
        return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(d, sample_per_worker=100):
    """The oracle, as it stands, on a bounded sample of the workload: `workers` processes each
    run one pCN-GM move for `sample_per_worker` particles (one sparse direct solve each).  The
    pool takes every core this process may run on, up to 16: a one-GPU share of the host."""
    import concurrent.futures
    import multiprocessing as mp
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    workers = max(1, min(16, usable))
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with concurrent.futures.ProcessPoolExecutor(workers, mp_context=ctx) as ex:
        res = list(ex.map(_oracle_chunk, [(d, w, sample_per_worker) for w in range(workers)]))
    wall = time.perf_counter() - t0
    moves = sum(r[0] for r in res)
    move_wall = max(r[1] for r in res)
    return dict(value=moves / move_wall, unit="particle-moves/s", cores=workers, kind="oracle",
                sample="%d particles x 1 pCN-GM move at 128^2 (M=8) over %d processes; %.1f s wall incl. setup"
                       % (moves, workers, wall),
                cpu_model=cpu_model(), cpus_usable=usable, cpus_visible=os.cpu_count())


def _oracle_chunk(args):
    d, w, n = args
    os.environ["OMP_NUM_THREADS"] = "1"
    import numpy as np
    from oracle.forward import phi as phi_of
    from oracle.gmfit import fit
    from oracle.moves import GM, gmpcn_moves, prior_sample
    from oracle.problem import Problem
    op = Problem(d)
    ids = np.arange(w * n, (w + 1) * n)
    xi = prior_sample(op.K, (w + 1) * n, 2503, 0)[ids]
    ph = np.array([phi_of(op, x, GRID) for x in xi])
    logw, mean, var = fit(xi[:, op.active()], M, seed=0, iters=10)
    gm = GM(logw, mean, var, op.active(), op.K)
    t0 = time.perf_counter()
    gmpcn_moves(op, GRID, xi, ph, gm, 0.2, 0.05, 1, 9, 500, ids=ids)
    return n, time.perf_counter() - t0


def pcnl_variant(dev, N=2048, n_moves=20):
    """pCN-Langevin moves at 128^2 (each proposal: forward and adjoint solves, gradient synthesis)."""
    import numpy as np
    import torch
    from paper_2503_16028_amd import smc
    d = json.load(open(os.path.join(ROOT, "tests", "golden", "problem_c4.json")))
    p = smc.Problem(d, N, tol64=1e-10, tol_inner=1e-3)
    xi = torch.empty(N, p.K, dtype=torch.float64, device=dev)
    smc.smc_prior_sample(p, N, 2503, 0, xi)
    xi.mul_(0.5)
    phi = torch.empty(N, dtype=torch.float64, device=dev)
    g = torch.empty(N, p.K, dtype=torch.float64, device=dev)
    acc = torch.empty(N, dtype=torch.int32, device=dev)
    smc.smc_value_and_grad(p, N, xi, smc.SMC_FP32_REFINE, None, phi, g)
    tau = float(min(1.0, 2.0 / phi.median().item()))
    smc.smc_pcnl_move(p, N, 0.2, tau, 1, 7, 1, smc.SMC_FP32_REFINE, xi, phi, g, acc)   # warm-up
    torch.cuda.synchronize()
    smc.smc_profile(p, 1)
    t0 = time.perf_counter()
    smc.smc_pcnl_move(p, N, 0.2, tau, n_moves, 7, 100, smc.SMC_FP32_REFINE, xi, phi, g, acc)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    pr = smc.smc_profile_read(p)
    smc.smc_profile(p, 0)
    return {"pcnl_128_N2048_moves_per_s": N * n_moves / dt,
            "pcnl_accept_rate": float(acc.sum().item()) / (N * n_moves),
            "pcnl_solve_ms_per_launch": pr["ms"] / max(1, pr["launches"]),
            "pcnl_cg_iters_per_solve": pr["iters"] / max(1, pr["solves"])}


def smc_gm_variant(dev, N=4096, M=8, stages=3):
    """SMC-GM (Alg. 3) at 128^2: per stage re-weighting, resampling, the device mixture fit (k-means++
    and 50 EM steps) and N fresh draws with their solves; and the fit alone."""
    import torch
    from paper_2503_16028_amd import smc
    from paper_2503_16028_amd.sampler import SMCGMSampler, fit_mixture
    d = json.load(open(os.path.join(ROOT, "tests", "golden", "problem_c3.json")))
    p = smc.Problem(d, N, tol64=1e-10, tol_inner=1e-3)
    s = SMCGMSampler(p, N, M, ess_frac=0.5, prec=smc.SMC_FP32_REFINE, seed=2503, device=dev)
    s.initialise()
    s.step()                                        # warm-up stage
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(stages):
        s.step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / stages
    reps = 5
    fit_mixture(p, N, s.xi, M, 1, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(reps):
        fit_mixture(p, N, s.xi, M, 1, 2 + r)
    torch.cuda.synchronize()
    fit_ms = 1e3 * (time.perf_counter() - t0) / reps
    return {"smc_gm_128_N4096_particles_per_s": N / dt, "smc_gm_stage_ms": 1e3 * dt,
            "gm_fit_ms_N4096_M8_50em": fit_ms}


def example1_variant(dev, N=20000, M=8, chain=200, K=64, sigma=0.1):
    """The paper's Example 1 (Sec. 3.1, no PDE): whole SMC-GM and SMC-pCN-GM runs of N = 20000
    particles (the paper's sample count) on the four-term L^2 likelihood with K = 64 cosine modes;
    SMC-pCN-GM with the paper's chain length of 200 moves per stage."""
    import numpy as np
    import torch
    from paper_2503_16028_amd import smc
    from paper_2503_16028_amd.sampler import SMCGMSampler, SMCSampler
    c = np.zeros((4, K))                  # f = cos(pi x), -cos(pi x), cos(2 pi x), cos(3 pi x) on phi_k = sqrt(2) cos(k pi x)
    for i, (k, sg) in enumerate(((1, 1.0), (1, -1.0), (2, 1.0), (3, 1.0))):
        c[i, k] = sg / np.sqrt(2.0)
    p = smc.L2MixProblem(K, K, 0.01, c, sigma, N)
    out = {}
    for name, make in (("smc_gm", lambda: SMCGMSampler(p, N, M, seed=1, device=dev)),
                       ("smc_pcngm_chain200", lambda: SMCSampler(p, N, M, chain, beta0=0.5, seed=1, device=dev))):
        make().run()                      # warm-up run
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = make().run()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out["example1_%s_N20000_samples_per_s" % name] = N / dt
        out["example1_%s_run_s" % name] = dt
        out["example1_%s_stages" % name] = len(r["history"])
        if name != "smc_gm":
            out["example1_%s_moves_per_s" % name] = N * chain * len(r["history"]) / dt
    return out


def runs_variant(dev):
    """Whole SMC-pCN-GM runs to temperature 1 of the 1D workload (64 intervals, N = 256, plain pCN, 10
    moves per stage, FP64) and of the 64^2 workload (N = 1024, M = 4, 20 moves per stage) in FP64 and in
    FP32 with refinement: wall time of each run after one warm-up run, and the moves per second."""
    import torch
    from paper_2503_16028_amd import smc
    from paper_2503_16028_amd.sampler import SMCSampler
    out = {}
    for name, precs in (("c1", (("fp64", smc.SMC_FP64),)),
                        ("c2", (("fp64", smc.SMC_FP64), ("fp32_refine", smc.SMC_FP32_REFINE)))):
        d = json.load(open(os.path.join(ROOT, "tests", "golden", "problem_%s.json" % name)))
        N, M, nm = int(d["N"]), int(d["M"]), int(d["n_moves"])
        p = smc.Problem(d, N, tol64=1e-10, tol_inner=1e-3)
        for tag, prec in precs:
            make = lambda: SMCSampler(p, N, M, nm, ess_frac=d["ess_frac"], beta0=d["beta0"], prec=prec, seed=0,
                                      device=dev)
            make().run()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = make().run()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            stages = len(r["history"])
            out["%s_%s_run_s" % (name, tag)] = dt
            out["%s_%s_stages" % (name, tag)] = stages
            out["%s_%s_moves_per_s" % (name, tag)] = N * nm * stages / dt
        p.close()
    return out


def mixed_variant(dev, counts=(4096, 3072, 1024), n_moves=20, stages=2):
    """Three samplers on 64^2, 128^2 and 256^2 (N = 8192) moved by one captured stage graph."""
    import numpy as np
    import torch
    from paper_2503_16028_amd import smc
    d = json.load(open(os.path.join(ROOT, "tests", "golden", "problem_c5.json")))
    N = sum(counts)
    p = smc.Problem(d, N, tol64=1e-10, tol_inner=1e-3)
    level = torch.cat([torch.full((c,), l, dtype=torch.int32) for l, c in enumerate(counts)]).to(dev)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        xi = torch.empty(N, p.K, dtype=torch.float64, device=dev)
        smc.smc_prior_sample(p, N, 2503, 0, xi)
        G = torch.empty(N, p.n_obs, dtype=torch.float64, device=dev)
        phi = torch.empty(N, dtype=torch.float64, device=dev)
        smc.smc_forward_batch(p, N, xi, level, smc.SMC_FP32_REFINE, G)
        smc.smc_potential(p, N, G, phi)
        M, kr = 8, p.kr
        logw = torch.full((3, M), -float(np.log(M)), dtype=torch.float64, device=dev)
        mean = torch.zeros(3, M, kr, dtype=torch.float64, device=dev)
        scale = torch.ones(3, M, kr, dtype=torch.float64, device=dev)
        beta = torch.full((3,), 0.2, dtype=torch.float64, device=dev)
        tau = torch.full((3,), 1e-4, dtype=torch.float64, device=dev)
        ctr = torch.zeros(1, dtype=torch.int64, device=dev)
        acc = torch.empty(N, dtype=torch.int32, device=dev)
        sd = smc.stage_desc(3, logw, mean, scale, beta, tau, ctr, 11)
        graph = smc.StageGraph(p, N, level, sd, n_moves, smc.SMC_FP32_REFINE, xi, phi, acc, s)
        graph.launch(s)                       # warm-up stage
        s.synchronize()
        t0 = time.perf_counter()
        for k in range(stages):
            ctr.add_(1 << 20)
            graph.launch(s)
        s.synchronize()
        dt = time.perf_counter() - t0
        graph.close()
    return {"mixed_64_128_256_N8192_moves_per_s": N * n_moves * stages / dt,
            "mixed_stage_ms": 1e3 * dt / stages,
            "mixed_counts": list(counts)}


def stage_graph_variant(dev, N=4096, M=8, n_moves=20, counts=(4096, 3072, 1024), mixed_stages=3):
    """Whole SMC-pCN-GM runs (every stage: tempering, resampling, gather, mixture fit, moves, step
    rule) made call by call and as one captured graph per stage; the same bits either way."""
    import torch
    from paper_2503_16028_amd import smc
    from paper_2503_16028_amd.sampler import MixedSampler, SMCSampler
    d = json.load(open(os.path.join(ROOT, "tests", "golden", "problem_c3.json")))
    p = smc.Problem(d, N, tol64=1e-10, tol_inner=1e-3)
    out, runs = {}, []
    for graph in (False, True):
        s = SMCSampler(p, N, M, n_moves, seed=2503, graph=graph, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.run()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        runs.append(s)
        key = "graph" if graph else "calls"
        out["c3_run_%s_s" % key] = dt
        out["c3_stage_%s_ms" % key] = 1e3 * dt / max(1, s.stage)
    out["c3_run_stages"] = runs[0].stage
    out["c3_graph_same_bits"] = bool(torch.equal(runs[0].xi, runs[1].xi) and runs[0].log_Z == runs[1].log_Z)
    p.close()
    d5 = json.load(open(os.path.join(ROOT, "tests", "golden", "problem_c5.json")))
    p5 = smc.Problem(d5, sum(counts), tol64=1e-10, tol_inner=1e-3)
    for graph in (True, "stage"):
        ms = MixedSampler(p5, counts, M, n_moves, seed=2503, graph=graph, device=dev)
        ms.initialise()
        ms.stream.synchronize()
        t0 = time.perf_counter()
        for _ in range(mixed_stages):
            ms.step()
        ms.stream.synchronize()
        dt = time.perf_counter() - t0
        key = "whole_graph" if graph == "stage" else "moves_graph"
        out["mixed_stage_%s_ms" % key] = 1e3 * dt / mixed_stages
        ms.close()
    p5.close()
    return out


SOLVE_ONLY = {
    # name: (problem, grids, particles per grid, precision)
    "c3_fp32": ("c3", [128], [4096], 1),
    "c3_fp64": ("c3", [128], [4096], 0),
    "c5_256_fp32": ("c5", [256], [1024], 1),
    "c5_mixed_fp32": ("c5", [64, 128, 256], [4096, 3072, 1024], 1),
    "c4_adjoint_fp32": ("c4", [128], [2048], 1),
}


def solve_only(name, reps, copy_probe):
    """Forward solves (synthesis and solve) of one workload, `reps` timed launches after one warm-up:
    the command the solvers' counter profiles are taken with.  c5_mixed_fp32 solves the three grids
    in one persistent launch (a level map); c4_adjoint_fp32 also solves the adjoint (the gradient)."""
    import torch
    from paper_2503_16028_amd import smc
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    prob, grids, counts, prec = SOLVE_ONLY[name]
    d = json.load(open(os.path.join(ROOT, "tests", "golden", "problem_%s.json" % prob)))
    N = sum(counts)
    p = smc.Problem(d, N, grids=grids, tol64=1e-10, tol_inner=1e-3)
    xi = torch.empty(N, p.K, dtype=torch.float64, device=dev)
    smc.smc_prior_sample(p, N, 2503, 0, xi)
    level = None
    if len(grids) > 1:
        level = torch.cat([torch.full((c,), l, dtype=torch.int32) for l, c in enumerate(counts)]).to(dev)
    G = torch.empty(N, p.n_obs, dtype=torch.float64, device=dev)
    grad = torch.empty(N, p.K, dtype=torch.float64, device=dev)
    phi = torch.empty(N, dtype=torch.float64, device=dev)

    def launch():
        if name.startswith("c4_adjoint"):
            smc.smc_value_and_grad(p, N, xi, prec, None, phi, grad)
        else:
            smc.smc_forward_batch(p, N, xi, level, prec, G)

    if copy_probe:
        src = torch.ones(32 << 20, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        del src, dst
    launch()
    torch.cuda.synchronize()
    smc.smc_profile(p, 1)
    for _ in range(reps):
        launch()
    pr = smc.smc_profile_read(p)
    smc.smc_profile(p, 0)
    assert smc.smc_status_flags(p) == 0
    print(json.dumps({"solve_only": name, "particles": counts, "grids": grids, "precision": "fp64" if prec == 0 else
                      "fp32+refine", "launches": pr["launches"], "ms_per_launch": pr["ms"] / max(1, pr["launches"]),
                      "cg_iters_per_solve": pr["iters"] / max(1, pr["solves"]),
                      "sweeps_per_solve": pr["sweeps"] / max(1, pr["solves"]),
                      "precond_apps_per_solve": pr["precond_apps"] / max(1, pr["solves"])}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--solve-only", choices=sorted(SOLVE_ONLY),
                    help="time only the forward solves of one workload (the solvers' profiling command)")
    ap.add_argument("--reps", type=int, default=5, help="timed launches of --solve-only")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--moves", type=int, default=N_MOVES, help="moves per stage (profiling runs use fewer)")
    ap.add_argument("--tile", type=int, default=0,
                    help="rows per thread of the 128^2 solver (0: autotune before timing)")
    ap.add_argument("--precond", choices=["auto", "jacobi"], default="auto",
                    help="preconditioner of the solves (jacobi: the Jacobi-scaled CG alone, a comparison point)")
    ap.add_argument("--fused-stage", action="store_true",
                    help="one persistent launch per stage instead of one launch per move step (comparison)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also copy 256 MiB device-to-device, to calibrate memory-traffic counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs the move stage on one GPU only (--gpus %d requested); sharding the particles "
              "across GPUs is not implemented" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.solve_only:
        solve_only(args.solve_only, args.reps, args.copy_probe)
        return
    d = json.load(open(PROBLEM))
    cpu = None if args.no_cpu else cpu_baseline(d)    # before anything touches the GPU

    import numpy as np
    import torch
    from paper_2503_16028_amd import smc
    from paper_2503_16028_amd.sampler import SMCSampler, fit_mixture

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    fast_poisson = args.precond == "auto"
    p = smc.Problem(d, N, tol64=1e-10, tol_inner=1e-3,
                    precond=smc.PRECOND_AUTO if fast_poisson else smc.PRECOND_JACOBI)
    unknowns = (GRID - 1) ** 2
    if args.fused_stage:
        smc.smc_set_stage_fusion(p, True)
    if not fast_poisson:
        tile, tile_ms = 16, {}   # the Jacobi-only 128^2 solver has one shape, 16 rows per thread
    elif args.tile:
        smc.smc_set_tile(p, 0, args.tile)
        tile, tile_ms = args.tile, {}
    else:
        tile, tile_ms = smc.smc_autotune(p, 0, N, reps=2)  # tile shape of the solver, before timing

    def stage_loop(prec, steps, warmup, n_moves):
        s = SMCSampler(p, N, M, n_moves, ess_frac=0.5, beta0=0.2, prec=prec, seed=2503, device=dev)
        s.initialise()
        timed, solve = 0.0, None
        for k in range(warmup + steps):
            if k == warmup:
                smc.smc_profile(p, 1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.stage += 1
            smc.smc_temper(N, s.phi, s.tau, s.ess_frac, s.h, s.tau_new, s.W, s.log_z, s.flags)
            u53 = int(np.random.default_rng([s.seed, s.stage]).integers(0, 1 << 53))
            smc.smc_resample(N, s.W, u53, s.idx, s.flags)
            smc.smc_gather(N, p.K, s.idx, s.xi, s.phi, s.xi2, s.phi2)
            s.xi, s.xi2, s.phi, s.phi2 = s.xi2, s.xi, s.phi2, s.phi
            s.tau.copy_(s.tau_new)
            tau = float(s.tau.item())
            t1 = time.perf_counter()
            gm = fit_mixture(p, N, s.xi, M, s.seed, s.stage << 20)   # stage input: mixture fit (not timed)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            smc.smc_gmpcn_move(p, N, gm, s.beta, tau, n_moves, s.seed, s.stage << 20, None, prec, s.xi, s.phi,
                               s.n_acc)
            rate = float(s.n_acc.cpu().numpy().sum()) / (N * n_moves)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            s.beta = min(1.0, 2 * s.beta) if rate > 0.3 else (0.5 * s.beta if rate < 0.15 else s.beta)
            if k >= warmup:
                timed += (t1 - t0) + (t3 - t2)
        solve = smc.smc_profile_read(p)
        smc.smc_profile(p, 0)
        return timed, solve, s

    if args.copy_probe:
        src = torch.ones(32 << 20, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    t32, prof32, s32 = stage_loop(smc.SMC_FP32_REFINE, args.steps, args.warmup, args.moves)
    moves = N * args.moves * args.steps
    value = moves / t32
    launches = max(1, prof32["launches"])
    kernel_ms = prof32["ms"] / launches
    # algorithmic work of the solve launches: four n^3 sine-transform products (2 FLOP per
    # multiply-add) per preconditioner application on the matrix cores, plus the CG vector work
    mfma_flops = 8.0 * GRID ** 3 * prof32["precond_apps"]
    valu_flops = unknowns * (FLOPS_PER_UNKNOWN_ITER * prof32["iters"] + FLOPS_PER_UNKNOWN_SWEEP * prof32["sweeps"])
    achieved = mfma_flops / (prof32["ms"] * 1e-3)
    variants = {}
    if not args.no_variants:
        variants.update(pcnl_variant(dev))
        variants.update(smc_gm_variant(dev))
        variants.update(example1_variant(dev))
        variants.update(mixed_variant(dev))
        variants.update(runs_variant(dev))
        variants.update(stage_graph_variant(dev))
        # FP64 conjugate gradients with the same preconditioner, on the headline's protocol: the same
        # seed, stages, warm-up and moves per stage, so the ratio compares precisions alone
        t64, prof64, _ = stage_loop(smc.SMC_FP64, args.steps, args.warmup, args.moves)
        variants["fp64_batched_moves_per_s"] = N * args.moves * args.steps / t64
        variants["fp64_batched_solve_ms_per_launch"] = prof64["ms"] / max(1, prof64["launches"])
        variants["fp64_batched_protocol"] = "%d stages of %d moves after %d warm-up stages" % (
            args.steps, args.moves, args.warmup)
        variants["fp32_refine_over_fp64"] = value / variants["fp64_batched_moves_per_s"]
        # the same stages as one persistent launch each (every move of a particle in one workgroup)
        smc.smc_set_stage_fusion(p, True)
        tf, _, _ = stage_loop(smc.SMC_FP32_REFINE, args.steps, args.warmup, args.moves)
        smc.smc_set_stage_fusion(p, False)
        variants["fused_stage_moves_per_s"] = N * args.moves * args.steps / tf
        # the same kernels launched once per particle, FP64
        S, nm, cap = 16, 1, 20.0       # particles, moves each, seconds cap
        xi = torch.empty(S, p.K, dtype=torch.float64, device=dev)
        smc.smc_prior_sample(p, S, 2503, 0, xi)
        G = torch.empty(S, p.n_obs, dtype=torch.float64, device=dev)
        phi = torch.empty(S, dtype=torch.float64, device=dev)
        smc.smc_forward_batch(p, S, xi, None, smc.SMC_FP64, G)
        smc.smc_potential(p, S, G, phi)
        gm = tuple(t.contiguous() for t in (torch.zeros(M, dtype=torch.float64, device=dev) - np.log(M),
                                             torch.zeros(M, p.kr, dtype=torch.float64, device=dev),
                                             torch.ones(M, p.kr, dtype=torch.float64, device=dev)))
        acc = torch.empty(S, dtype=torch.int32, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = 0
        for k in range(S):
            smc.smc_gmpcn_move(p, 1, gm, 0.2, 0.5, nm, 7, 100, None, smc.SMC_FP64, xi[k:k + 1], phi[k:k + 1],
                               acc[k:k + 1])
            torch.cuda.synchronize()
            done += 1
            if time.perf_counter() - t0 > cap:
                break
        variants["fp64_per_particle_moves_per_s"] = done * nm / (time.perf_counter() - t0)
        variants["fp64_per_particle_sample"] = "%d particles x %d move, one launch sequence per particle" % (done, nm)
        variants["fp32_refine_batched_moves_per_s"] = value
    traffic = measured_traffic(tile) if fast_poisson else None
    l2_bytes = measured_traffic(tile, "l2_request_bytes_per_launch") if fast_poisson else None
    # HBM roofline of the solve (the forward solves' target is a fraction of the HBM peak): bytes per
    # launch from the committed FETCH_SIZE/WRITE_SIZE summary of this kernel, over the live launch
    # time.  The streaming byte model of a Jacobi-PCG solve, U (48 I + 20 S + 12) bytes per solve,
    # would exceed the HBM peak here: the CG vectors and the transforms stay on chip, and only the
    # FP64 refinement (field, iterate, scaling) crosses to memory.
    stream_model = N * (GRID ** 2) * (
        48.0 * prof32["iters"] / max(1, prof32["solves"]) + 20.0 * prof32["sweeps"] / max(1, prof32["solves"]) + 12.0)
    hbm_achieved = None if traffic is None else traffic / (kernel_ms * 1e-3)
    solves32 = max(1, prof32["solves"])
    lds_launch = N * lds_bytes_per_solve(prof32["iters"] / solves32, prof32["precond_apps"] / solves32,
                                         prof32["sweeps"] / solves32)
    out = {
        "metric": "particle GM-pCN moves/sec (solve+Phi) at 128^2, N=4096; FP32+refine vs FP64",
        "value": value,
        "unit": "particle-moves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t32 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 CG + f64 refinement",
        "data": "synthetic",
        "config": {"workload": "2D Darcy 128x128, N=4096 particles, 8-component GM-pCN over 64 active modes, "
                               "20 moves per tempering stage, 10 mirrored observations",
                   "grid": GRID, "particles": N, "mixture": M, "moves_per_stage": args.moves,
                   "solver": ("Jacobi-scaled CG in FP32, fast-Poisson (FP16 MFMA sine transform) preconditioner, "
                              "inside FP64 residual refinement to 1e-10") if fast_poisson else
                             "Jacobi-scaled CG in FP32 (no further preconditioner), inside FP64 residual refinement "
                             "to 1e-10"},
        "roofline": {"bound": "hbm",
                     "achieved": None if hbm_achieved is None else hbm_achieved / 1e9,
                     "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": None if hbm_achieved is None else hbm_achieved / HBM_PEAK,
                     "traffic": traffic,
                     "traffic_unit": "bytes per launch (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, calibrated on a copy)",
                     "kernel": "cg_onchip<float,128,%d,%s>" % (tile, "fast-Poisson" if fast_poisson else "Jacobi"),
                     "kernel_ms_per_launch": kernel_ms,
                     "streaming_model_bytes_per_launch": stream_model,
                     "streaming_model_frac": stream_model / (kernel_ms * 1e-3) / HBM_PEAK,
                     "lds": {"bytes_per_launch": lds_launch, "achieved": lds_launch / (kernel_ms * 1e-3) / 1e12,
                             "peak": LDS_PEAK / 1e12, "unit": "TB/s",
                             "frac": lds_launch / (kernel_ms * 1e-3) / LDS_PEAK},
                     "l2": None if l2_bytes is None else
                     {"bytes_per_launch": l2_bytes, "achieved": l2_bytes / (kernel_ms * 1e-3) / 1e12,
                      "peak": L2_PEAK / 1e12, "unit": "TB/s", "frac": l2_bytes / (kernel_ms * 1e-3) / L2_PEAK,
                      "counts": "vector-cache requests to L2 (counters), 128-byte reads and 64-byte writes"},
                     "mfma": {"achieved": achieved / 1e12, "peak": F16_MFMA_PEAK / 1e12, "unit": "TFLOP/s",
                              "frac": achieved / F16_MFMA_PEAK,
                              "counts": "8 n^3 FLOP of dense sine-transform products per preconditioner application"},
                     "valu_tflops": valu_flops / (prof32["ms"] * 1e-3) / 1e12,
                     "cg_iters_per_solve": prof32["iters"] / max(1, prof32["solves"]),
                     "precond_apps_per_solve": prof32["precond_apps"] / max(1, prof32["solves"]),
                     "sweeps_per_solve": prof32["sweeps"] / max(1, prof32["solves"])},
        "autotune": {"rows_per_thread": tile, "ms_per_forward_launch": {str(k): v for k, v in tile_ms.items()}},
        "cpu_baseline": cpu,
        "variants": variants,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
