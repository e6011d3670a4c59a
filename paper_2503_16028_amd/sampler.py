"""SMC drivers over the C ABI: SMC-pCN-GM (Alg. 1 with the pCN-GM mutation) and SMC-GM (Alg. 3).

SMC-pCN-GM, per stage, in the order S^N P_{j+1} L_{j+1} of Sec. 2.2 (eq. (decidemuJN)):
  smc_temper    next increment h by ESS bisection (App. C), weights, log Z increment
  smc_resample  systematic resampling of the re-weighted cloud (Alg. 1)
  smc_gather    copy the selected rows
  smc_gm_fit    Gaussian mixture over the active modes (the stage input)
  smc_gmpcn_move  n_moves pCN-GM steps at the new temperature (Alg. 2)
  step size     beta <- 2 beta if acceptance > 0.3, beta / 2 if < 0.15 (App. C), beta <= 1
SMC-GM replaces the moves by smc_gm_draw: every particle becomes an independent draw from the
fitted mixture, accepted without a test, and its potential is what the next stage re-weights.
Both loops end when the cumulative temperature reaches 1.  Every step runs on the device; the
host reads back the temperature (and the acceptance count) once per stage.  With graph=True the
whole SMC-pCN-GM stage (every call above and the step-size rule) is one captured graph
(smc_sampler_graph_create) replayed once per stage, with the same bits as the calls one by one.
Random numbers: stage s draws its resampling uniform from Philox block 0x80000001 and its moves, mixture fit and
mixture draws at counters s * 2^20 (+ move index), so a run is a function of its seed alone.
"""
import math

import torch

from . import smc

STAGE_STRIDE = 1 << 20


def fit_mixture(problem, N, xi, M, seed, ctr, iters=50, var_floor=1e-3):
    """Device mixture fit of xi[0..N) (k-means++ then EM, smc_gm_fit): (logw, mean, scale)."""
    f64 = dict(dtype=torch.float64, device=xi.device)
    logw = torch.empty(M, **f64)
    mean = torch.empty(M, problem.kr, **f64)
    scale = torch.empty(M, problem.kr, **f64)
    smc.smc_gm_fit(problem, N, xi, M, iters, var_floor, seed, ctr, logw, mean, scale)
    return logw, mean, scale


def pcn_mixture(kr, device):
    """The single zero-mean unit-scale component: plain pCN."""
    return (torch.zeros(1, dtype=torch.float64, device=device),
            torch.zeros(1, kr, dtype=torch.float64, device=device),
            torch.ones(1, kr, dtype=torch.float64, device=device))


class SMCSampler:
    def __init__(self, problem, N, M, n_moves, ess_frac=0.5, beta0=0.2, prec=smc.SMC_FP32_REFINE, seed=0,
                 device="cuda", fit_iters=50, graph=False):
        self.graph = bool(graph)
        self._sg = None
        self.p, self.N, self.M, self.n_moves = problem, int(N), int(M), int(n_moves)
        self.fit_iters = int(fit_iters)
        self.ess_frac, self.beta, self.prec, self.seed = ess_frac, float(beta0), prec, int(seed)
        dev = torch.device(device)
        K = problem.K
        f64 = dict(dtype=torch.float64, device=dev)
        self.xi = torch.empty(N, K, **f64)
        self.xi2 = torch.empty(N, K, **f64)
        self.phi = torch.empty(N, **f64)
        self.phi2 = torch.empty(N, **f64)
        self.W = torch.empty(N, **f64)
        self.tau = torch.zeros(1, **f64)
        self.tau_new = torch.zeros(1, **f64)
        self.h = torch.zeros(1, **f64)
        self.log_z = torch.zeros(1, **f64)
        self.idx = torch.empty(N, dtype=torch.int32, device=dev)
        self.n_acc = torch.empty(N, dtype=torch.int32, device=dev)
        self.flags = torch.zeros(1, dtype=torch.int32, device=dev)
        self.active = torch.tensor(problem.active, dtype=torch.long, device=dev)
        self.dev = dev
        self.stage = 0
        self.log_Z = 0.0
        self.history = []

    def initialise(self):
        p, N = self.p, self.N
        smc.smc_prior_sample(p, N, self.seed, 0, self.xi)
        smc.smc_phi_batch(p, N, self.xi, None, self.prec, self.phi)

    def mixture(self):
        if self.M == 1:
            return pcn_mixture(self.p.kr, self.dev)
        return fit_mixture(self.p, self.N, self.xi, self.M, self.seed, self.stage * STAGE_STRIDE, self.fit_iters)

    def step(self):
        """One stage: temper, resample, gather, mixture, moves, step-size rule."""
        if self.graph:
            raise RuntimeError("a sampler built with graph=True runs its stages through run()")
        p, N = self.p, self.N
        self.stage += 1
        base = self.stage * STAGE_STRIDE
        smc.smc_temper(N, self.phi, self.tau, self.ess_frac, self.h, self.tau_new, self.W, self.log_z, self.flags)
        u53 = smc.smc_philox_u53(self.seed, base)
        smc.smc_resample(N, self.W, u53, self.idx, self.flags)
        smc.smc_gather(N, p.K, self.idx, self.xi, self.phi, self.xi2, self.phi2)
        self.xi, self.xi2 = self.xi2, self.xi
        self.phi, self.phi2 = self.phi2, self.phi
        self.tau.copy_(self.tau_new)
        tau = float(self.tau.item())
        self._check_step(tau)
        gm = self.mixture()
        smc.smc_gmpcn_move(p, N, gm, self.beta, tau, self.n_moves, self.seed, base, None, self.prec, self.xi,
                           self.phi, self.n_acc)
        rate = float(self.n_acc.cpu().numpy().sum()) / (N * max(1, self.n_moves))
        self.log_Z += float(self.log_z.item())
        self.history.append(dict(stage=self.stage, tau=tau, h=float(self.h.item()), beta=self.beta, rate=rate))
        if rate > 0.3:
            self.beta = min(1.0, 2.0 * self.beta)
        elif rate < 0.15:
            self.beta *= 0.5
        return tau

    def _check_step(self, tau):
        """Stop at once when the temperature cannot advance: a zero step below temperature 1 (the
        device also sets SMC_FLAG_STALL) would leave every later stage where this one is."""
        if tau < 1.0 and float(self.h.item()) == 0.0:
            raise RuntimeError("temperature bisection stalled at stage %d (tau = %.17g)" % (self.stage, tau))

    def run(self, max_stages=500, stop_after=None):
        """Run to temperature 1 (at most max_stages stages in all).  A sampler restored with
        load_state_dict continues where the saved one stopped; stop_after ends this call after that
        many stages (for a checkpoint) with the sampler still below temperature 1."""
        if self.graph:
            return self._run_graph(max_stages, stop_after)
        if self.stage == 0:
            self.initialise()
        done = 0
        while float(self.tau.item()) < 1.0 and self.stage < max_stages:
            if stop_after is not None and done >= stop_after:
                break
            self.step()
            done += 1
        if int(self.flags.item()) & smc.FLAG_STALL:
            raise RuntimeError("temperature bisection stalled")
        return dict(xi=self.xi, phi=self.phi, log_Z=self.log_Z, history=self.history)

    GRAPH_RECORD = 1024   # stages a graph-driven run can record

    def _stage_graph(self):
        """The whole-stage graph over this sampler's tensors (built once, on its own stream)."""
        if self._sg is None:
            dev, M, kr = self.dev, self.M, self.p.kr
            f64 = dict(dtype=torch.float64, device=dev)
            self._gstream = torch.cuda.Stream(device=dev)
            logw, mean, scale = pcn_mixture(kr, dev) if M == 1 else (torch.zeros(M, **f64),
                                                                    torch.zeros(M, kr, **f64),
                                                                    torch.ones(M, kr, **f64))
            self._gt = dict(xi=self.xi, phi=self.phi, xi2=self.xi2, phi2=self.phi2, W=self.W, idx=self.idx,
                            tau=self.tau, tau_new=self.tau_new, h=self.h, log_z=self.log_z,
                            beta=torch.full((1,), self.beta, **f64), logw=logw.reshape(1, M),
                            mean=mean.reshape(1, M, kr), scale=scale.reshape(1, M, kr),
                            ctr=torch.zeros(1, dtype=torch.int64, device=dev), n_acc=self.n_acc,
                            record=torch.full((self.GRAPH_RECORD, 1, 5), math.nan, **f64), flags=self.flags)
            torch.cuda.synchronize(dev)
            self._sg = smc.SamplerGraph(self.p, [self.N], M, self.n_moves, self.fit_iters, self.ess_frac, 1e-3,
                                        self.seed, STAGE_STRIDE, self.prec, self._gt, self._gstream,
                                        self.GRAPH_RECORD)
        return self._sg

    def _run_graph(self, max_stages, stop_after):
        if max_stages > self.GRAPH_RECORD:
            raise ValueError("a graph-driven run records at most %d stages" % self.GRAPH_RECORD)
        if self.stage == 0:
            self.initialise()
        g = self._stage_graph()
        t = self._gt
        first = self.stage
        torch.cuda.synchronize(self.dev)
        with torch.cuda.stream(self._gstream):
            t["ctr"].fill_((self.stage + 1) * STAGE_STRIDE)   # stage s runs at counter s * 2^20
            t["beta"].fill_(self.beta)
            done = 0
            while float(self.tau.item()) < 1.0 and self.stage < max_stages:
                if stop_after is not None and done >= stop_after:
                    break
                g.launch(self._gstream)
                self.stage += 1
                done += 1
                self._check_step(float(self.tau.item()))
            rec = t["record"][:, 0].cpu()
            self.beta = float(t["beta"].item())
        for s in range(first, self.stage):
            tau, h, beta, rate, lz = (float(v) for v in rec[s])
            self.log_Z += lz
            self.history.append(dict(stage=s + 1, tau=tau, h=h, beta=beta, rate=rate))
        torch.cuda.synchronize(self.dev)
        if int(self.flags.item()) & smc.FLAG_STALL:
            raise RuntimeError("temperature bisection stalled")
        return dict(xi=self.xi, phi=self.phi, log_Z=self.log_Z, history=self.history)

    # ---------------------------------------------------------------- checkpoint and resume
    # Every random number of a stage is keyed by (seed, stage, move, particle), so a run restored
    # from its state after any stage continues with the same bits as one never interrupted.
    def _config(self):
        return dict(kind=type(self).__name__, N=self.N, M=self.M, n_moves=self.n_moves, prec=int(self.prec),
                    seed=self.seed, ess_frac=float(self.ess_frac), fit_iters=self.fit_iters, K=int(self.p.K))

    def state_dict(self):
        """The sampler's state between stages: particles, potentials, temperature, evidence, step
        size, stage counter, device flags and history, on the host."""
        torch.cuda.synchronize(self.dev)
        return dict(config=self._config(), stage=self.stage, beta=self.beta, log_Z=self.log_Z,
                    history=[dict(h) for h in self.history], xi=self.xi.cpu(), phi=self.phi.cpu(),
                    tau=self.tau.cpu(), flags=self.flags.cpu())

    def load_state_dict(self, state):
        if state["config"] != self._config():
            raise ValueError("checkpoint of a different sampler: %r, not %r" % (state["config"], self._config()))
        self.stage, self.beta, self.log_Z = int(state["stage"]), float(state["beta"]), float(state["log_Z"])
        self.history = [dict(h) for h in state["history"]]
        self.xi.copy_(state["xi"].to(self.dev))
        self.phi.copy_(state["phi"].to(self.dev))
        self.tau.copy_(state["tau"].to(self.dev))
        self.flags.copy_(state["flags"].to(self.dev))
        torch.cuda.synchronize(self.dev)

    def save(self, path):
        torch.save(self.state_dict(), path)

    def load(self, path):
        self.load_state_dict(torch.load(path, weights_only=True))


class SMCGMSampler(SMCSampler):
    """SMC-GM (Alg. 3): re-weight, resample, fit the mixture to the resampled cloud, replace every
    particle by an independent draw from it (accepted without a test) and evaluate its potential.
    Random numbers: stage s fits and draws at counter s * 2^20 (distinct Philox blocks)."""

    def __init__(self, problem, N, M, ess_frac=0.5, prec=smc.SMC_FP32_REFINE, seed=0, device="cuda",
                 fit_iters=50):
        super().__init__(problem, N, M, 0, ess_frac=ess_frac, prec=prec, seed=seed, device=device,
                         fit_iters=fit_iters)

    def step(self):
        p, N = self.p, self.N
        self.stage += 1
        base = self.stage * STAGE_STRIDE
        smc.smc_temper(N, self.phi, self.tau, self.ess_frac, self.h, self.tau_new, self.W, self.log_z, self.flags)
        u53 = smc.smc_philox_u53(self.seed, base)
        smc.smc_resample(N, self.W, u53, self.idx, self.flags)
        smc.smc_gather(N, p.K, self.idx, self.xi, self.phi, self.xi2, self.phi2)
        self.xi, self.xi2 = self.xi2, self.xi
        self.tau.copy_(self.tau_new)
        self._check_step(float(self.tau.item()))
        gm = fit_mixture(p, N, self.xi, self.M, self.seed, base, self.fit_iters)
        smc.smc_gm_draw(p, N, gm, self.seed, base, None, self.prec, self.xi2, self.phi)
        self.xi, self.xi2 = self.xi2, self.xi
        tau = float(self.tau.item())
        self.log_Z += float(self.log_z.item())
        self.history.append(dict(stage=self.stage, tau=tau, h=float(self.h.item())))
        return tau


class MixedSampler:
    """Independent SMC-pCN-GM samplers on the grids of one problem, moved together.

    Sampler g owns the particles [off_g, off_g + N_g) and solves on grid g; it has its own
    temperature, increment, step size, resampling, mixture and evidence, exactly as SMCSampler
    would run it on that grid alone.  Each stage, every sampler still below temperature 1
    re-weights, resamples and fits its mixture on its own rows; then one smc_gmpcn_stage (captured
    once as a HIP graph) moves all of them, each move's solves one launch per grid.  A sampler
    whose temperature reaches 1 parks its particles (level SMC_LEVEL_PARKED):
    its final cloud is kept as it is and costs nothing in later stages.

    Random numbers: moves at counter s * 2^20 + m, with a particle's global index as its word, so
    sampler 0 draws exactly what SMCSampler draws with N_0 particles; sampler g takes its
    resampling uniform and mixture seeding at counter s * 2^20 + g.
    """

    def __init__(self, problem, counts, M, n_moves, ess_frac=0.5, beta0=0.2, prec=smc.SMC_FP32_REFINE, seed=0,
                 device="cuda", fit_iters=50, graph=True):
        """graph: True captures the move stage (smc_stage_graph_create) and runs tempering,
        resampling and the fits as separate calls; "stage" captures the whole stage of every
        sampler (smc_sampler_graph_create), so a stage is one launch; False makes every call."""
        G = len(counts)
        if G != len(problem.grids):
            raise ValueError("one sampler per grid of the problem (%d), got %d" % (len(problem.grids), G))
        if M < 2:
            raise ValueError("MixedSampler fits a mixture of M >= 2 components")
        self.p, self.counts, self.M, self.n_moves = problem, [int(c) for c in counts], int(M), int(n_moves)
        self.N = sum(self.counts)
        self.offs = [sum(self.counts[:g]) for g in range(G)]
        self.ess_frac, self.prec, self.seed, self.fit_iters = ess_frac, prec, int(seed), int(fit_iters)
        self.betas = [float(beta0)] * G
        dev = torch.device(device)
        f64 = dict(dtype=torch.float64, device=dev)
        N, K, kr = self.N, problem.K, problem.kr
        self.stream = torch.cuda.Stream(device=dev)
        with torch.cuda.stream(self.stream):
            self.xi = torch.empty(N, K, **f64)
            self.xi2 = torch.empty(N, K, **f64)
            self.phi = torch.empty(N, **f64)
            self.phi2 = torch.empty(N, **f64)
            self.W = torch.empty(N, **f64)
            self.idx = torch.empty(N, dtype=torch.int32, device=dev)
            self.n_acc = torch.zeros(N, dtype=torch.int32, device=dev)
            self.level = torch.cat([torch.full((c,), g, dtype=torch.int32) for g, c in enumerate(self.counts)]).to(dev)
            self.home = self.level.clone()
            self.flags = torch.zeros(1, dtype=torch.int32, device=dev)
            self.tau = torch.zeros(G, **f64)
            self.tau_new = torch.zeros(G, **f64)
            self.h = torch.zeros(G, **f64)
            self.log_z = torch.zeros(G, **f64)
            self.logw = torch.full((G, M), -math.log(M), **f64)
            self.mean = torch.zeros(G, M, kr, **f64)
            self.scale = torch.ones(G, M, kr, **f64)
            self.beta = torch.tensor(self.betas, **f64)
            self.ctr = torch.zeros(1, dtype=torch.int64, device=dev)
        self.sd = smc.stage_desc(G, self.logw, self.mean, self.scale, self.beta, self.tau, self.ctr, self.seed)
        self.stream.synchronize()
        self.graph = None
        self.whole = graph == "stage"
        self.sg = None
        if graph and not self.whole:
            self.graph = smc.StageGraph(problem, N, self.level, self.sd, self.n_moves, prec, self.xi, self.phi,
                                        self.n_acc, self.stream)
        self.stage = 0
        self.running = list(range(G))
        self.log_Z = [0.0] * G
        self.history = [[] for _ in range(G)]

    def rows(self, g):
        return slice(self.offs[g], self.offs[g] + self.counts[g])

    def initialise(self):
        with torch.cuda.stream(self.stream):
            smc.smc_prior_sample(self.p, self.N, self.seed, 0, self.xi)
            smc.smc_phi_batch(self.p, self.N, self.xi, self.level, self.prec, self.phi)

    GRAPH_RECORD = 1024   # stages a whole-stage graph records

    def _whole_graph(self):
        if self.sg is None:
            G = len(self.counts)
            f64 = dict(dtype=torch.float64, device=self.xi.device)
            with torch.cuda.stream(self.stream):
                self.record = torch.full((self.GRAPH_RECORD, G, 5), math.nan, **f64)
            self.stream.synchronize()
            t = dict(xi=self.xi, phi=self.phi, xi2=self.xi2, phi2=self.phi2, W=self.W, idx=self.idx, tau=self.tau,
                     tau_new=self.tau_new, h=self.h, log_z=self.log_z, beta=self.beta, logw=self.logw,
                     mean=self.mean, scale=self.scale, ctr=self.ctr, level=self.level, n_acc=self.n_acc,
                     record=self.record, flags=self.flags)
            self.sg = smc.SamplerGraph(self.p, self.counts, self.M, self.n_moves, self.fit_iters, self.ess_frac,
                                       1e-3, self.seed, STAGE_STRIDE, self.prec, t, self.stream, self.GRAPH_RECORD)
        return self.sg

    def _step_whole(self):
        """One stage of every sampler as one launch of the whole-stage graph; the host reads the
        temperatures to stop and to catch a stalled step."""
        g = self._whole_graph()
        self.stage += 1
        with torch.cuda.stream(self.stream):
            if self.stage == 1:
                self.ctr.fill_(STAGE_STRIDE)
                self.beta.copy_(torch.tensor(self.betas, dtype=torch.float64))
            g.launch(self.stream)
            taus = self.tau.cpu().numpy()
            hs = self.h.cpu().numpy()
        for k in self.running:
            if taus[k] < 1.0 and hs[k] == 0.0:
                raise RuntimeError("temperature bisection of sampler %d stalled at stage %d" % (k, self.stage))
        self.running = [k for k in self.running if taus[k] < 1.0]
        return len(self.running)

    def _collect_whole(self):
        rec = self.record.cpu().numpy()
        for g in range(len(self.counts)):
            for s in range(self.stage):
                tau, h, beta, rate, lz = (float(v) for v in rec[s, g])
                if math.isnan(tau):
                    continue
                self.log_Z[g] += lz
                self.history[g].append(dict(stage=s + 1, tau=tau, h=h, beta=beta, rate=rate))
        self.betas = [float(b) for b in self.beta.cpu().numpy()]

    def step(self):
        """One stage of every running sampler: temper, resample, gather, fit; then one move stage."""
        if self.whole:
            return self._step_whole()
        p, K = self.p, self.p.K
        self.stage += 1
        base = self.stage * STAGE_STRIDE
        with torch.cuda.stream(self.stream):
            for g in self.running:
                r, n = self.rows(g), self.counts[g]
                one = slice(g, g + 1)
                smc.smc_temper(n, self.phi[r], self.tau[one], self.ess_frac, self.h[one], self.tau_new[one], self.W[r],
                               self.log_z[one], self.flags)
                smc.smc_resample(n, self.W[r], smc.smc_philox_u53(self.seed, base + g), self.idx[r], self.flags)
                smc.smc_gather(n, K, self.idx[r], self.xi[r], self.phi[r], self.xi2[r], self.phi2[r])
                self.xi[r].copy_(self.xi2[r])            # the captured stage reads xi and phi in place
                self.phi[r].copy_(self.phi2[r])
                self.tau[one].copy_(self.tau_new[one])
                smc.smc_gm_fit(p, n, self.xi[r], self.M, self.fit_iters, 1e-3, self.seed, base + g, self.logw[g],
                               self.mean[g], self.scale[g])
            self.beta.copy_(torch.tensor(self.betas, dtype=torch.float64))
            self.ctr.fill_(base)
            if self.graph is not None:
                self.graph.launch(self.stream)
            else:
                smc.smc_gmpcn_stage(p, self.N, self.level, self.sd, self.n_moves, self.prec, self.xi, self.phi,
                                    self.n_acc)
            acc = self.n_acc.cpu().numpy()
            taus = self.tau.cpu().numpy()
            hs = self.h.cpu().numpy()
            lzs = self.log_z.cpu().numpy()
            for g in self.running:
                if taus[g] < 1.0 and hs[g] == 0.0:
                    raise RuntimeError("temperature bisection of sampler %d stalled at stage %d" % (g, self.stage))
            for g in list(self.running):
                r = self.rows(g)
                rate = float(acc[r].sum()) / (self.counts[g] * max(1, self.n_moves))
                self.log_Z[g] += float(lzs[g])
                self.history[g].append(dict(stage=self.stage, tau=float(taus[g]), h=float(hs[g]), beta=self.betas[g],
                                            rate=rate))
                if rate > 0.3:
                    self.betas[g] = min(1.0, 2.0 * self.betas[g])
                elif rate < 0.15:
                    self.betas[g] *= 0.5
                if taus[g] >= 1.0:
                    self.level[r].fill_(smc.LEVEL_PARKED)
                    self.running.remove(g)
            self.stream.synchronize()
        return len(self.running)

    def run(self, max_stages=500):
        if self.whole and max_stages > self.GRAPH_RECORD:
            raise ValueError("a whole-stage graph records at most %d stages" % self.GRAPH_RECORD)
        self.initialise()
        for _ in range(max_stages):
            if self.step() == 0:
                break
        self.stream.synchronize()
        if self.whole:
            self._collect_whole()
        if int(self.flags.item()) & smc.FLAG_STALL:
            raise RuntimeError("temperature bisection stalled")
        return [dict(xi=self.xi[self.rows(g)], phi=self.phi[self.rows(g)], log_Z=self.log_Z[g],
                     history=self.history[g]) for g in range(len(self.counts))]

    def close(self):
        if self.graph is not None:
            self.graph.close()
            self.graph = None
        if self.sg is not None:
            self.sg.close()
            self.sg = None
