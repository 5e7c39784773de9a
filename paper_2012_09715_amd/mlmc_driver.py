"""Nested multilevel Monte Carlo driver (Section 4.1) over the fused level
kernels of libaicdf.

The regular estimator uses the EXACT kind on every level; the nested one
uses the APPROX kind (two-way differences with approximate normals; for CIR
the trained surrogate or Section 5.1's piecewise-polynomial chi-squared
table) plus the CORRECTION kind (four-way differences).  Per
level the driver
  1. runs pilot calls of every kind and reads the variance v of Y and the
     device time c per path (HIP events around the level kernel),
  2. asks the library for the optimal allocation at RMSE eps
     (mlmc_allocate: T^, T~, m^_l, m~_l, M~_l),
  3. runs the allocated path counts (continuing each stream after the pilot
     paths) and forms the estimators and their measured device times.
The speed-up is reported three ways: T^/T~ from the cost formula with the
measured (v, c); the ratio of the summed device times of the two estimators'
level calls at the same target RMSE, run one after another; and the ratio of
their wall-clock times when each estimator's level calls are enqueued from
one host thread on a few streams with the library's stream-ordered calls and
waited for once (the latency-bound high levels, a few hundred paths of 2^l
serial steps each, then overlap instead of adding up, and no call waits for
the host).  The concurrent pass repeats the same calls on the same paths, so
its sums are bit-identical to the sequential pass.
"""
import math
import threading
import time

import torch

import paper_2012_09715_amd as A

GBM_CALL = dict(S0=1.0, r=0.05, sigma=0.2, T=1.0, K=1.0, scheme=0, payoff=1)
CIR_PARAMS = dict(v0=0.04, kappa=0.5, theta=0.04, xi=0.3, T=1.0, functional=1)

KINDS = (A.KIND_EXACT, A.KIND_APPROX, A.KIND_CORRECTION)


def level_call(model, params, level, n, kind, approx, seed, offset=0):
    if model == "gbm":
        return A.mlmc_level_gbm(params, level, n, kind, approx, seed, offset)
    if isinstance(approx, A.Chi2Table):
        return A.mlmc_level_cir_table(params, level, n, kind, approx, seed, offset)
    if approx == "sankaran":
        return A.mlmc_level_cir_sankaran(params, level, n, kind, seed, offset)
    if approx == "em":
        return A.mlmc_level_cir_em(params, level, n, kind, seed, offset)
    return A.mlmc_level_cir(params, level, n, kind, approx, seed, offset)


def level_call_async(model, params, level, n, kind, approx, seed, offset, sums):
    """The stream-ordered form of level_call: enqueues on the current stream,
    the device writes the 8 sums into `sums`."""
    if model == "gbm":
        return A.mlmc_level_gbm_async(params, level, n, kind, approx, seed, offset, sums)
    if isinstance(approx, A.Chi2Table):
        return A.mlmc_level_cir_table_async(params, level, n, kind, approx, seed, offset, sums)
    if approx == "sankaran":
        return A.mlmc_level_cir_sankaran_async(params, level, n, kind, seed, offset, sums)
    if approx == "em":
        return A.mlmc_level_cir_em_async(params, level, n, kind, seed, offset, sums)
    return A.mlmc_level_cir_async(params, level, n, kind, approx, seed, offset, sums)


def batch_supported(model, approx):
    return True


def level_batch(model, params, jobs, approx, seed, sums):
    """All (level, kind, n_paths, path_offset) jobs of one estimator in one
    launch of the level kernel and one final pass (stream-ordered, current
    stream); row j of `sums` receives job j's 8 sums."""
    if model == "gbm":
        return A.mlmc_levels_gbm(params, jobs, approx, seed, sums)
    return A.mlmc_levels_cir(params, jobs, approx, seed, sums)


class Acc:
    """Running totals of one (level, kind) over several calls."""

    def __init__(self):
        self.n = 0.0
        self.s1 = 0.0
        self.s2 = 0.0
        self.ms = 0.0
        self.fallbacks = 0

    def add(self, s):
        self.n += s["n"]
        self.s1 += s["sum"][0]
        self.s2 += s["sum"][1]
        self.ms += s["kernel_ms"]
        self.fallbacks += s["fallbacks"]

    @property
    def mean(self):
        return self.s1 / self.n if self.n else 0.0

    @property
    def var(self):
        if self.n < 2:
            return 0.0
        m = self.mean
        return max(self.s2 / self.n - m * m, 0.0) * self.n / (self.n - 1)

    @property
    def cost(self):
        """device seconds per path"""
        return self.ms * 1e-3 / self.n if self.n else 0.0


def cost_paths(level, steps_budget=1 << 26, floor=1 << 18):
    """Paths per cost measurement: enough path-steps (2^26) to fill the GPU
    and amortise the per-call overhead."""
    return max(steps_budget >> level, floor)


LATENCY_PATHS = 256


def pilot(model, params, L, approx, seed, n_pilot, steps_budget=1 << 26):
    """Per level and kind: variance from n_pilot paths, cost per path from a
    call large enough to fill the GPU (cost_paths), and the device time of a
    call too small to fill it (LATENCY_PATHS paths: the serial time of one
    path, the floor under any call's duration)."""
    accs = [[Acc() for _ in KINDS] for _ in range(L + 1)]
    costs = [[0.0 for _ in KINDS] for _ in range(L + 1)]
    lats = [[0.0 for _ in KINDS] for _ in range(L + 1)]
    for l in range(L + 1):
        for k in KINDS:
            a = accs[l][k]
            a.add(level_call(model, params, l, n_pilot, k, approx, seed, 0))
            nc = cost_paths(l, steps_budget)
            # warm launch, then timed ones on fresh paths (not used in sums)
            level_call(model, params, l, min(nc, 4096), k, approx, seed + 7919, 0)
            s = level_call(model, params, l, nc, k, approx, seed + 7919, 1 << 36)
            costs[l][k] = s["kernel_ms"] * 1e-3 / nc
            s = level_call(model, params, l, LATENCY_PATHS, k, approx, seed + 7919, 1 << 37)
            lats[l][k] = s["kernel_ms"] * 1e-3
    return accs, costs, lats


def allocate(eps, accs, costs):
    vh = [a[A.KIND_EXACT].var for a in accs]
    v2 = [a[A.KIND_APPROX].var for a in accs]
    v4 = [max(a[A.KIND_CORRECTION].var, 1e-300) for a in accs]
    ch = [c[A.KIND_EXACT] for c in costs]
    c2 = [c[A.KIND_APPROX] for c in costs]
    c4 = [c[A.KIND_CORRECTION] for c in costs]
    vh = [max(v, 1e-300) for v in vh]
    v2 = [max(v, 1e-300) for v in v2]
    r = A.mlmc_allocate(eps, vh, ch, v2, c2, v4, c4)
    r.update(v_hat=vh, v2=v2, v4=v4, c_hat=ch, c2=c2, c4=c4)
    return r


_STREAMS = []


def _streams(k):
    """A fixed pool of k streams at the default priority (the library keeps a
    workspace per stream it has seen, so the pool is reused)."""
    while len(_STREAMS) < k:
        _STREAMS.append(torch.cuda.Stream())
    return _STREAMS[:k]


def warm_streams(job, n_streams=4):
    """Runs `job` once on each of the n_streams pool streams (each from its own
    thread): the library creates a stream's workspace on its first level call,
    which should not fall inside a timed pass."""
    def worker(st):
        with torch.cuda.stream(st):
            job()

    threads = [threading.Thread(target=worker, args=(st,)) for st in _streams(n_streams)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()


def run_concurrent(jobs, n_streams=4):
    """Runs zero-argument level calls on n_streams streams, one host thread
    per stream taking the next job in list order (put the dearest first); the
    library's calls release the GIL while they wait for the device.  Returns
    the results in job order and the wall-clock milliseconds from the first
    launch to the last result."""
    streams = _streams(n_streams)
    results = [None] * len(jobs)
    errors = []
    nxt = [0]
    lock = threading.Lock()

    def worker(st):
        with torch.cuda.stream(st):
            while True:
                with lock:
                    i = nxt[0]
                    nxt[0] += 1
                if i >= len(jobs) or errors:
                    return
                try:
                    results[i] = jobs[i]()
                except BaseException as e:  # re-raised on the calling thread
                    errors.append(e)
                    return

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    threads = [threading.Thread(target=worker, args=(st,)) for st in streams]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    wall = (time.perf_counter() - t0) * 1e3
    if errors:
        raise errors[0]
    return results, wall


def run_async(jobs, costs, n_streams=4):
    """Enqueues stream-ordered level calls from this thread on n_streams
    streams: each job(sums) writes its 8 sums into the given device row; the
    dearest job (by `costs`) goes first, each to the stream with the least
    queued cost.  One wait at the end.  Returns the result dicts in job order
    and the wall-clock milliseconds from the first launch to the last result
    on the host."""
    streams = _streams(n_streams)
    sums = torch.zeros((max(len(jobs), 1), 8), dtype=torch.float64, device="cuda")
    order = sorted(range(len(jobs)), key=lambda i: -costs[i])
    load = [0.0] * n_streams
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in order:
        j = min(range(n_streams), key=load.__getitem__)
        with torch.cuda.stream(streams[j]):
            jobs[i](sums[i])
        load[j] += costs[i]
    for st in streams:
        st.synchronize()
    host = sums.cpu()
    wall = (time.perf_counter() - t0) * 1e3
    return [A.sums_dict(host[i]) for i in range(len(jobs))], wall


def run_estimators(model, params, L, eps, approx, seed, accs, alloc, lats=None, n_streams=4, split_kinds=None):
    """Runs the allocated path counts on fresh paths of every stream (the
    pilot paths are not reused, so the estimate is independent of the
    allocation) and returns the two estimators, their standard errors and
    their measured device times.  For the concurrent pass a call of m paths
    is expected to take max(m c, latency) (lats: the pilot's latencies)."""
    out = {}
    plan = {A.KIND_EXACT: alloc["m_hat"], A.KIND_APPROX: alloc["m_tilde"], A.KIND_CORRECTION: alloc["M_tilde"]}
    cost = {A.KIND_EXACT: alloc["c_hat"], A.KIND_APPROX: alloc["c2"], A.KIND_CORRECTION: alloc["c4"]}
    runs = [[Acc() for _ in KINDS] for _ in range(L + 1)]
    time_ms = {k: 0.0 for k in KINDS}
    calls = {}
    for l in range(L + 1):
        for k in KINDS:
            want = max(int(math.ceil(plan[k][l])), 2)
            off = int(accs[l][k].n)
            calls[(l, k)] = (want, off)
            r = runs[l][k]
            s = level_call(model, params, l, want, k, approx, seed, off)
            r.add(s)
            time_ms[k] += r.ms
            calls[(l, k)] += (s,)
    # the same calls again, each estimator's levels enqueued on several
    # streams at once (stream-ordered calls, one wait per estimator)
    warm_streams(lambda: level_call(model, params, 0, 2, A.KIND_APPROX, approx, seed, 0), n_streams)
    wall = {}
    same = True
    for name, kinds in (("hat", (A.KIND_EXACT,)), ("tilde", (A.KIND_APPROX, A.KIND_CORRECTION))):
        keys = [(l, k) for l in range(L + 1) for k in kinds]
        jobs = [(lambda sums, lk=lk: level_call_async(model, params, lk[0], calls[lk][0], lk[1], approx, seed,
                                                      calls[lk][1], sums)) for lk in keys]
        est = [max(calls[lk][0] * cost[lk[1]][lk[0]], lats[lk[0]][lk[1]] if lats else 0.0) for lk in keys]
        res, wall[name] = run_async(jobs, est, n_streams)
        for lk, r in zip(keys, res):
            ref = calls[lk][2]
            same = (same and r["n"] == ref["n"] and r["sum"] == ref["sum"] and r["sum_pf"] == ref["sum_pf"]
                    and r["sum_pc"] == ref["sum_pc"] and r["fallbacks"] == ref["fallbacks"])
    # the same calls once more, each estimator as ONE batched call (one level
    # launch and one final pass), timed by events on the stream
    if batch_supported(model, approx):
        stream = torch.cuda.current_stream()
        bsums = torch.zeros((A.MAX_JOBS, 8), dtype=torch.float64, device="cuda")
        level_batch(model, params, [(0, A.KIND_EXACT, 2, 0)], approx, seed, bsums)  # warm: workspace buffers
        torch.cuda.synchronize()
        dev_ms = {}
        bsame = True
        for name, kinds in (("hat", (A.KIND_EXACT,)), ("tilde", (A.KIND_APPROX, A.KIND_CORRECTION))):
            keys = [(l, k) for l in range(L + 1) for k in kinds]
            est = {lk: max(calls[lk][0] * cost[lk[1]][lk[0]], lats[lk[0]][lk[1]] if lats else 0.0) for lk in keys}
            keys.sort(key=lambda lk: -est[lk])
            jobs = [(lk[0], lk[1], calls[lk][0], calls[lk][1]) for lk in keys]
            # the nested estimator's APPROX jobs (light kernels, high occupancy)
            # and CORRECTION jobs (exact inverses, many registers) either share
            # one launch or take one each (split_kinds)
            groups = [jobs]
            split = split_kinds
            if split is None:
                # one launch per kind once the estimator's work (at full
                # throughput) exceeds the launch floor of ~50 us; below it one
                # launch for both kinds
                split = sum(calls[lk][0] * cost[lk[1]][lk[0]] for lk in keys) > 5e-5
            if split and len(kinds) > 1:
                groups = [[j for j in jobs if j[1] == k] for k in kinds]
            times = []
            for rep in range(3):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                row = 0
                for g in groups:
                    level_batch(model, params, g, approx, seed, bsums[row:row + len(g)])
                    row += len(g)
                e1.record(stream)
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1))
            jobs = [j for g in groups for j in g]
            keys = [(j[0], j[1]) for j in jobs]
            if name == "tilde":
                n_launch_tilde = len(groups)
            dev_ms[name] = min(times)
            host = bsums.cpu()
            for j, lk in enumerate(keys):
                r, ref = A.sums_dict(host[j]), calls[lk][2]
                bsame = (bsame and r["n"] == ref["n"] and r["sum"] == ref["sum"] and r["sum_pf"] == ref["sum_pf"]
                         and r["sum_pc"] == ref["sum_pc"])
        out.update(batched_launches={"hat": 1, "tilde": n_launch_tilde},
                   device_ms_hat_batched=dev_ms["hat"], device_ms_tilde_batched=dev_ms["tilde"],
                   measured_speedup_batched=dev_ms["hat"] / dev_ms["tilde"], batched_sums_identical=bool(bsame))
    theta_hat = sum(runs[l][A.KIND_EXACT].mean for l in range(L + 1))
    var_hat = sum(runs[l][A.KIND_EXACT].var / runs[l][A.KIND_EXACT].n for l in range(L + 1))
    theta_tilde = sum(runs[l][A.KIND_APPROX].mean + runs[l][A.KIND_CORRECTION].mean for l in range(L + 1))
    var_tilde = sum(runs[l][A.KIND_APPROX].var / runs[l][A.KIND_APPROX].n
                    + runs[l][A.KIND_CORRECTION].var / runs[l][A.KIND_CORRECTION].n for l in range(L + 1))
    t_hat = time_ms[A.KIND_EXACT]
    t_tilde = time_ms[A.KIND_APPROX] + time_ms[A.KIND_CORRECTION]
    out.update(theta_hat=theta_hat, se_hat=math.sqrt(var_hat), theta_tilde=theta_tilde,
               se_tilde=math.sqrt(var_tilde), device_ms_hat=t_hat, device_ms_tilde=t_tilde,
               measured_speedup=t_hat / t_tilde if t_tilde > 0 else None,
               wall_ms_hat_concurrent=wall["hat"], wall_ms_tilde_concurrent=wall["tilde"],
               measured_speedup_concurrent=wall["hat"] / wall["tilde"], concurrent_streams=n_streams,
               concurrent_sums_identical=bool(same),
               fallbacks=sum(runs[l][k].fallbacks for l in range(L + 1) for k in KINDS),
               fallbacks_per_level=[sum(runs[l][k].fallbacks for k in KINDS) for l in range(L + 1)],
               level_ms={name: [runs[l][k].ms for l in range(L + 1)]
                         for name, k in (("exact", A.KIND_EXACT), ("approx", A.KIND_APPROX),
                                         ("correction", A.KIND_CORRECTION))})
    return out


def nested_mlmc(model, params, L, eps, approx, seed, n_pilot=1 << 16, steps_budget=1 << 26, target_paths=None,
                split_kinds=None):
    """Pilot, allocate and run both estimators.  With target_paths, eps is
    lowered so that the regular estimator allocates about that many paths in
    total (the allocation scales as eps^-2)."""
    accs, costs, lats = pilot(model, params, L, approx, seed, n_pilot, steps_budget)
    alloc = allocate(eps, accs, costs)
    if target_paths:
        eps = eps * math.sqrt(sum(alloc["m_hat"]) / target_paths)
        alloc = allocate(eps, accs, costs)
    est = run_estimators(model, params, L, eps, approx, seed, accs, alloc, lats, split_kinds=split_kinds)
    per_level = []
    for l in range(L + 1):
        per_level.append({
            "level": l,
            "v_hat": alloc["v_hat"][l], "v2": alloc["v2"][l], "v4": alloc["v4"][l],
            "c_hat_ns": alloc["c_hat"][l] * 1e9, "c2_ns": alloc["c2"][l] * 1e9, "c4_ns": alloc["c4"][l] * 1e9,
            "latency_us": [lats[l][k] * 1e6 for k in KINDS],
            "log2_v4_over_vhat": math.log2(alloc["v4"][l] / alloc["v_hat"][l]) if alloc["v_hat"][l] > 1e-299 else None,
            "m_hat": alloc["m_hat"][l], "m_tilde": alloc["m_tilde"][l], "M_tilde": alloc["M_tilde"][l],
        })
    return {"eps": eps, "levels": L, "T_hat_s": alloc["T_hat"], "T_tilde_s": alloc["T_tilde"],
            "formula_speedup": alloc["T_hat"] / alloc["T_tilde"],
            "paths_hat": sum(math.ceil(m) for m in alloc["m_hat"]),
            "paths_tilde": sum(math.ceil(m) for m in alloc["m_tilde"]) + sum(math.ceil(m) for m in alloc["M_tilde"]),
            **est, "per_level": per_level}


NU_CIR = 4 * CIR_PARAMS["kappa"] * CIR_PARAMS["theta"] / CIR_PARAMS["xi"] ** 2
SURROGATE_RANGE = (-8.0, 10.0)


def train_surrogate(n_train=10_000_000, epochs=64, batch=65536, lr=1e-2, seed=20201217, n_eval=1 << 18, log=print):
    """Builds and trains the CIR surrogate on n_train exact FP64 targets;
    returns (surrogate, report) with the held-out RMSE against exact targets."""
    s = A.Surrogate.create(NU_CIR, *SURROGATE_RANGE, seed=seed)
    t0 = time.perf_counter()
    u, ll, t = s.make_data(n_train, seed)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ue, lle, te = s.make_data(n_eval, seed + 1)
    before = float(torch.sqrt(((s.forward(ue, lle) - te) ** 2).mean()))
    loss = s.train(u, ll, t, epochs=epochs, batch=batch, lr=lr, seed=seed)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    err = (s.forward(ue, lle) - te).double()
    rep = {"n_train": n_train, "epochs": epochs, "batch": batch, "lr": lr,
           "data_seconds": t1 - t0, "train_seconds": t2 - t1, "final_train_mse": loss,
           "holdout_rmse_before": before, "holdout_rmse": float(torch.sqrt((err ** 2).mean())),
           "holdout_max_abs": float(err.abs().max()), "nu": NU_CIR, "loglam_range": SURROGATE_RANGE}
    log(f"surrogate: held-out RMSE {rep['holdout_rmse']:.3e} (untrained {before:.3e}), "
        f"data {rep['data_seconds']:.2f} s, training {rep['train_seconds']:.2f} s")
    del u, ll, t
    return s, rep


FIG4B_PARAMS = dict(v0=1.0, kappa=0.5, theta=1.0, xi=1.0, T=1.0, functional=0)


def variance_study(params=FIG4B_PARAMS, levels=range(0, 9), n=1 << 16, seed=4242):
    """Figure 4b on the device: log2 Var(P^ - P~) / Var(P^) for the fine
    functional on the same draws and time step (the TWOWAY kind: per-path
    (P^ - P~, P^, P~) in path_out) for the truncated Euler-Maruyama scheme,
    the piecewise linear and cubic chi-squared tables and the Sankaran
    approximation, per level (2^l steps).  params["functional"] 0 is X_T,
    1 the trapezoidal time average (the path-dependent, Asian, case of
    Section 5.2)."""
    nu = 4 * params["kappa"] * params["theta"] / params["xi"] ** 2
    tabs = {d: A.Chi2Table.create(nu, d) for d in (1, 3)}
    po = torch.empty(n * 3, dtype=torch.float64, device="cuda")
    calls = {"em": lambda l, sd: A.mlmc_level_cir_em(params, l, n, A.KIND_TWOWAY, sd, 0, path_out=po),
             "linear": lambda l, sd: A.mlmc_level_cir_table(params, l, n, A.KIND_TWOWAY, tabs[1], sd, 0,
                                                            path_out=po),
             "cubic": lambda l, sd: A.mlmc_level_cir_table(params, l, n, A.KIND_TWOWAY, tabs[3], sd, 0,
                                                           path_out=po),
             "sankaran": lambda l, sd: A.mlmc_level_cir_sankaran(params, l, n, A.KIND_TWOWAY, sd, 0, path_out=po)}
    out = {"params": params, "nu": nu, "paths": n, "levels": list(levels),
           "log2_ratio": {k: [] for k in calls}}
    for l in levels:
        for j, (k, fn) in enumerate(calls.items()):
            fn(l, seed + 1000 * j + l)
            v = po.view(n, 3)
            out["log2_ratio"][k].append(math.log2(max(float(v[:, 0].var()), 1e-300) / float(v[:, 1].var())))
    return out


GBM_X = dict(S0=1.0, r=0.05, sigma=0.2, T=1.0, K=1.0, scheme=0, payoff=0)


def fig3_tables():
    """The approximations of Section 4.1's variance study (Figure 3, Table 3):
    Rademacher variables, the 1024-interval constant table, and the 16-row
    linear and cubic dyadic tables (FP32 coefficients)."""
    return {"rademacher": A.Table.rademacher(), "const1024": A.Table.const(1024, 0),
            "linear16": A.Table.dyadic(16, 1), "cubic16": A.Table.dyadic(16, 3)}


def fig3_study(levels=range(0, 11), n=1 << 20, seed=3030):
    """Figure 3 on the device: GBM with P = X_T, Euler-Maruyama and Milstein;
    per level the two-way variance v^_l = Var(P^_l - P^_(l-1)) (exact
    normals) and the four-way variance V~_l = Var(D_l) of the correction
    kind for each approximation, n paths per level and kind.  Returns log2 of
    both, and the Table 3 drop log2(V~_l / v^_l) averaged over the levels
    l >= 1."""
    tabs = fig3_tables()
    out = {"paths": n, "levels": list(levels), "params": GBM_X}
    for scheme, sname in ((0, "em"), (1, "milstein")):
        p = dict(GBM_X, scheme=scheme)
        var = lambda s: max(s["sum"][1] / s["n"] - (s["sum"][0] / s["n"]) ** 2, 1e-300)
        vh = [var(A.mlmc_level_gbm(p, l, n, A.KIND_EXACT, None, seed + 17 * l)) for l in levels]
        r = {"log2_v_hat": [math.log2(v) for v in vh], "log2_V4": {}, "drop": {}}
        for j, (name, tab) in enumerate(tabs.items()):
            v4 = [var(A.mlmc_level_gbm(p, l, n, A.KIND_CORRECTION, tab, seed + 1000 * (j + 1) + 17 * l))
                  for l in levels]
            r["log2_V4"][name] = [math.log2(v) for v in v4]
            d = [math.log2(a / b) for a, b, l in zip(v4, vh, levels) if l >= 1]
            r["drop"][name] = sum(d) / len(d)
        out[sname] = r
    return out


def _sig(x, n=3):
    if isinstance(x, float) and x != 0.0 and math.isfinite(x):
        return float(f"{x:.{n}g}")
    return x


def compact(full):
    """The benchmark's MLMC results in a compact form for the one-line JSON
    record: per estimator the speed-ups, device times, estimates and, per
    level, log2 of the variances v^_l, v~_l, V~_l, the costs c^_l, c~_l,
    C~_l (ns per path), the allocated path counts m^_l, m~_l, M~_l and, for
    the surrogate, the steps counted outside its trained range."""
    out = {}
    for key, r in full.items():
        if key == "fig4b_time_average":
            continue  # in the detail file only
        if key in ("surrogate", "fig4b"):
            if key == "surrogate":
                out[key] = {k: _sig(v) for k, v in r.items()}
            else:
                out[key] = {"log2_ratio": {k: [round(x, 2) for x in v] for k, v in r["log2_ratio"].items()}}
            continue
        if key == "fig3":
            out[key] = {s: {"log2_v_hat": [round(x, 2) for x in r[s]["log2_v_hat"]],
                            "log2_V4": {t: [round(x, 2) for x in v] for t, v in r[s]["log2_V4"].items()},
                            "drop": {t: round(v, 2) for t, v in r[s]["drop"].items()}}
                        for s in ("em", "milstein")}
            out[key]["paths"] = r["paths"]
            continue
        c = {k: _sig(v, 4 if k.startswith("theta") else 3) for k, v in _short(r).items()
             if k != "levels" and not (k == "fallbacks" and not v)}
        if key not in ("gbm_em", "gbm_milstein_1e8", "cir", "cir_1e8"):
            out[key] = c  # per-level figures for the configurations' estimators only
            continue
        pl = r.get("per_level", [])
        lg = lambda v: round(math.log2(v), 2) if v and v > 1e-299 else None
        c["per_level"] = {
            "log2_v_hat": [lg(p["v_hat"]) for p in pl], "log2_v2": [lg(p["v2"]) for p in pl],
            "log2_v4": [lg(p["v4"]) for p in pl],
            "c_hat_ns": [_sig(p["c_hat_ns"]) for p in pl], "c2_ns": [_sig(p["c2_ns"]) for p in pl],
            "c4_ns": [_sig(p["c4_ns"]) for p in pl],
            "m_hat": [math.ceil(p["m_hat"]) for p in pl], "m_tilde": [math.ceil(p["m_tilde"]) for p in pl],
            "M_tilde": [math.ceil(p["M_tilde"]) for p in pl]}
        fbl = r.get("fallbacks_per_level")
        if fbl and any(fbl):  # surrogate steps outside the trained log-lambda range, per level
            c["per_level"]["fallbacks"] = fbl
        out[key] = c
    return out


def _short(r):
    keys = ("eps", "levels", "formula_speedup", "measured_speedup", "measured_speedup_concurrent",
            "measured_speedup_batched", "device_ms_hat_batched", "device_ms_tilde_batched", "batched_launches",
            "batched_sums_identical", "T_hat_s", "T_tilde_s", "paths_hat", "paths_tilde", "theta_hat", "se_hat",
            "theta_tilde", "se_tilde", "fallbacks")
    return {k: r[k] for k in keys if k in r}


def bench_summary(log=print, seed=20201217, large_paths=1e8):
    """Nested MLMC speed-ups on one GPU.

    At RMSE 1e-3 (the formula speed-up T^/T~ uses costs measured on
    GPU-filling calls; the estimators themselves are sub-millisecond):
      gbm_em         GBM, Euler-Maruyama, discounted call, levels 0..8,
                     16-row linear dyadic table (FP32)
      gbm_em_rademacher  the same with Rademacher variables (Table 3's
                     "too crude" comparator)
      gbm_em_geometric  the same with a cubic table on geometric intervals,
                     r = 0.7, 64 rows (Theorem 2.5 with r != 1/2)
      gbm_milstein   the same with the Milstein scheme, levels 0..10
      cir            CIR time average, levels 0..6, trained BF16 surrogate
      cir_poly1/3    the same with Section 5.1's piecewise linear / cubic
                     chi-squared tables (16 knots, 15 intervals per half)
      cir_sankaran   the same with the Sankaran approximation
    At the RMSE for which the regular estimator allocates ~1e8 paths (both
    estimators then fill the GPU and the device-time ratio is meaningful):
      gbm_milstein_1e8 (levels 0..10), cir_1e8 (levels 0..10, surrogate),
      cir_poly1_1e8 (levels 0..10, linear chi-squared table)."""
    res = {}
    lin16 = A.Table.dyadic(16, 1)
    log("variance study (Figure 3, Table 3): GBM, P = X_T, Euler-Maruyama and Milstein, levels 0..10")
    res["fig3"] = fig3_study()
    for sch in ("em", "milstein"):
        log(f"  {sch}: log2 v^_l " + " ".join(f"{x:6.2f}" for x in res["fig3"][sch]["log2_v_hat"]))
        for k, v in res["fig3"][sch]["log2_V4"].items():
            log(f"  {sch}: {k:10s} log2 V~_l " + " ".join(f"{x:6.2f}" for x in v)
                + f"   drop {res['fig3'][sch]['drop'][k]:.2f}")
    log("mlmc: GBM Euler-Maruyama, levels 0..8")
    res["gbm_em"] = nested_mlmc("gbm", GBM_CALL, 8, 1e-3, lin16, seed)
    log(f"  formula speedup {res['gbm_em']['formula_speedup']:.3f}")
    log("mlmc: GBM Euler-Maruyama, levels 0..8, Rademacher variables")
    res["gbm_em_rademacher"] = nested_mlmc("gbm", GBM_CALL, 8, 1e-3, A.Table.rademacher(), seed + 6)
    log(f"  formula speedup {res['gbm_em_rademacher']['formula_speedup']:.3f}")
    log("mlmc: GBM Euler-Maruyama, levels 0..8, geometric cubic table r = 0.7")
    res["gbm_em_geometric"] = nested_mlmc("gbm", GBM_CALL, 8, 1e-3, A.Table.geometric(0.7, 64, 3), seed + 7)
    log(f"  formula speedup {res['gbm_em_geometric']['formula_speedup']:.3f}")
    log("mlmc: GBM Milstein, levels 0..10")
    res["gbm_milstein"] = nested_mlmc("gbm", dict(GBM_CALL, scheme=1), 10, 1e-3, lin16, seed + 1)
    log(f"  formula speedup {res['gbm_milstein']['formula_speedup']:.3f}")
    log("mlmc: GBM Milstein, levels 0..10, ~1e8 paths")
    res["gbm_milstein_1e8"] = nested_mlmc("gbm", dict(GBM_CALL, scheme=1), 10, 1e-3, lin16, seed + 3,
                                          target_paths=large_paths)
    r = res["gbm_milstein_1e8"]
    log(f"  eps {r['eps']:.2e}: formula {r['formula_speedup']:.3f}, measured {r['measured_speedup']:.3f} "
        f"({r['device_ms_hat']:.1f} ms vs {r['device_ms_tilde']:.1f} ms), concurrent "
        f"{r['measured_speedup_concurrent']:.3f} ({r['wall_ms_hat_concurrent']:.1f} ms vs "
        f"{r['wall_ms_tilde_concurrent']:.1f} ms)")
    sur, rep = train_surrogate(seed=seed, log=log)
    res["surrogate"] = rep
    log("mlmc: CIR time average, levels 0..6, surrogate")
    res["cir"] = nested_mlmc("cir", CIR_PARAMS, 6, 1e-3, sur, seed + 2, steps_budget=1 << 24)
    log(f"  formula speedup {res['cir']['formula_speedup']:.3f}")
    for deg in (1, 3):
        tab = A.Chi2Table.create(NU_CIR, deg)
        key = f"cir_poly{deg}"
        log(f"mlmc: CIR time average, levels 0..6, chi-squared table degree {deg}")
        res[key] = nested_mlmc("cir", CIR_PARAMS, 6, 1e-3, tab, seed + 2, steps_budget=1 << 24)
        log(f"  formula speedup {res[key]['formula_speedup']:.3f}")
    log("mlmc: CIR time average, levels 0..6, Sankaran approximation")
    res["cir_sankaran"] = nested_mlmc("cir", CIR_PARAMS, 6, 1e-3, "sankaran", seed + 2, steps_budget=1 << 24)
    log(f"  formula speedup {res['cir_sankaran']['formula_speedup']:.3f}")
    log("mlmc: CIR time average, levels 0..10, surrogate, ~1e8 paths")
    res["cir_1e8"] = nested_mlmc("cir", CIR_PARAMS, 10, 1e-3, sur, seed + 4, n_pilot=1 << 14,
                                 steps_budget=1 << 24, target_paths=large_paths)
    r = res["cir_1e8"]
    log(f"  eps {r['eps']:.2e}: formula {r['formula_speedup']:.3f}, measured {r['measured_speedup']:.3f} "
        f"({r['device_ms_hat']:.1f} ms vs {r['device_ms_tilde']:.1f} ms), concurrent "
        f"{r['measured_speedup_concurrent']:.3f} ({r['wall_ms_hat_concurrent']:.1f} ms vs "
        f"{r['wall_ms_tilde_concurrent']:.1f} ms)")
    for func, key in ((0, "fig4b"), (1, "fig4b_time_average")):
        log(f"variance study (Figure 4b, functional {func}): kappa 1/2, theta = xi = T = v0 = 1, levels 0..8")
        res[key] = variance_study(dict(FIG4B_PARAMS, functional=func))
        for k, v in res[key]["log2_ratio"].items():
            log(f"  {k:8s} log2 Var(P - P~)/Var(P): " + " ".join(f"{x:6.2f}" for x in v))
    log("mlmc: CIR time average, levels 0..10, chi-squared table degree 1, ~1e8 paths")
    res["cir_poly1_1e8"] = nested_mlmc("cir", CIR_PARAMS, 10, 1e-3, A.Chi2Table.create(NU_CIR, 1), seed + 5,
                                       n_pilot=1 << 14, steps_budget=1 << 24, target_paths=large_paths)
    r = res["cir_poly1_1e8"]
    log(f"  eps {r['eps']:.2e}: formula {r['formula_speedup']:.3f}, measured {r['measured_speedup']:.3f} "
        f"({r['device_ms_hat']:.1f} ms vs {r['device_ms_tilde']:.1f} ms), concurrent "
        f"{r['measured_speedup_concurrent']:.3f} ({r['wall_ms_hat_concurrent']:.1f} ms vs "
        f"{r['wall_ms_tilde_concurrent']:.1f} ms)")
    return res
