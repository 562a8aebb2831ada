#!/usr/bin/env python3
"""Benchmark of the Schwinger-model HMC hot path on one MI355X.

A step is one HMC trajectory (refresh, adapted nested force-gradient molecular dynamics
of Eq. (11) with the fermion-force CG solves and force-gradient-shifted force, Delta H,
Metropolis) for every chain of the batched workload:
  512 independent chains, L drawn from {16, 32, 64, 128} with weights 4:3:2:1,
  beta ~ U[1, 4], m0 ~ U[0.02, 0.2] (seeded), tau = 1, n_outer = 8, n_inner = 4,
  CG in FP32 with FP64 reliable updates to a true relative residual of 1e-10,
  Delta H / Metropolis / energies in FP64.
The chains are thermalised from the hot start first (untimed), then the autotuner picks the
launch settings (workgroup size, persistent-solver limit, step-kernel variant, check interval,
reliable-update factor, chain groups) and its pick is used as is.  value = chain-trajectories per second over the
timed steps (inputs resident in HBM), one hmc_trajectory call per step.
Beside it:
  - the dominant CG kernel's roofline figure, event-timed in a pass of the same workload run
    as one chain group right after the timed steps (with several groups the kernels of
    different groups overlap in time, so a kernel's duration would not be its own);
  - the CG step kernels' algorithmic bytes per trajectory over the timed wall time per
    trajectory (the bandwidth the whole job draws, the groups overlapping);
  - the same workload with its CG iteration slots replayed as captured graph chunks;
  - the Delta H error against the FP64 oracle: sampled chains are loaded with oracle-made
    thermalised links and run one trajectory of the whole batch at the timed tolerance and at
    1e-12, against the oracle's trajectory from the same links and random numbers;
  - the same workload timed at CG tolerance 1e-12 (the setting that meets the 1e-8 target);
  - the plain FP64 single-chain 32 x 32 path, mixed against FP64 precision on 256 x 256, and
    the mixed-precision Delta H error against stored oracle trajectories at 128^2 and 256^2;
  - the CPU oracle on all available host cores (sampled workload, per-unit timings).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
METRIC = "HMC trajectories/sec at fixed acceptance; Dslash+CG achieved HBM GB/s"

# The library attributes algorithmic bytes to its sampled, event-timed CG launches (bytes
# per site: mixed FP32 slot 104 / 56 for step 1 / step 2, FP64 residual-recomputation slot
# 144 / 224, FP64 solver 224 / 128; times the sites of the chains not yet converged).
KERNELS = {0: ("k_cg_step1<true, false>", "mixed-precision CG step 1: x update, direction, t = D p"),
           1: ("k_cg_step2<true, false>", "mixed-precision CG step 2: r -= alpha D^dagger t")}


def hbm_traffic(kernel):
    """The committed rocprofv3 record of `kernel` (HBM bytes per launch from the FETCH_SIZE and
    WRITE_SIZE runs, and the kernel-trace mean duration of the same command), or None if the
    kernels have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_batched512.json")
    src = os.path.join(ROOT, "paper_1512_03812_amd", "csrc", "kernels.hip")
    try:
        rec = json.load(open(path))
        if rec["kernel_source_sha256"] != hashlib.sha256(open(src, "rb").read()).hexdigest():
            return None
        return rec["kernels"][kernel]
    except (OSError, KeyError, ValueError):
        return None


def workload(seed=1512, n_chains=512):
    import numpy as np
    g = np.random.default_rng(seed)
    L = g.choice([16, 32, 64, 128], size=n_chains, p=[0.4, 0.3, 0.2, 0.1]).tolist()
    beta = g.uniform(1.0, 4.0, size=n_chains).tolist()
    m0 = g.uniform(0.02, 0.2, size=n_chains).tolist()
    return L, beta, m0


SCHEDULE = ("adapted_nested_fg", 1.0, 8, 4)


def make_batch(args):
    import paper_1512_03812_amd as hmc
    L, beta, m0 = workload(args.seed, args.chains)
    if args.uniform_L:
        L = [args.uniform_L] * len(L)
    lat = hmc.Lattice.batch(L, L, beta, m0, seed=args.seed)
    lat.hot_start()
    lat.set_solver(tol=1e-10, max_iter=20000, reliable_delta=args.reliable_delta)
    lat.set_check_interval(args.check_interval)
    lat.set_fused_cg(args.cg_kernels == "fused")
    if args.block:
        lat.set_block_size(args.block)
    return lat, L, beta, m0


def timed_steps(lat, steps, prec="mixed"):
    import torch
    acc, status, iters, force_evals, solves = [], [], 0, 0, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = lat.trajectory(*SCHEDULE, prec=prec)
        acc += r.accepted
        status += r.status
        iters += sum(r.n_cg_iters)
        force_evals, solves = r.n_force_evals, r.n_solves
    torch.cuda.synchronize()
    return dict(dt=time.perf_counter() - t0, acc=acc, status=status, force_evals=force_evals,
                solves=solves, cg_iters_per_traj=iters / max(1, steps))


def run_batched(args):
    """Thermalisation, autotuning, warm-up, the timed steps, then the single-group roofline
    pass (every 32nd CG slot event-timed)."""
    lat, L, beta, m0 = make_batch(args)
    for _ in range(args.therm):
        lat.trajectory(*SCHEDULE, prec="mixed")
    tune = None
    if not args.no_tune:
        # with a fixed group count (--groups) the tuner leaves the groups alone
        tune = lat.autotune("mixed", 1e-10, schedule=None if args.groups else SCHEDULE)
    used = {"groups": args.groups or (tune["groups"] if tune else 1),
            "persistent_limit": (args.persistent_limit if args.persistent_limit >= 0 else
                                 (tune["persistent_limit"] if tune else 2048))}
    lat.set_cg_groups(used["groups"])
    lat.set_persistent_limit(used["persistent_limit"])
    for _ in range(args.warmup):
        lat.trajectory(*SCHEDULE, prec="mixed")
    first_timed = lat.trajectory_counter
    res = timed_steps(lat, args.steps)
    res.update(L=L, sites=lat.V_total, n_chains=lat.n_chains, tune=tune, used=used,
               timed_trajectories=[first_timed, lat.trajectory_counter])
    # roofline pass: one group, the persistent solver off (every CG kernel runs alone)
    lat.set_cg_groups(1)
    lat.set_persistent_limit(0)
    lat.set_timing(not args.no_timing)
    rp = timed_steps(lat, args.roofline_steps)
    res["s1"], res["s2"] = lat.kernel_stats(0), lat.kernel_stats(1)
    lat.set_timing(False)
    res["roofline_pass"] = {"trajectories": args.roofline_steps, "groups": 1, "persistent_limit": 0,
                            "ms_per_step": round(1e3 * rp["dt"] / max(1, args.roofline_steps), 3),
                            "cg_iters_per_traj": rp["cg_iters_per_traj"]}
    lat.set_cg_groups(used["groups"])
    lat.set_persistent_limit(used["persistent_limit"])
    res["lat"] = lat
    return res


def dH_error_vs_oracle(lat, tols):
    """Sampled chains get the oracle's thermalised links (tests/golden, written by the oracle
    alone); one trajectory of the whole batch per tolerance, with the trajectory counter of the
    oracle's record, is compared chain by chain with the oracle's FP64 trajectory (CG 1e-14)."""
    import numpy as np
    import torch
    path = os.path.join(ROOT, "tests", "golden", "batched_workload_thermalised.json")
    with open(path) as fh:
        gold = json.load(fh)
    q_saved = lat.q.clone()
    ctr_saved = lat.trajectory_counter
    lex = lat.unpack_links(lat.q)
    for ref in gold["chains"]:
        c = ref["chain"]
        o = 2 * lat.offsets[c]
        lex[o:o + 2 * ref["L"] ** 2] = torch.tensor(ref["links"], dtype=torch.float64,
                                                     device=lex.device)
    q_check = lat.pack_links(lex)
    out = {}
    for tol in tols:
        lat.q.copy_(q_check)
        lat.mark_links_changed()
        lat.trajectory_counter = gold["n_therm"]
        lat.set_solver(tol=tol, max_iter=20000)
        r = lat.trajectory(gold["scheme"], gold["tau"], gold["n_outer"], gold["n_inner"], prec="mixed")
        errs = [abs(r.dH[ref["chain"]] - ref["dH"]) for ref in gold["chains"]]
        same = all(bool(r.accepted[ref["chain"]]) == ref["accepted"] for ref in gold["chains"])
        out[f"{tol:g}"] = {"max_abs_dH_error": float(np.max(errs)), "dH_errors": [float(e) for e in errs],
                           "same_decisions": same}
    lat.set_solver(tol=1e-10, max_iter=20000)
    lat.q.copy_(q_saved)
    lat.mark_links_changed()
    lat.trajectory_counter = ctr_saved
    return {"chains": [ref["chain"] for ref in gold["chains"]],
            "L": [ref["L"] for ref in gold["chains"]],
            "reference": (f"FP64 oracle trajectory (CG 1e-14) from links after {gold['n_therm']} oracle "
                          "trajectories (tests/golden/batched_workload_thermalised.json)"),
            "by_cg_tolerance": out}


def run_graph(lat, steps):
    """The timed steps again with captured CG iteration chunks (hmc_set_graph): each solve's
    slots replay a recorded chunk of check-interval slots; the host reads the active count
    once per chunk.  Same chains, settings and results as the eager steps."""
    lat.set_graph(True)
    lat.trajectory(*SCHEDULE, prec="mixed")  # records the chunks
    r = timed_steps(lat, steps)
    lat.set_graph(False)
    n = lat.n_chains * steps
    return {"value": round(n / r["dt"], 3), "unit": "chain-trajectories/s", "steps": steps,
            "ms_per_step": round(1e3 * r["dt"] / steps, 3),
            "how": "captured chunks of CG iteration slots, the rest of each trajectory eager"}


def run_tight(lat, steps):
    """The workload at CG tolerance 1e-12, the setting whose Delta H meets the 1e-8 target."""
    lat.set_solver(tol=1e-12, max_iter=20000)
    lat.trajectory(*SCHEDULE, prec="mixed")
    r = timed_steps(lat, steps)
    lat.set_solver(tol=1e-10, max_iter=20000)
    n = lat.n_chains * steps
    return {"value": round(n / r["dt"], 3), "unit": "chain-trajectories/s", "steps": steps,
            "ms_per_step": round(1e3 * r["dt"] / steps, 3), "cg_tolerance": 1e-12,
            "acceptance": round(sum(r["acc"]) / len(r["acc"]), 4),
            "cg_iters_per_step": r["cg_iters_per_traj"]}


def run_concurrent(args, n_ctx=2):
    """The same workload as n_ctx contexts (chains k, k + n_ctx, ... in context k), each on a
    stream of its own, advanced together by hmc_trajectories_concurrent (one host thread per
    context): chain-trajectories/s over the same number of timed steps."""
    import torch
    import paper_1512_03812_amd as hmc
    L, beta, m0 = workload(args.seed, args.chains)
    lats = []
    for k in range(n_ctx):
        idx = list(range(k, len(L), n_ctx))
        with torch.cuda.stream(torch.cuda.Stream()):
            lat = hmc.Lattice.batch([L[i] for i in idx], [L[i] for i in idx], [beta[i] for i in idx],
                                    [m0[i] for i in idx], seed=args.seed + 7919 * k)
            lat.hot_start()
            lat.set_solver(tol=1e-10, max_iter=20000, reliable_delta=args.reliable_delta)
            lat.set_check_interval(args.check_interval)
            lat.trajectory("adapted_nested_fg", 1.0, 8, 4, prec="mixed")
            if not args.no_tune:
                lat.autotune("mixed", 1e-10)
            lat.set_persistent_limit(args.persistent_limit if args.persistent_limit >= 0 else 0)
        lats.append(lat)
    for _ in range(max(0, args.warmup - 1)):
        hmc.trajectories_concurrent(lats, "adapted_nested_fg", 1.0, 8, 4, "mixed")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    acc = []
    for _ in range(args.steps):
        for r in hmc.trajectories_concurrent(lats, "adapted_nested_fg", 1.0, 8, 4, "mixed"):
            acc += r.accepted
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"value": round(len(L) * args.steps / dt, 3), "unit": "chain-trajectories/s",
            "contexts": n_ctx, "ms_per_step": round(1e3 * dt / args.steps, 3),
            "acceptance": round(sum(acc) / len(acc), 4),
            "how": ("the workload's chains split over two contexts (even and odd chain indices), "
                    "each on its own stream, advanced by hmc_trajectories_concurrent")}


def run_single_fp64(args):
    """The plain FP64 single-chain path: 32 x 32, beta 2, m0 0.1, same scheme."""
    import torch
    import paper_1512_03812_amd as hmc
    lat = hmc.Lattice(32, 2.0, 0.1, seed=args.seed)
    lat.hot_start()
    lat.set_solver(tol=1e-12)
    for w in range(2):
        lat.trajectory("adapted_nested_fg", 1.0, 8, 4)
        if w == 0 and not args.no_tune:
            lat.autotune("fp64", 1e-12)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    acc = []
    n = args.single_steps
    for _ in range(n):
        acc += lat.trajectory("adapted_nested_fg", 1.0, 8, 4).accepted
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the same trajectories replayed from a captured HIP graph
    lat.set_graph(True)
    lat.trajectory("adapted_nested_fg", 1.0, 8, 4)  # capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n):
        lat.trajectory("adapted_nested_fg", 1.0, 8, 4)
    torch.cuda.synchronize()
    dtg = time.perf_counter() - t0
    return {"value": n / dt, "unit": "trajectories/s", "ms_per_traj": 1e3 * dt / n,
            "graph_value": n / dtg, "graph_ms_per_traj": 1e3 * dtg / n,
            "acceptance": sum(acc) / len(acc), "dtype": "f64",
            "config": "32x32, beta 2.0, m0 0.1, adapted nested FG tau 1 n_outer 8 n_inner 4, CG tol 1e-12"}


def run_precision(args, sizes, n_traj, n_therm):
    """Mixed precision against FP64 on single lattices: beta 4, m0 0.05, adapted nested FG
    tau 1, 8 x 4.  After n_therm untimed mixed trajectories from the hot start, each
    trajectory is run three times from the same links and trajectory counter (so with the
    same momenta and pseudofermion): FP64 CG to 1e-12 (the Delta H reference), FP64 to
    1e-10 and mixed CG to a true residual of 1e-10.  The chain continues from the mixed
    run.  Throughputs are timed per precision over the n_traj trajectories."""
    import numpy as np
    import torch
    import paper_1512_03812_amd as hmc
    out = []
    for L in sizes:
        lat = hmc.Lattice(L, 4.0, 0.05, seed=args.seed)
        lat.hot_start()
        lat.set_solver(tol=1e-10)
        if not args.no_tune:
            lat.trajectory("adapted_nested_fg", 1.0, 8, 4, prec="mixed")
            lat.autotune("mixed", 1e-10)
        for _ in range(n_therm):
            lat.trajectory("adapted_nested_fg", 1.0, 8, 4, prec="mixed")
        runs = (("fp64_1e-12", "fp64", 1e-12), ("fp64", "fp64", 1e-10), ("mixed", "mixed", 1e-10))
        secs = {k: 0.0 for k, _, _ in runs}
        dH = {k: [] for k, _, _ in runs}
        acc = {k: [] for k, _, _ in runs}
        for _ in range(n_traj):
            q0 = lat.q.clone()
            ctr = lat.trajectory_counter
            for i, (key, prec, tol) in enumerate(runs):
                if i:
                    lat.q.copy_(q0)
                    lat.mark_links_changed()
                    lat.trajectory_counter = ctr
                lat.set_solver(tol=tol)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = lat.trajectory("adapted_nested_fg", 1.0, 8, 4, prec=prec)
                torch.cuda.synchronize()
                secs[key] += time.perf_counter() - t0
                dH[key].append(r.dH[0])
                acc[key].append(r.accepted[0])
        ref = np.array(dH["fp64_1e-12"])
        print(f"precision L={L}: done", file=sys.stderr, flush=True)
        out.append({
            "L": L, "trajectories": n_traj, "thermalisation": n_therm,
            "traj_per_s": {k: round(n_traj / secs[k], 3) for k in secs},
            "mixed_over_fp64": round(secs["fp64"] / secs["mixed"], 3),
            "max_abs_dH_error": {k: float(np.max(np.abs(np.array(dH[k]) - ref)))
                                 for k in ("fp64", "mixed")},
            "accept_decisions_agree": {k: acc[k] == acc["fp64_1e-12"] for k in ("fp64", "mixed")},
            "acceptance": round(sum(acc["mixed"]) / n_traj, 3),
            "mean_abs_dH": round(float(np.mean(np.abs(ref))), 5),
        })
    return out


def precision_dH_error_vs_oracle(tols):
    """The Delta H error against the FP64 oracle on the precision lattices (128 x 128 and
    256 x 256, beta 4, m0 0.05, adapted nested FG 8 x 4): the oracle's trajectories from the
    seeded hot start stored in tests/golden/precision_trajectories.json (written by the oracle
    alone, CG 1e-12) are replayed in mixed precision at each tolerance."""
    import paper_1512_03812_amd as hmc
    with open(os.path.join(ROOT, "tests", "golden", "precision_trajectories.json")) as fh:
        gold = json.load(fh)
    out = {}
    for key in sorted(gold, key=int):
        rec = gold[key]
        L = int(key)
        out[key] = {"trajectories": len(rec["trajectories"]), "reference": f"FP64 oracle, CG {rec['tol']:g}",
                    "by_cg_tolerance": {}}
        for tol in tols:
            lat = hmc.Lattice(L, rec["beta"], rec["m0"], seed=rec["seed"])
            lat.hot_start()
            lat.set_solver(tol=tol)
            errs, same = [], True
            for ref in rec["trajectories"]:
                r = lat.trajectory(rec["scheme"], rec["tau"], rec["n_outer"], rec["n_inner"], prec="mixed")
                errs.append(abs(r.dH[0] - ref["dH"]))
                same = same and r.accepted[0] == ref["accepted"]
            out[key]["by_cg_tolerance"][f"{tol:g}"] = {"max_abs_dH_error": max(errs),
                                                       "dH_errors": errs, "same_decisions": same}
            del lat
    return out


def cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0)), "model": model}


def cpu_baseline(args):
    """The oracle (plain FP64 C, -O2, no fast-math) on a bounded, stratified sample of the
    workload, plus its per-unit costs on the small configurations.

    Workload rate: full oracle trajectories (adapted nested FG, tau 1, 8 x 4, CG to 1e-10)
    from the hot start of the first `cores` chains with L = 16, 32 and 64, and one
    fermion-force solve of the first `cores` chains with L = 64 and 128 (an L = 128
    trajectory is taken as its solve time times the trajectory/solve ratio of the L = 64
    chains); per-size mean times, weighted by the workload's count of chains of each size,
    give the time of one trajectory of all 512 chains on one core; the tasks run as `cores`
    concurrent threads (the oracle keeps no global state and its calls release the
    interpreter lock), so value = cores x 512 / that time, with each task timed under the
    full load.  `cores` is the number of CPUs this process may use, at most 16.  The same
    sample with one task per size, run alone on one core, gives single_core_value."""
    from concurrent.futures import ThreadPoolExecutor
    import numpy as np
    import oracle
    from tests import inputs
    L, beta, m0 = workload(args.seed, args.chains)
    info = cpu_info()
    cores = max(1, min(16, info["usable_cpus"]))

    def first(Ls, k):
        return [i for i, l in enumerate(L) if l == Ls][:k]

    def traj_task(c):
        q = oracle.random_links(L[c], L[c], args.seed, c)
        t0 = time.perf_counter()
        oracle.hmc_trajectory(q, beta[c], m0[c], args.seed, c, 0, *SCHEDULE, tol=1e-10)
        return ("traj", L[c], time.perf_counter() - t0)

    def solve_task(c):
        q = oracle.random_links(L[c], L[c], args.seed, c)
        phi = oracle.dirac_dagger(q, oracle.random_zeta(L[c], L[c], args.seed, c, 0), m0[c])
        t0 = time.perf_counter()
        oracle.fermion_force(q, phi, m0[c], tol=1e-10)
        return ("solve", L[c], time.perf_counter() - t0)

    def estimate(results):
        per_L = {}
        for Ls in (16, 32, 64):
            ts = [t for kind, l, t in results if kind == "traj" and l == Ls]
            if ts:
                per_L[Ls] = sum(ts) / len(ts)
        s64 = [t for kind, l, t in results if kind == "solve" and l == 64]
        s128 = [t for kind, l, t in results if kind == "solve" and l == 128]
        ratio = per_L[64] / (sum(s64) / len(s64))
        per_L[128] = ratio * sum(s128) / len(s128)
        return per_L, ratio, sum(per_L[Ls] * L.count(Ls) for Ls in per_L)

    def sample(k):
        tasks = [(traj_task, c) for Ls in (16, 32, 64) for c in first(Ls, k)]
        return tasks + [(solve_task, c) for Ls in (64, 128) for c in first(Ls, k)]

    t_begin = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        many = list(ex.map(lambda fc: fc[0](fc[1]), sample(cores)))
    per_L, ratio, total = estimate(many)
    t_many = time.perf_counter() - t_begin
    t_begin = time.perf_counter()
    one = [fn(c) for fn, c in sample(1)]
    per_L1, ratio1, total1 = estimate(one)
    t_one = time.perf_counter() - t_begin

    # per-unit costs on one core: C1 (8 x 8), C2 (32 x 32, five schemes), C4 (256 x 256)
    units = {}
    q8 = oracle.random_links(8, 8, args.seed, 0)
    t0 = time.perf_counter()
    for t in range(10):
        oracle.hmc_trajectory(q8, 2.0, 0.1, args.seed, 0, t, "omelyan", 1.0, 10, 1, tol=1e-12)
    units["c1_trajectory_s"] = (time.perf_counter() - t0) / 10
    q32 = oracle.random_links(32, 32, args.seed, 0)
    units["c2_trajectory_s"] = {}
    for scheme, n_outer, n_inner in (("leapfrog", 16, 1), ("omelyan", 8, 1), ("force_gradient", 4, 1),
                                     ("nested_fg", 4, 2), ("adapted_nested_fg", 4, 4)):
        t0 = time.perf_counter()
        oracle.hmc_trajectory(q32, 2.0, 0.1, args.seed, 0, 0, scheme, 1.0, n_outer, n_inner, tol=1e-12)
        units["c2_trajectory_s"][f"{scheme} {n_outer}x{n_inner}"] = round(time.perf_counter() - t0, 4)
    phi32 = oracle.dirac_dagger(q32, oracle.random_zeta(32, 32, args.seed, 0, 0), 0.1)
    t0 = time.perf_counter()
    _, it32, _ = oracle.cg(q32, phi32, 0.1, tol=1e-12)
    t32 = time.perf_counter() - t0
    units["c2_solve_ms"] = round(1e3 * t32, 3)
    units["c2_cg_iteration_ns_per_site"] = round(1e9 * t32 / max(1, it32) / 1024, 2)
    q256 = inputs.smooth_angles(256, 256, args.seed, 0.5)
    psi = inputs.random_spinor(256, 256, args.seed)
    t0 = time.perf_counter()
    for _ in range(5):
        oracle.dirac(q256, psi, 0.05)
    units["dslash_ns_per_site"] = round(1e9 * (time.perf_counter() - t0) / 5 / 65536, 2)
    phi256 = oracle.dirac_dagger(q256, psi, 0.05)
    t0 = time.perf_counter()
    _, it256, _ = oracle.cg(q256, phi256, 0.05, tol=1e-10)
    t256 = time.perf_counter() - t0
    units["c4_solve_ms"] = round(1e3 * t256, 1)
    units["c4_cg_iteration_ns_per_site"] = round(1e9 * t256 / max(1, it256) / 65536, 2)
    units["c4_trajectory_s_extrapolated"] = round(33 * t256, 1)
    units["how"] = ("one core; C1: 8x8 beta 2 m0 0.1, 5-stage 10 steps, tol 1e-12, mean of 10 trajectories; "
                    "C2: 32x32 beta 2 m0 0.1 hot start, one trajectory per scheme at its "
                    ">=90%-acceptance step setting, tol 1e-12, and one CG solve of phi = D^dagger zeta; "
                    "Dslash: 256x256; C4: 256x256 m0 0.05, smooth links, CG to 1e-10, trajectory = 33 "
                    "solves (4 n_outer + 1 of the adapted scheme at 8 x 4) x the solve time")
    return {"value": round(cores * len(L) / total, 4), "unit": "chain-trajectories/s",
            "cores": cores, "kind": "oracle", "cpu": info,
            "sample": (f"{len(many)} oracle tasks on {cores} concurrent threads ({t_many:.1f} s wall): full "
                       f"trajectories from the hot start of the first {cores} chains with L=16, 32, 64 and "
                       f"one solve each of the first {cores} chains with L=64 and 128 (L=128 trajectory = "
                       f"solve x the L=64 trajectory/solve ratio, {ratio:.1f}); weighted by the workload's "
                       f"L counts; value = cores x chains / weighted time per chain-trajectory set"),
            "single_core_value": round(len(L) / total1, 4),
            "single_core_sample": f"one task per size, alone on one core ({t_one:.1f} s)",
            "seconds_per_chain_traj_by_L": {str(k): round(v, 3) for k, v in per_L.items()},
            "seconds_per_chain_traj_by_L_single_core": {str(k): round(v, 3) for k, v in per_L1.items()},
            "per_unit": units}


def copy_ceilings(seed, mib=1024, reps=10):
    """Measured bandwidth ceilings of this GPU: torch's copy and the library's streaming copy
    (16-byte nontemporal accesses, on its own stream) of `mib` MiB, in GB/s of bytes read plus
    written."""
    import torch
    import paper_1512_03812_amd as hmc
    n = mib << 20
    a = torch.ones(n // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    torch_gbs = round(2 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    small = hmc.Lattice(8, 2.0, 0.1, seed=seed)
    small.stream_copy(a, b)
    torch.cuda.synchronize()
    e0.record(small.stream)
    for _ in range(reps):
        small.stream_copy(a, b)
    e1.record(small.stream)
    torch.cuda.synchronize()
    lib_gbs = round(2 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    del a, b, small
    torch.cuda.empty_cache()
    return torch_gbs, lib_gbs


def run_sweep(args):
    """Roofline sweep on single large lattices, and on one batch of equal chains (beta 2,
    m0 0.1, hot start), at each workgroup size of --sweep-blocks: FP64 dslash (the median of
    three runs of 20 launches), and CG iterations in FP64 and in mixed precision (512 iteration
    slots, every 32nd event-timed), beside the library's streaming copy of 1 GiB (and torch's
    copy) as the measured bandwidth ceiling."""
    import torch
    import paper_1512_03812_amd as hmc
    out = {"metric": "Dslash and CG iteration achieved HBM GB/s (single large lattices)",
           "unit": "GB/s", "peak": HBM_PEAK_GBS, "sizes": []}
    out["torch_copy_gbs"], out["copy_ceiling_gbs"] = copy_ceilings(args.seed)
    cases = [(L, 1) for L in args.sweep_sizes]
    if args.sweep_batch and args.sweep_batch[0] > 0:
        cases.append((args.sweep_batch[1], args.sweep_batch[0]))
    for L, nb in cases:
        lat = (hmc.Lattice(L, 2.0, 0.1, seed=args.seed) if nb == 1 else
               hmc.Lattice.batch([L] * nb, [L] * nb, 2.0, 0.1, seed=args.seed))
        lat.hot_start()
        lat.set_fused_cg(args.cg_kernels == "fused")
        V = lat.V_total
        psi = torch.randn(2, V, dtype=torch.complex128, device="cuda")
        dst = lat.new_spinor()
        for block in ([args.block] if args.block else args.sweep_blocks):
            lat.set_block_size(block)
            for _ in range(3):
                lat.dslash(psi, out=dst)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            reps, runs = 20, []
            for _ in range(3):
                torch.cuda.synchronize()
                ev[0].record(lat.stream)
                for _ in range(reps):
                    lat.dslash(psi, out=dst)
                ev[1].record(lat.stream)
                torch.cuda.synchronize()
                runs.append(1e3 * ev[0].elapsed_time(ev[1]) / reps)
            us = sorted(runs)[1]  # the median of three runs of 20 launches
            row = {"L": L, "chains": nb, "sites": V, "block": block, "dslash64_us": round(us, 2),
                   "dslash64_gbs": round(96 * V / (us * 1e-6) / 1e9, 1)}
            for prec in ("fp64", "mixed"):
                lat.set_persistent_limit(0)
                lat.set_timing(True)
                lat.cg_solve(psi, tol=1e-30, max_iter=512, prec=prec)
                s1, s2 = lat.kernel_stats(0), lat.kernel_stats(1)
                lat.set_timing(False)
                t1, t2 = s1["timed_ms"] * 1e-3, s2["timed_ms"] * 1e-3
                row[f"cg_{prec}_step1_gbs"] = round(s1["timed_bytes"] / t1 / 1e9, 1)
                row[f"cg_{prec}_step1_us"] = round(1e6 * t1 / max(1, s1["timed_launches"]), 2)
                row[f"cg_{prec}_step2_us"] = round(1e6 * t2 / max(1, s2["timed_launches"]), 2)
                row[f"cg_{prec}_step2_gbs"] = round(s2["timed_bytes"] / t2 / 1e9, 1)
                row[f"cg_{prec}_iter_us"] = round(1e6 * (t1 + t2) / max(1, s2["timed_launches"]), 2)
                row[f"cg_{prec}_iter_gbs"] = round((s1["timed_bytes"] + s2["timed_bytes"]) / (t1 + t2) / 1e9, 1)
            out["sizes"].append(row)
            print(json.dumps(row), file=sys.stderr, flush=True)
        del lat, psi, dst
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


# The paper's numerical study (Sec. 4): 32 x 32, beta 1, m0 = -0.231367, tau 2, micro step
# h/10 in the nested schemes; |Delta H| over independent momentum (and pseudofermion) sets on
# one thermalised configuration.  Schemes: (label, scheme, exact force-gradient term, inner
# steps M).  Eqs. (5), (10), (11) carry the exact term C; the Taylor-shifted variant of Eq. (5)
# is the "approx. force-gradient" row of Table 1.
PAPER_SCHEMES = [("leapfrog", "leapfrog", False, 1), ("omelyan", "omelyan", False, 1),
                 ("nested_leapfrog", "nested_leapfrog", False, 10),
                 ("nested_omelyan", "nested_omelyan", False, 5),
                 ("force_gradient", "force_gradient", True, 1),
                 ("force_gradient_approx", "force_gradient", False, 1),
                 ("nested_fg", "nested_fg", True, 5),
                 ("adapted_nested_fg", "adapted_nested_fg", True, 5),
                 ("omelyan_11stage", "omelyan_11stage", False, 1)]
DINV_PER_STEP = {"leapfrog": 4, "omelyan": 6, "nested_leapfrog": 4, "nested_omelyan": 6,
                 "force_gradient": 8, "nested_fg": 8, "adapted_nested_fg": 8, "omelyan_11stage": 12}


# Step-count grids (n_outer, n_inner) per scheme for the acceptance table of the plain FP64
# 32 x 32 configuration (beta 2, m0 0.1, tau 1).
C2_GRID = {"leapfrog": [(8, 1), (16, 1), (32, 1), (64, 1)],
           "omelyan": [(8, 1), (16, 1), (32, 1), (64, 1)],
           "force_gradient": [(4, 1), (8, 1), (16, 1), (32, 1)],
           "nested_fg": [(n, m) for n in (4, 8, 16) for m in (2, 4)],
           "adapted_nested_fg": [(n, m) for n in (4, 8, 16) for m in (2, 4)]}
C5_GRID = [(n, m) for n in (2, 3, 4, 6, 8) for m in (2, 4)]


def run_acceptance_table(args):
    """Trajectories/s at fixed (>= 90 %) acceptance.  Plain FP64 32 x 32: per scheme and
    step-count pair, the acceptance over 100 chains (one batched trajectory each, from
    configurations thermalised by 200 5-stage trajectories), and the single-chain FP64 rate;
    the smallest setting with acceptance >= 0.9 is the scheme's point.  Batched workload: the
    same scan of (n_outer, n_inner) for the adapted nested scheme in mixed precision, after
    the benchmark's thermalisation and autotuning, each setting from the same links over
    --table-steps trajectories; its point is the fastest setting with acceptance >= 0.9."""
    import math
    import torch
    import paper_1512_03812_amd as hmc
    out = {"metric": "trajectories/s at >= 90% acceptance", "c2": {}, "c5": None}
    n = args.table_chains
    bat = hmc.Lattice.batch([32] * n, [32] * n, 2.0, 0.1, seed=args.seed)
    bat.hot_start()
    bat.set_solver(tol=1e-12)
    for _ in range(args.table_therm):
        bat.trajectory("omelyan", 1.0, 10, 1)
    q_th = bat.q.clone()
    traj0 = bat.trajectory_counter
    one = hmc.Lattice(32, 2.0, 0.1, seed=args.seed)
    one.set_solver(tol=1e-12)
    one.pack_links(bat.unpack_links(q_th)[:2 * 1024], out=one.q)
    q1 = one.q.clone()
    for scheme, grid in C2_GRID.items():
        rows = []
        for n_outer, n_inner in grid:
            bat.q.copy_(q_th)
            bat.trajectory_counter = traj0
            r = bat.trajectory(scheme, 1.0, n_outer, n_inner)
            acc = sum(r.accepted) / n
            one.q.copy_(q1)
            one.trajectory(scheme, 1.0, n_outer, n_inner)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.table_single):
                one.trajectory(scheme, 1.0, n_outer, n_inner)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / args.table_single
            row = {"n_outer": n_outer, "n_inner": n_inner, "acceptance": acc,
                   "mean_abs_dH": sum(abs(d) for d in r.dH) / n, "dinv_per_traj": r.n_dinv,
                   "single_chain_traj_per_s": round(1.0 / dt, 2)}
            rows.append(row)
            print(json.dumps({"c2": scheme, **row}), file=sys.stderr, flush=True)
        ok = [x for x in rows if x["acceptance"] >= 0.9]
        best = min(ok, key=lambda x: (x["dinv_per_traj"], -x["single_chain_traj_per_s"])) if ok else None
        out["c2"][scheme] = {"points": rows, "at_90pct": best}
    # batched workload
    L, beta, m0 = workload(args.seed, args.chains)
    lat = hmc.Lattice.batch(L, L, beta, m0, seed=args.seed)
    lat.hot_start()
    lat.set_solver(tol=1e-10, max_iter=20000, reliable_delta=args.reliable_delta)
    # the benchmark's preparation: thermalisation, then the autotuner with the benchmark's
    # schedule (chain groups included)
    for _ in range(max(1, args.therm)):
        lat.trajectory("adapted_nested_fg", 1.0, 8, 4, prec="mixed")
    if not args.no_tune:
        lat.autotune("mixed", 1e-10, schedule=("adapted_nested_fg", 1.0, 8, 4))
    if args.persistent_limit >= 0:
        lat.set_persistent_limit(args.persistent_limit)
    for _ in range(2):
        lat.trajectory("adapted_nested_fg", 1.0, 8, 4, prec="mixed")
    q5 = lat.q.clone()
    t5 = lat.trajectory_counter
    rows = []
    for n_outer, n_inner in C5_GRID:
        lat.q.copy_(q5)
        lat.trajectory_counter = t5
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        acc = []
        for _ in range(args.table_steps):
            acc += lat.trajectory("adapted_nested_fg", 1.0, n_outer, n_inner, prec="mixed").accepted
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        row = {"n_outer": n_outer, "n_inner": n_inner, "acceptance": sum(acc) / len(acc),
               "chain_traj_per_s": round(len(acc) / dt, 1)}
        rows.append(row)
        print(json.dumps({"c5": "adapted_nested_fg", **row}), file=sys.stderr, flush=True)
    ok = [x for x in rows if x["acceptance"] >= 0.9]
    out["c5"] = {"points": rows, "at_90pct": max(ok, key=lambda x: x["chain_traj_per_s"]) if ok else None}
    print(json.dumps(out), flush=True)


def run_paper_study(args):
    """Sec. 4: |Delta H| versus the step size for every integrator, and the inversions of D per
    trajectory at 90% acceptance (Table 1), on a configuration thermalised here (the paper's
    own configuration is not available): a statistical comparison only."""
    import math
    import torch
    import paper_1512_03812_amd as hmc
    L, beta, m0, tau = 32, 1.0, -0.231367, 2.0
    th = hmc.Lattice(L, beta, m0, seed=args.seed)
    th.hot_start()
    th.set_solver(tol=1e-10, max_iter=50000)
    acc = []
    for k in range(args.study_therm):
        acc += th.trajectory("adapted_nested_fg", 1.0, 20, 5, prec="mixed").accepted
    q_lex = th.unpack_links(th.q)
    sg, plaq, _ = th.actions()
    print(json.dumps({"thermalisation": {"trajectories": args.study_therm,
                                         "acceptance": sum(acc) / max(1, len(acc)),
                                         "plaquette": plaq[0]}}), file=sys.stderr, flush=True)
    n = args.study_sets
    lat = hmc.Lattice.batch([L] * n, [L] * n, [beta] * n, [m0] * n, seed=args.seed + 1)
    lat.set_solver(tol=1e-10, max_iter=50000)
    q_all = q_lex.repeat(n)
    out = {"metric": "paper study: <|Delta H|> vs h and inversions of D per trajectory at 90% acceptance",
           "config": {"L": L, "beta": beta, "m0": m0, "tau": tau, "sets": n,
                      "thermalisation_trajectories": args.study_therm, "plaquette": plaq[0],
                      "cg": "mixed precision, true residual 1e-10"},
           "schemes": []}
    names = set(args.study_schemes) if args.study_schemes else None
    for label, name, exact, M in PAPER_SCHEMES:
        if names and label not in names:
            continue
        lat.set_fg_mode("exact" if exact else "shift")
        # the paper's count (Sec. 3): the exact C of Eq. (5) costs 10 per step
        dinv_step = 10 if (exact and name == "force_gradient") else DINV_PER_STEP[name]
        rows = []
        for n_outer in args.study_n:
            lat.pack_links(q_all, out=lat.q)
            lat.trajectory_counter = 0           # the same momentum sets for every point
            lat.refresh()
            t0 = time.perf_counter()
            r = lat.integrate(name, tau, n_outer, M, prec="mixed")
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            dH = [d for d, st in zip(r.dH, r.status) if st == 0 and math.isfinite(d)]
            a = sorted(abs(d) for d in dH)
            mean = sum(a) / len(a)
            sd = math.sqrt(sum((x - mean) ** 2 for x in a) / max(1, len(a) - 1))
            accp = sum(min(1.0, math.exp(-d)) if d > -700 else 1.0 for d in dH) / n
            row = {"h": tau / n_outer, "n_outer": n_outer, "M": M, "mean_abs_dH": mean, "std_abs_dH": sd,
                   "median_abs_dH": a[len(a) // 2], "max_abs_dH": a[-1],
                   "sets_abs_dH_above_10": sum(1 for x in a if x > 10.0),
                   "mean_dH": sum(dH) / len(dH), "acceptance": accp, "failed": n - len(dH),
                   "dinv_per_traj": dinv_step * n_outer, "dinv_per_traj_run": r.n_dinv,
                   "seconds": round(dt, 3)}
            rows.append(row)
            print(json.dumps({"scheme": label, **row}), file=sys.stderr, flush=True)
        # h at 90% acceptance: interpolate log(1 - acceptance) linearly in log h
        h90 = None
        pts = sorted((r["h"], 1.0 - r["acceptance"]) for r in rows if 0 < r["acceptance"] < 1)
        for (h1, e1), (h2, e2) in zip(pts, pts[1:]):
            if e1 <= 0.1 <= e2 and e1 > 0:
                w = (math.log(0.1) - math.log(e1)) / (math.log(e2) - math.log(e1))
                h90 = math.exp(math.log(h1) + w * (math.log(h2) - math.log(h1)))
        out["schemes"].append({"scheme": label, "M": M, "dinv_per_step": dinv_step, "points": rows,
                               "h_at_90pct": h90,
                               "dinv_per_traj_at_90pct": (dinv_step * tau / h90) if h90 else None})
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=1512)
    ap.add_argument("--chains", type=int, default=512)
    ap.add_argument("--single-steps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-single", action="store_true")
    ap.add_argument("--concurrent", action="store_true",
                    help="also time the workload as two contexts advanced by hmc_trajectories_concurrent")
    ap.add_argument("--therm", type=int, default=30,
                    help="untimed trajectories from the hot start before tuning and warm-up")
    ap.add_argument("--groups", type=int, default=0,
                    help="chain groups of the timed steps (0: the autotuner's pick; otherwise the "
                         "tuner does not search them)")
    ap.add_argument("--roofline-steps", type=int, default=3,
                    help="trajectories of the single-group, event-timed roofline pass")
    ap.add_argument("--graph-steps", type=int, default=4,
                    help="timed trajectories with captured CG iteration chunks (0: skip)")
    ap.add_argument("--tight-steps", type=int, default=4,
                    help="timed trajectories of the workload at CG tolerance 1e-12 (0: skip)")
    ap.add_argument("--no-oracle-check", action="store_true",
                    help="skip the Delta H comparison with the oracle's thermalised trajectories")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner")
    ap.add_argument("--block", type=int, default=0, help="fixed workgroup size (with --no-tune)")
    ap.add_argument("--uniform-L", type=int, default=0,
                    help="exploration: every chain of the batch L x L (not the benchmark workload)")
    ap.add_argument("--check-interval", type=int, default=32,
                    help="CG slots between convergence checks (workgroup compaction)")
    ap.add_argument("--reliable-delta", type=float, default=1e-4,
                    help="mixed CG: FP64 residual recomputation when the FP32 residual has dropped "
                         "by this factor")
    ap.add_argument("--cg-kernels", choices=["fused", "two"], default="two",
                    help="one fused kernel per CG iteration where the chains allow it, or two")
    ap.add_argument("--persistent-limit", type=int, default=-1,
                    help="persistent-solver limit in sites for the timed steps (-1: the autotuner's pick)")
    ap.add_argument("--sweep", action="store_true",
                    help="roofline sweep on single large lattices instead of the HMC benchmark")
    ap.add_argument("--sweep-sizes", type=int, nargs="+", default=[256, 512, 1024, 2048, 4096, 8192])
    ap.add_argument("--sweep-blocks", type=int, nargs="+", default=[256, 512],
                    help="workgroup sizes of the sweep (each lattice is measured at every one)")
    ap.add_argument("--sweep-batch", type=int, nargs=2, default=[1024, 128], metavar=("CHAINS", "L"),
                    help="also sweep a batch of CHAINS chains of L x L (0 0: none)")
    ap.add_argument("--acceptance-table", action="store_true",
                    help="trajectories/s at >= 90%% acceptance per scheme and step count")
    ap.add_argument("--table-chains", type=int, default=100)
    ap.add_argument("--table-therm", type=int, default=200)
    ap.add_argument("--table-single", type=int, default=3)
    ap.add_argument("--table-steps", type=int, default=5)
    ap.add_argument("--paper-study", action="store_true",
                    help="the paper's integrator study (Sec. 4) instead of the HMC benchmark")
    ap.add_argument("--study-sets", type=int, default=200)
    ap.add_argument("--study-therm", type=int, default=200)
    ap.add_argument("--study-n", type=int, nargs="+", default=[12, 16, 20, 24, 32, 48, 64, 96, 128, 192])
    ap.add_argument("--study-schemes", nargs="+", default=None)
    ap.add_argument("--precision-study", action="store_true",
                    help="mixed precision against FP64 on single lattices (beta 4, m0 0.05)")
    ap.add_argument("--precision-sizes", type=int, nargs="+", default=[128, 256])
    ap.add_argument("--precision-trajs", type=int, default=50)
    ap.add_argument("--precision-therm", type=int, default=30)
    ap.add_argument("--no-timing", action="store_true",
                    help="do not bracket the CG kernels with events (roofline figure omitted)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="run one streaming copy of MIB MiB first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the chains of this workload are independent and "
              "the library has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.sweep:
        run_sweep(args)
        return
    if args.paper_study:
        run_paper_study(args)
        return
    if args.acceptance_table:
        run_acceptance_table(args)
        return
    if args.precision_study:
        print(json.dumps({"precision": run_precision(args, args.precision_sizes,
                                                     args.precision_trajs,
                                                     args.precision_therm)}), flush=True)
        return

    if args.copy_calibration:
        # one streaming copy of known size, whose HBM counters scale the other kernels'
        import paper_1512_03812_amd as hmc
        n = args.copy_calibration * (1 << 20)
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        small = hmc.Lattice(8, 2.0, 0.1, seed=args.seed)
        small.stream_copy(src, dst)
        torch.cuda.synchronize()
        del src, dst, small

    b = run_batched(args)
    lat = b.pop("lat")
    n_traj = b["n_chains"] * args.steps
    value = n_traj / b["dt"]
    s1, s2 = b["s1"], b["s2"]
    # the dominant kernel: the CG step with the larger event-timed share
    which = 0 if s1["timed_ms"] >= s2["timed_ms"] else 1
    sd = (s1, s2)[which]
    kname, kdesc = KERNELS[which]
    ach = sd["timed_bytes"] / (sd["timed_ms"] * 1e-3) / 1e9 if sd["timed_ms"] > 0 else 0.0
    t12 = (s1["timed_ms"] + s2["timed_ms"]) * 1e-3
    rec = hbm_traffic(kname)
    traffic = None
    if rec and rec.get("kernel_trace_mean_us"):
        # counter bytes per dispatch over the kernel-trace mean duration of the same dispatches
        traffic = round(rec["hbm_bytes_per_launch"] / (rec["kernel_trace_mean_us"] * 1e-6) / 1e9, 1)
    cg_gbs = (s1["timed_bytes"] + s2["timed_bytes"]) / t12 / 1e9 if t12 > 0 else 0.0
    # CG bytes per trajectory against the wall time of the timed steps: the bandwidth the whole
    # job draws for its solves, with the tuned chain groups overlapping one another's launches
    rpass = b["roofline_pass"]
    wall = None
    if s1["launches"] and rpass["cg_iters_per_traj"]:
        per_traj = (s1["all_bytes"] + s2["all_bytes"]) / max(1, args.roofline_steps)
        per_traj *= b["cg_iters_per_traj"] / rpass["cg_iters_per_traj"]
        ms = 1e3 * b["dt"] / max(1, args.steps)
        wall = {"gbs": round(per_traj / (ms * 1e-3) / 1e9, 1),
                "frac": round(per_traj / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "bytes_per_traj": round(per_traj), "ms_per_traj": round(ms, 3),
                "how": ("algorithmic bytes of every CG step-kernel launch per trajectory (counted "
                        "in the roofline pass, scaled by the timed steps' CG iterations per "
                        "trajectory) over the timed steps' wall time per trajectory, which "
                        "includes every other kernel and every host wait")}
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "chain-trajectories/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * b["dt"] / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": ("batched: 512 chains, L in {16,32,64,128} weights 4:3:2:1, beta U[1,4], "
                         "m0 U[0.02,0.2], hot start, adapted nested FG tau=1 n_outer=8 n_inner=4, "
                         "mixed CG (FP32 + FP64 reliable updates) to true residual 1e-10"),
            "n_chains": b["n_chains"], "sites": b["sites"], "scheme": "adapted_nested_fg",
            "parallelism": "single GPU, chains batched in every launch",
            "thermalisation_trajectories": args.therm,
            "timed_trajectory_counters": b["timed_trajectories"],
        },
        "autotune": {"pick": b["tune"], "used": b["used"],
                     "searched": {"block": [128, 256, 512, 1024], "persistent_limit": [0, 1024, 2048],
                                  "step_variant": ["plain", "two_sites", "resident", "waves8"],
                                  "check_interval": [16, 32, 64], "reliable_delta": [1e-3, 1e-4, 1e-5],
                                  "groups": [1, 2, 3, 4]}},
        "acceptance": round(sum(b["acc"]) / len(b["acc"]), 4),
        "chain_failures": sum(1 for s in b["status"] if s != 0),
        "cg_iters_per_step": b["cg_iters_per_traj"],
        "force_evals_per_traj": b["force_evals"],
        "solves_per_traj": b["solves"],
        "roofline": {
            "bound": "hbm", "kernel": f"{kname} ({kdesc})",
            "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
            "traffic_record": rec,
            "avg_launch_us": round(1e3 * sd["timed_ms"] / max(1, sd["timed_launches"]), 3),
            "avg_bytes_per_launch": round(sd["timed_bytes"] / max(1, sd["timed_launches"])),
            "avg_bytes_per_launch_all_slots": round(sd["all_bytes"] / max(1, sd["launches"])),
            "timed_launches": sd["timed_launches"], "launches": sd["launches"],
            "sample_every": sd["sample_every"],
            "share_of_cg_step_time": round(sd["timed_ms"] / max(1e-30, s1["timed_ms"] + s2["timed_ms"]), 3),
            "measured_in": b["roofline_pass"],
        },
        "cg_step1_step2_gbs": round(cg_gbs, 1),
        "cg_bytes_over_wall_time": wall,
        "site_trajectories_per_s": round(value * b["sites"] / b["n_chains"], 1),
        "cg_steps": {KERNELS[k][0]: {"avg_launch_us": round(1e3 * st["timed_ms"] / max(1, st["timed_launches"]), 3),
                                     "achieved_gbs": round(st["timed_bytes"] / max(1e-30, st["timed_ms"] * 1e-3) / 1e9, 1),
                                     "timed_launches": st["timed_launches"],
                                     "avg_bytes_per_launch_all_slots": round(st["all_bytes"] / max(1, st["launches"]))}
                     for k, st in ((0, s1), (1, s2))},
    }
    # the measured copy ceiling of this GPU beside the peak (a 1 GiB copy, beyond the
    # Infinity Cache)
    # (not in the counter runs, whose only streaming copy is the calibration one)
    if not args.copy_calibration:
        torch_gbs, lib_gbs = copy_ceilings(args.seed)
        out["roofline"]["copy_ceiling_gbs"] = lib_gbs
        out["roofline"]["torch_copy_gbs"] = torch_gbs
        out["roofline"]["frac_of_copy_ceiling"] = round(ach / lib_gbs, 4)
        if traffic:
            out["roofline"]["traffic_frac_of_copy_ceiling"] = round(traffic / lib_gbs, 4)
        if wall:
            wall["frac_of_copy_ceiling"] = round(wall["gbs"] / lib_gbs, 4)
    if not args.no_oracle_check:
        out["dH_error_vs_oracle"] = dH_error_vs_oracle(lat, (1e-10, 1e-12))
    if args.graph_steps > 0:
        out["captured"] = run_graph(lat, args.graph_steps)
    if args.tight_steps > 0:
        out["cg_tol_1e-12"] = run_tight(lat, args.tight_steps)
    del lat
    if args.concurrent:
        out["concurrent_contexts"] = run_concurrent(args)
    if not args.no_single:
        out["fp64_single_chain"] = run_single_fp64(args)
        # the batch's chain-trajectories per second against the plain FP64 single chain's
        # trajectories per second on the same GPU
        out["fp64_single_chain"]["batched_over_single"] = round(value / out["fp64_single_chain"]["value"], 1)
        out["precision"] = run_precision(args, [256], 3, 2)
        if not args.no_oracle_check:
            out["precision_dH_error_vs_oracle"] = precision_dH_error_vs_oracle((1e-10, 1e-12))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
