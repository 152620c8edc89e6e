"""Benchmark of the p-dit sweep on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: the N=256 QAP (D = rounded Euclidean distances of 256 uniform
points in [0, 100]^2, F symmetric 0/1 at density 0.1, zero diagonals; 512
replicas from random permutations; 10^5 sweeps of a geometric beta schedule
from 0.5/s to 2000/s, s the instance's RMS swap change).  The schedule is cut
into slices of --slice sweeps (default 5000, 20 slices); one step is one
slice of the whole hot path on the 512 replicas: validation and width
selection, the exact H recompute (bf16 MFMA), the slice's sweeps on the
automatic kernel plan, and the read-out of energies, best states and the
per-sweep energy trace.  The steps resume each other through the sweep
offset and the carried best state, so warmup W plus K steps run the first
(W + K) slices of the one schedule; the defaults (W = 1, K = 19) run all of
it.

Printed: one JSON line with p-dit updates/s of the timed slices (the value);
the plain path (int32 H in device memory) timed on the first 100 sweeps of
every other slice, from the fast path's own state at that slice's start, and
its estimated full-schedule time; sweeps and seconds to the target energy
(the final best: the plain path follows the same trajectory); the roofline
of the sweep kernels; and the CPU oracle on a bounded sample of the same
workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "p-dit updates/s + time-to-target gap; batched+int8 MFMA vs plain, 1 GPU"
# 32-bit integer lane operations per second of one MI355X (the non-packed
# VALU rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz)
VALU_PEAK = 256 * 64 * 2.4e9


def method_ops_per_update(N: int, alpha: float) -> float:
    """Algorithmic integer work of one p-dit update of the method: the energy
    change of all N candidates (about 13 operations each: the H row, column
    and diagonal terms of Eq. 3 and the D/F correction), the row minimum and
    the CDF scan (2 log2 N), and with probability alpha the O(N^2) rank-1
    update of H after an accepted exchange."""
    import math
    return 13 * N + 2 * math.log2(N) + alpha * N * N
# int32 vector lane-ops per second of one MI355X: 256 CUs x 4 SIMD x 16 lanes
# x 2.4 GHz (non-packed 32-bit integer VALU rate)
ALU_PEAK_OPS = 256 * 64 * 2.4e9
# integer operations of the table kernel's algorithm: an update reads and
# compares its N candidates' energy changes (1 op each); an accepted move
# updates the N x N table (2 subtractions and a multiply-add per entry), forms
# the four H' vectors (4 N dot products of length N, 2 ops per term) and
# rebuilds rows r and t (2 N entries, about 10 ops each)
def ops_per_update(N: int, alpha: float) -> float:
    return N + alpha * (11 * N * N + 20 * N)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_table_n64_counters.json")
FAST_SRC = os.path.join(ROOT, "paper_2605_24408_amd", "csrc", "sweep_table.hip")
TRAFFIC_N256 = os.path.join(ROOT, "profiles", "sweep_reg_n256_counters.json")
REG_SRC = os.path.join(ROOT, "paper_2605_24408_amd", "csrc", "sweep_reg.hip")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (n256: schedule slices, default 19; n64: full runs, default 5)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps before them (default 1)")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-path comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-replicas", type=int, default=32)
    ap.add_argument("--cpu-sweeps", type=int, default=30,
                    help="n256: oracle sweeps per sampled state (CPU baseline)")
    ap.add_argument("--slice", type=int, default=0,
                    help="n256: sweeps per step (default: the schedule cut into warmup + steps "
                         "slices, so that the run covers all of it)")
    ap.add_argument("--sweep", default="auto", choices=["auto", "fast", "large"],
                    help="n256: sweep kernel of the timed path")
    ap.add_argument("--workload", default="n256",
                    choices=["n256", "n64", "n12", "uneven", "n256p", "n512", "pt", "cupim",
                             "clique", "hrec", "cupim256"],
                    help="n256 is the benchmark configuration; n64 times the N=64 workload's "
                         "full schedule; hrec times the H recompute step on its own at the "
                         "N=256 and N=512 workloads' shapes; the others report the "
                         "fast-vs-plain comparison for the other workload shapes (n256p: a "
                         "prefix of the N=256 schedule)")
    ap.add_argument("--sweeps", type=int, default=0,
                    help="run only the first SWEEPS sweeps of the schedule (0 = all)")
    ap.add_argument("--ttt-slices", type=int, default=0,
                    help="n12, n256p, n512, uneven: time to target of the automatic plan over "
                         "the whole schedule, run in this many slices")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one 256 MiB device-to-device copy (calibrates the "
                         "profiler's byte counters against a kernel of known traffic)")
    return ap.parse_args()


def src_hash(path: str) -> str:
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def other_workload(args):
    """Automatic plan ("fast"), the kernel without a stored H ("large") and
    the plain path on one of the other workload shapes; one JSON line, not
    the benchmark figure."""
    import numpy as np
    import torch

    from paper_2605_24408_amd import pdit
    from paper_2605_24408_amd import workloads as W

    dev = torch.device("cuda", 0)
    if args.workload == "uneven":
        insts = W.config_uneven()
    else:
        insts = [{"n12": W.config_n12, "n256p": W.config_n256, "n512": W.config_n512}[args.workload]()]
    if args.sweeps:
        for i in insts:
            i.beta = i.beta[: args.sweeps]
    dbatch = [(torch.from_numpy(i.D).to(dev), torch.from_numpy(i.F).to(dev),
               torch.from_numpy(i.perms).to(dev), torch.from_numpy(i.beta).to(dev)) for i in insts]
    perms0 = [p.clone() for _, _, p, _ in dbatch]
    updates = sum(i.R * i.N * i.T for i in insts)
    out = {"workload": args.workload, "instances": len(insts),
           "replicas": sum(i.R for i in insts), "sweeps": insts[0].T, "updates": updates}
    results = {}
    # the kernel without a stored H forced: single instances only (a batch of
    # small N would put every instance on it)
    for path in (("fast", "large", "plain") if len(insts) == 1 else ("fast", "plain")):
        ctx = pdit.Pdit(sweep={"fast": "auto"}.get(path, path),
                        recompute="plain" if path == "plain" else "auto")
        times = []
        for rep in range(1 if path == "plain" else 2):
            for (_, _, p, _), p0 in zip(dbatch, perms0):
                p.copy_(p0)
            ctx.set_sweep_offset(0)
            ctx.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if len(dbatch) > 1:
                ctx.run_sweeps_batch(dbatch, W.PHILOX_SEED)
            else:
                D, F, p, b = dbatch[0]
                ctx.run_sweeps(D, F, p, b, W.PHILOX_SEED)
            Eb, _ = ctx.best()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        cnt = ctx.counters()
        results[path] = (min(times), Eb.cpu().numpy(), cnt)
        out[path] = {"updates_per_s": updates / min(times), "seconds": min(times),
                     "kernel_ms": ctx.last_timing()[1],
                     "acceptance": cnt["accepted"] / max(cnt["updates"], 1), "ties": cnt["ties"]}
        ctx.close()
    out["speedup"] = results["plain"][0] / results["fast"][0]
    out["identical_best"] = bool(all(np.array_equal(results[p][1], results["plain"][1])
                                     for p in results))
    print(json.dumps(out), flush=True)


def ttt_workload(args):
    """Time to target on one of the other workloads (automatic plan only):
    the whole schedule in --ttt-slices slices resumed through the sweep
    offset, each slice recording every replica's energy after every sweep.
    An instance's target is the best energy over its replicas at the end of
    the schedule; the batch reaches a gap when every instance has.  A first
    hit is taken at the end of a sweep (a best state found inside a sweep
    and left again by its end is seen at the next sweep end below the same
    energy, or not at all).  A one-call run of the same schedule must end in
    the same best states (the slices resume exactly)."""
    import numpy as np
    import torch

    from paper_2605_24408_amd import pdit
    from paper_2605_24408_amd import workloads as W

    dev = torch.device("cuda", 0)
    insts = W.config_uneven() if args.workload == "uneven" else \
        [{"n12": W.config_n12, "n256p": W.config_n256, "n512": W.config_n512}[args.workload]()]
    T = insts[0].T
    K = args.ttt_slices
    S = -(-T // K)
    dbatch = [(torch.from_numpy(i.D).to(dev), torch.from_numpy(i.F).to(dev),
               torch.from_numpy(i.perms).to(dev), torch.from_numpy(i.beta).to(dev)) for i in insts]
    perms0 = [p.clone() for _, _, p, _ in dbatch]
    best = [np.full(T, np.iinfo(np.int64).max, dtype=np.int64) for _ in insts]
    ctx = pdit.Pdit()
    ctx.reset()
    ends = []
    torch.cuda.synchronize()
    start = time.perf_counter()
    for j in range(K):
        t0, t1 = j * S, min(T, (j + 1) * S)
        if t0 >= t1:
            break
        traces = [torch.zeros((i.R, t1 - t0), dtype=torch.int64, device=dev) for i in insts]
        ctx.set_sweep_offset(t0)
        if len(insts) > 1:
            ctx.run_sweeps_batch([(D, F, p, b[t0:t1].contiguous(), None, tr)
                                  for (D, F, p, b), tr in zip(dbatch, traces)], W.PHILOX_SEED)
        else:
            D, F, p, b = dbatch[0]
            ctx.set_recording(None, traces[0])
            ctx.run_sweeps(D, F, p, b[t0:t1].contiguous(), W.PHILOX_SEED)
        torch.cuda.synchronize()
        ends.append((t1, time.perf_counter() - start))
        for k, tr in enumerate(traces):
            best[k][t0:t1] = tr.min(dim=0).values.cpu().numpy()
        print(f"slice {j}: sweeps {t0}..{t1}, {ends[-1][1]:.2f} s", file=sys.stderr, flush=True)
    Eb_s, _ = ctx.best()
    Eb_s = Eb_s.cpu().numpy()
    ctx.close()
    # the same schedule in one call
    one = pdit.Pdit()
    for (_, _, p, _), p0 in zip(dbatch, perms0):
        p.copy_(p0)
    one.reset()
    one.set_sweep_offset(0)
    torch.cuda.synchronize()
    t_one = time.perf_counter()
    if len(insts) > 1:
        one.run_sweeps_batch(dbatch, W.PHILOX_SEED)
    else:
        D, F, p, b = dbatch[0]
        one.run_sweeps(D, F, p, b, W.PHILOX_SEED)
    Eb_1, _ = one.best()
    torch.cuda.synchronize()
    t_one = time.perf_counter() - t_one
    Eb_1 = Eb_1.cpu().numpy()
    one.close()

    def seconds_at(sweep):   # sweep index (0-based) -> seconds, within its slice
        prev_t, prev_s = 0, 0.0
        for t1, sec in ends:
            if sweep < t1:
                return prev_s + (sec - prev_s) * (sweep + 1 - prev_t) / (t1 - prev_t)
            prev_t, prev_s = t1, sec
        return None

    offs = np.cumsum([0] + [i.R for i in insts])
    targets = [int(Eb_s[offs[k]:offs[k + 1]].min()) for k in range(len(insts))]
    out = {"workload": args.workload, "instances": len(insts), "replicas": int(offs[-1]),
           "sweeps": T, "slices": len(ends), "seconds_sliced": ends[-1][1],
           "seconds_one_call": t_one, "same_best_as_one_call": bool(np.array_equal(Eb_s, Eb_1)),
           "target": "per instance, the best energy over its replicas at the end"}
    for gap in (0.01, 0.001, 0.0):
        hits = []
        for k in range(len(insts)):
            h = np.nonzero(best[k] <= targets[k] + abs(targets[k]) * gap)[0]
            hits.append(int(h[0]) if h.size else None)
        reached = [h for h in hits if h is not None]
        last = max(reached) if len(reached) == len(hits) else None
        out[f"gap_{gap:g}"] = {"instances_reached_at_a_sweep_end": len(reached),
                               "sweep_all_reached": None if last is None else last + 1,
                               "seconds": None if last is None else seconds_at(last),
                               "median_instance_sweep": float(np.median(reached)) + 1
                               if reached else None}
    print(json.dumps(out), flush=True)


def pt_workload(args):
    """Parallel tempering against annealing on the N=64 instance, with the
    ladder from the beta-range selection: 32 grid values from 0.01/s to
    100/s (s: the RMS swap change of the instance), 64 trial replicas x 400
    sweeps, 10 rungs.  Then 102 ladders (1020 replicas), 4-sweep periods, a
    100-period timeout and 10^4 sweeps, against annealing of the same
    replicas over the benchmark schedule (0.001 -> 1.0) and over the selected
    range.  One JSON line with update rates, best energies and the time each
    run needs to reach the others' final best; not the benchmark figure."""
    import numpy as np
    import torch

    from paper_2605_24408_amd import pdit
    from paper_2605_24408_amd import workloads as W

    dev = torch.device("cuda", 0)
    L, sets, period, timeout = 10, 102, 4, 100
    R = L * sets
    inst = W.config_n64(R=R)
    T = args.sweeps or inst.T
    N = inst.N
    n_periods = T // period
    chunks = 10
    D = torch.from_numpy(inst.D).to(dev)
    F = torch.from_numpy(inst.F).to(dev)
    perm0 = torch.from_numpy(inst.perms).to(dev)
    seed = W.PHILOX_SEED
    perm = perm0.clone()
    slot = torch.empty(R, dtype=torch.int32, device=dev)
    since = torch.empty(sets, dtype=torch.int32, device=dev)
    ctx = pdit.Pdit(sweep="fast", recompute="i8")

    # ---- beta-range selection ----
    s = W.energy_scale(inst.D, inst.F)
    grid = torch.from_numpy(np.geomspace(0.01 / s, 100.0 / s, 32).astype(np.float32)).to(dev)
    trial_R, trial_sweeps = 64, 400
    ctx.beta_select(D, F, perm0[:trial_R].contiguous(), grid, trial_sweeps, seed, L)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    E_sum, ladder, rng = ctx.beta_select(D, F, perm0[:trial_R].contiguous(), grid, trial_sweeps,
                                         seed, L)
    lo, hi = (int(x) for x in rng.cpu().numpy())
    t_sel = time.perf_counter() - t0
    sel = {"grid": f"geometric 0.01/s -> 100/s, 32 values, s = {s:.1f}", "trial_replicas": trial_R,
           "trial_sweeps": trial_sweeps, "seconds": t_sel, "lo": lo, "hi": hi,
           "beta_lo": float(grid[lo]), "beta_hi": float(grid[hi]),
           "mean_ending_energy": (E_sum.cpu().numpy() / trial_R).tolist(),
           "ladder": ladder.cpu().numpy().tolist()}

    def run_pt(record, schedule="fused", dynamics="sequential"):
        perm.copy_(perm0)
        slot.copy_(torch.arange(L, dtype=torch.int32, device=dev).repeat(sets))
        since.zero_()
        ctx.set_sweep_offset(0)
        ctx.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        curve = []
        per_chunk = (n_periods + chunks - 1) // chunks if record else n_periods
        done = 0
        while done < n_periods:
            k = min(per_chunk, n_periods - done)
            ctx.run_pt(D, F, perm, ladder, slot, since, k, period, timeout, seed, schedule,
                       dynamics)
            done += k
            if record:
                e, _ = ctx.best()
                v = int(e.min())  # synchronises before the clock is read
                curve.append((done * period, time.perf_counter() - t0, v))
        e, _ = ctx.best()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, e.cpu().numpy(), curve

    def run_anneal(beta, record):
        perm.copy_(perm0)
        ctx.set_sweep_offset(0)
        ctx.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        curve = []
        step = (T + chunks - 1) // chunks if record else T
        done = 0
        while done < T:
            k = min(step, T - done)
            ctx.run_sweeps(D, F, perm, beta[done:done + k].contiguous(), seed)
            done += k
            if record:
                e, _ = ctx.best()
                v = int(e.min())
                curve.append((done, time.perf_counter() - t0, v))
        e, _ = ctx.best()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, e.cpu().numpy(), curve

    run_pt(False)
    t_pt, eb_pt, _ = run_pt(False)
    _, _, c_pt = run_pt(True)
    cnt = ctx.counters()
    run_pt(False, "periodic")
    t_per, eb_per, _ = run_pt(False, "periodic")
    run_pt(False, "periodic", "cupim")
    t_cu, eb_cu, _ = run_pt(False, "periodic", "cupim")
    _, _, c_cu = run_pt(True, "periodic", "cupim")
    schedules = {"benchmark schedule 0.001 -> 1.0":
                 torch.from_numpy(inst.beta[:T].copy()).to(dev),
                 "selected range": torch.from_numpy(
                     W.beta_geometric(float(grid[lo]), float(grid[hi]), T)).to(dev)}
    anneal = {}
    for name, beta in schedules.items():
        run_anneal(beta, False)
        t_an, eb_an, _ = run_anneal(beta, False)
        _, _, c_an = run_anneal(beta, True)
        anneal[name] = (t_an, eb_an, c_an)
    ctx.close()
    upd = R * N * n_periods * period

    def reach(curve, target):
        hit = [c for c in curve if c[2] <= target]
        return None if not hit else {"sweeps": hit[0][0], "seconds": hit[0][1]}

    ladder_best = eb_pt.reshape(sets, L).min(axis=1)
    out = {"workload": "qap_n64_uniform99_parallel_tempering", "N": N, "replicas": R,
           "ladders": sets, "rungs": L, "period_sweeps": period, "timeout_periods": timeout,
           "sweeps": T, "beta_selection": sel}
    out["pt"] = {"updates_per_s": upd / t_pt, "seconds": t_pt, "best": int(eb_pt.min()),
                 "mean_ladder_best": float(ladder_best.mean()),
                 "acceptance": cnt["accepted"] / max(cnt["updates"], 1), "curve": c_pt,
                 "schedule": "fused (one cooperative launch, sets meet on the device)",
                 "periodic_schedule": {"updates_per_s": upd / t_per, "seconds": t_per,
                                       "identical_best": bool(np.array_equal(eb_per, eb_pt))}}
    out["pt_cupim"] = {"updates_per_s": upd / t_cu, "seconds": t_cu, "best": int(eb_cu.min()),
                       "mean_ladder_best": float(eb_cu.reshape(sets, L).min(axis=1).mean()),
                       "curve": c_cu, "reaches_pt_best": reach(c_cu, int(eb_pt.min())),
                       "schedule": "periodic, concurrent updates (GPU-CUPIM)"}
    out["pt"]["reaches_pt_cupim_best"] = reach(c_pt, int(eb_cu.min()))
    for name, (t_an, eb_an, c_an) in anneal.items():
        out["pt"]["reaches_best_of_anneal_" + name] = reach(c_pt, int(eb_an.min()))
        out["pt_cupim"]["reaches_best_of_anneal_" + name] = reach(c_cu, int(eb_an.min()))
        out["anneal " + name] = {"updates_per_s": R * N * T / t_an, "seconds": t_an,
                                 "best": int(eb_an.min()), "mean_best": float(eb_an.mean()),
                                 "curve": c_an, "reaches_pt_best": reach(c_an, int(eb_pt.min()))}
    print(json.dumps(out), flush=True)


def cupim_workload(args):
    """GPU-CUPIM (concurrent updates) against the sequential p-dit sweep on
    the N=64 instance, 1024 replicas, 10^4 iterations, on two schedules: the
    benchmark's geometric 0.001 -> 1.0 and a geometric anneal across the
    range the beta selection picks (hot: most draws move).  One JSON line
    with update rates (N updates per iteration on both), kernel times, best
    energies and the time each needs to reach the other's final best; not the
    benchmark figure."""
    import numpy as np
    import torch

    from paper_2605_24408_amd import pdit
    from paper_2605_24408_amd import workloads as W

    dev = torch.device("cuda", 0)
    inst = W.config_n64()
    N, R = inst.N, inst.R
    T = args.sweeps or inst.T
    D = torch.from_numpy(inst.D).to(dev)
    F = torch.from_numpy(inst.F).to(dev)
    perm0 = torch.from_numpy(inst.perms).to(dev)
    perm = perm0.clone()
    seed = W.PHILOX_SEED
    ctx = pdit.Pdit(sweep="fast", recompute="i8")
    s = W.energy_scale(inst.D, inst.F)
    grid = torch.from_numpy(np.geomspace(0.01 / s, 100.0 / s, 32).astype(np.float32)).to(dev)
    _, _, rng = ctx.beta_select(D, F, perm0[:64].contiguous(), grid, 400, seed, 10)
    lo, hi = (int(x) for x in rng.cpu().numpy())
    schedules = {"benchmark 0.001 -> 1.0": inst.beta[:T].copy(),
                 "selected range": W.beta_geometric(float(grid[lo]), float(grid[hi]), T)}
    chunks = 10

    def run(method, beta, record):
        perm.copy_(perm0)
        ctx.set_sweep_offset(0)
        ctx.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        curve, kms = [], 0.0
        step = (T + chunks - 1) // chunks if record else T
        done = 0
        while done < T:
            k = min(step, T - done)
            b = beta[done:done + k].contiguous()
            (ctx.run_cupim if method == "cupim" else ctx.run_sweeps)(D, F, perm, b, seed)
            done += k
            if record:
                e, _ = ctx.best()
                v = int(e.min())
                curve.append((done, time.perf_counter() - t0, v))
        e, _ = ctx.best()
        torch.cuda.synchronize()
        if not record:
            kms = ctx.last_timing()[1]
        cnt = ctx.counters()
        return time.perf_counter() - t0, e.cpu().numpy(), curve, kms, cnt

    def reach(curve, target):
        hit = [c for c in curve if c[2] <= target]
        return None if not hit else {"sweeps": hit[0][0], "seconds": hit[0][1]}

    out = {"workload": "qap_n64_uniform99_cupim_vs_sequential", "N": N, "replicas": R,
           "iterations": T, "beta_range": [float(grid[lo]), float(grid[hi])]}
    for name, bnp in schedules.items():
        beta = torch.from_numpy(bnp).to(dev)
        res = {}
        for method in ("cupim", "sequential"):
            run(method, beta, False)
            t, eb, _, kms, cnt = run(method, beta, False)
            _, _, curve, _, _ = run(method, beta, True)
            res[method] = (t, eb, curve, kms, cnt)
        row = {}
        for method, (t, eb, curve, kms, cnt) in res.items():
            other = res["sequential" if method == "cupim" else "cupim"]
            row[method] = {"updates_per_s": R * N * T / t, "seconds": t, "kernel_ms": kms,
                           "best": int(eb.min()), "mean_best": float(eb.mean()),
                           "accepted_per_iteration": cnt["accepted"] / (R * T),
                           "curve": curve, "reaches_other_best": reach(curve, int(other[1].min()))}
        out[name] = row
    ctx.close()
    print(json.dumps(out), flush=True)


def clique_workload(args):
    """The clique-flow sweep against the general on-chip kernel and the plain
    path on the N=256 tai256c stand-in (16 x 16 grid distances, a clique of
    92 facilities), 512 replicas, the first 2000 sweeps of its schedule (the
    plain path: the first 100).  All three give identical results on the
    common prefix.  One JSON line; not the benchmark figure."""
    import numpy as np
    import torch

    from paper_2605_24408_amd import pdit
    from paper_2605_24408_amd import workloads as W

    dev = torch.device("cuda", 0)
    inst = W.config_clique256()
    N, R = inst.N, inst.R
    T = args.sweeps or 2000
    D = torch.from_numpy(inst.D).to(dev)
    F = torch.from_numpy(inst.F).to(dev)
    perm0 = torch.from_numpy(inst.perms).to(dev)
    perm = perm0.clone()
    out = {"workload": inst.name, "N": N, "replicas": R, "clique": 92,
           "beta": "geometric 0.5/s -> 2000/s over 10^4 sweeps, prefix"}
    finals = {}
    for path, sweep, steps in (("clique", "clique", T), ("general", "fast", T),
                               ("plain", "plain", min(T, 100))):
        ctx = pdit.Pdit(sweep=sweep, recompute="auto" if sweep != "plain" else "plain")
        beta = torch.from_numpy(inst.beta[:steps].copy()).to(dev)
        best = None
        for _ in range(2 if path != "plain" else 1):
            perm.copy_(perm0)
            ctx.set_sweep_offset(0)
            ctx.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.run_sweeps(D, F, perm, beta, W.PHILOX_SEED)
            e, _ = ctx.best()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        cnt = ctx.counters()
        plan = ctx.last_plan()
        finals[path] = (steps, perm.cpu().numpy().copy(), e.cpu().numpy())
        out[path] = {"sweeps": steps, "updates_per_s": R * N * steps / best, "seconds": best,
                     "kernel_ms": ctx.last_timing()[1], "plan": plan,
                     "acceptance": cnt["accepted"] / max(cnt["updates"], 1),
                     "best": int(e.min().item())}
        ctx.close()
    out["clique_vs_general"] = out["clique"]["updates_per_s"] / out["general"]["updates_per_s"]
    out["clique_vs_plain"] = out["clique"]["updates_per_s"] / out["plain"]["updates_per_s"]
    out["identical_clique_general"] = bool(np.array_equal(finals["clique"][1], finals["general"][1]))
    print(json.dumps(out), flush=True)


def cpu_info() -> dict:
    """Host cores and CPU model (for the CPU baseline)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def n256_workload(args):
    """The benchmark: the N=256 workload's schedule in slices (see the module
    docstring)."""
    import numpy as np
    import torch

    from paper_2605_24408_amd import pdit
    from paper_2605_24408_amd import workloads as W

    dev = torch.device("cuda", 0)
    inst = W.config_n256()
    N, R, T = inst.N, inst.R, inst.T
    if args.steps is None:
        args.steps = 19
    if args.warmup is None:
        args.warmup = 1
    if args.steps < 1 or args.warmup < 0:
        print("steps must be at least 1 and warmup at least 0", file=sys.stderr)
        sys.exit(2)
    S = args.slice or -(-T // (args.warmup + args.steps))
    n_slices = (T + S - 1) // S
    if args.warmup + args.steps > n_slices:
        print(f"warmup + steps must be at most {n_slices} slices of {S} sweeps", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        # a plain device-to-device copy of 256 MiB: the profiler's byte counters
        # for it calibrate those of the sweep kernel
        src = torch.ones(64 << 20, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    D = torch.from_numpy(inst.D).to(dev)
    F = torch.from_numpy(inst.F).to(dev)
    beta = torch.from_numpy(inst.beta).to(dev)
    perm = torch.from_numpy(inst.perms).to(dev)
    seed = W.PHILOX_SEED
    trace = torch.zeros((R, S), dtype=torch.int64, device=dev)
    ctx = pdit.Pdit(sweep=args.sweep)
    ctx.set_sweep_offset(0)
    ctx.reset()

    # the plain path is sampled at the start of every other slice, from the
    # fast path's own state there (the two follow the same trajectory)
    sample_at = set(range(0, n_slices, 2))
    saved = {}
    per_slice = []
    best_trace = np.full(T, np.iinfo(np.int64).max, dtype=np.int64)
    last_trace = [trace]

    def one_slice(i, timed):
        t0, t1 = i * S, min(T, (i + 1) * S)
        if i in sample_at:
            Eb, pb = ctx.best() if i > 0 else (None, None)
            saved[i] = (perm.clone(), None if Eb is None else Eb.clone(),
                        None if pb is None else pb.clone())
        tr = trace if t1 - t0 == S else torch.zeros((R, t1 - t0), dtype=torch.int64, device=dev)
        ctx.set_recording(None, tr)
        ctx.run_sweeps(D, F, perm, beta[t0:t1], seed)
        last_trace[0] = tr
        return t0, t1

    # ---------------- warmup slices (untimed) ----------------
    for i in range(args.warmup):
        t0, t1 = one_slice(i, False)
        torch.cuda.synchronize()
        best_trace[t0:t1] = last_trace[0].min(dim=0).values.cpu().numpy()
        cnt = ctx.counters()
        per_slice.append({"slice": i, "timed": False, "kernel_ms": ctx.last_timing()[1],
                          "alpha": cnt["accepted"] / cnt["updates"], "plan": ctx.last_plan()})
        print(f"warmup slice {i}: {per_slice[-1]['kernel_ms']:.0f} ms of sweep kernel",
              file=sys.stderr, flush=True)
    # ---------------- timed slices ----------------
    torch.cuda.synchronize()
    start = time.perf_counter()
    for i in range(args.warmup, args.warmup + args.steps):
        t0, t1 = one_slice(i, True)
        cnt = ctx.counters()   # waits for the slice: per-slice acceptance and timing
        best_trace[t0:t1] = last_trace[0].min(dim=0).values.cpu().numpy()
        per_slice.append({"slice": i, "timed": True, "kernel_ms": ctx.last_timing()[1],
                          "alpha": cnt["accepted"] / cnt["updates"], "plan": ctx.last_plan(),
                          "end_s": time.perf_counter() - start, "ties": cnt["ties"]})
        print(f"slice {i}: {per_slice[-1]['kernel_ms']:.0f} ms of sweep kernel", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - start
    run_sweeps = min(T, (args.warmup + args.steps) * S)
    timed_updates = R * N * sum(min(T, (i + 1) * S) - i * S
                                for i in range(args.warmup, args.warmup + args.steps))
    value = timed_updates / elapsed
    Eb, pb = ctx.best()
    Eb_fast = Eb.cpu().numpy()
    timed = [p for p in per_slice if p["timed"]]
    kernel_s = sum(p["kernel_ms"] for p in timed) / 1e3
    alpha_timed = float(np.mean([p["alpha"] for p in timed]))

    # ---------------- roofline of the sweep kernels (timed slices) ----------------
    ops = sum(method_ops_per_update(N, p["alpha"]) * R * N * S for p in timed)
    achieved = ops / kernel_s
    plans = sorted({(p["plan"]["sweep"], p["plan"]["size_class"]) for p in timed})
    # HBM bytes per launch of the sweep kernel from the profiler's counters
    # (FETCH_SIZE + WRITE_SIZE, calibrated on a copy of known size), stored with
    # the hash of the kernel source they were taken on; null once it changed
    traffic, traffic_src = None, None
    if os.path.exists(TRAFFIC_N256):
        rec = json.load(open(TRAFFIC_N256))
        if rec.get("kernel_source_sha") == src_hash(REG_SRC) and rec.get("slice_sweeps") == S:
            traffic = rec.get("bytes_per_launch")
            traffic_src = "stored: " + os.path.relpath(TRAFFIC_N256, ROOT)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12,
                "unit": "T int32 lane-op/s", "frac": achieved / VALU_PEAK, "traffic": traffic,
                "traffic_source": traffic_src,
                "kernels": [f"{k} (class {c})" if c else k for k, c in plans],
                "kernel_s": kernel_s,
                "ops_per_update": "13 N + 2 log2 N + alpha N^2 per slice (alpha measured)",
                "mean_alpha": alpha_timed}

    # ---------------- time to target ----------------
    target = int(Eb_fast.min())
    ttt = {"target_energy": target,
           "target": "final best over all replicas of the schedule run (the plain path "
                     "follows the same trajectory and ends at the same best)"}
    ends = {p["slice"]: p.get("end_s") for p in per_slice}
    for gap in (0.01, 0.001, 0.0):
        lim = target + abs(target) * gap
        hit = np.nonzero(best_trace[:run_sweeps] <= lim)[0]
        if hit.size:
            k = int(hit[0])
            sl = k // S
            prev_end = ends.get(sl - 1) if sl > args.warmup else 0.0
            end = ends.get(sl)
            ttt[f"gap_{gap:g}"] = {"sweep": k + 1, "timed": end is not None,
                                   "seconds_at_slice_end": end,
                                   "seconds_interpolated": None if end is None else
                                   prev_end + (end - prev_end) * ((k % S) + 1) / S}

    # ---------------- plain path on the sampled slices ----------------
    plain_rec = None
    if not args.no_plain:
        plain = pdit.Pdit(sweep="plain", recompute="plain")
        fastc = pdit.Pdit(sweep=args.sweep)
        PS = min(100, S)
        samples, same = [], True
        for i in sorted(saved):
            p0, eb0, pb0 = saved[i]
            res = {}
            for name, c in (("plain", plain), ("fast", fastc)):
                p = p0.clone()
                c.set_sweep_offset(i * S)
                c.reset()
                torch.cuda.synchronize()
                t_ = time.perf_counter()
                c.run_sweeps(D, F, p, beta[i * S:i * S + PS].contiguous(), seed)
                e = c.energy()
                torch.cuda.synchronize()
                res[name] = (time.perf_counter() - t_, p.cpu().numpy(), e.cpu().numpy(),
                             c.counters(), c.last_timing()[1] / 1e3)
            same = same and np.array_equal(res["plain"][1], res["fast"][1]) and \
                np.array_equal(res["plain"][2], res["fast"][2])
            cnt, ks = res["plain"][3], res["plain"][4]
            a_ = cnt["accepted"] / cnt["updates"]
            # the plain kernel's algorithmic HBM bytes: per update the row, column
            # and diagonal of H (3N elements), and per accepted exchange the
            # read and write of the whole N x N H (4-byte elements)
            hbm = cnt["updates"] * (3 * N + a_ * 2 * N * N) * 4
            samples.append({"slice": i, "plain_s": res["plain"][0], "fast_s": res["fast"][0],
                            "alpha": a_, "plain_kernel_s": ks, "plain_hbm_GBps": hbm / ks / 1e9,
                            "plain_hbm_frac": hbm / ks / PEAK_HBM})
        plain.close()
        fastc.close()
        # each sample stands for the two slices it starts (every other slice)
        est = sum(x["plain_s"] / PS * S * 2 for x in samples)
        fast_total = sum(p["kernel_ms"] for p in per_slice) / 1e3
        hot = samples[0]
        plain_rec = {"sweeps_per_sample": PS, "samples": samples,
                     "hbm_roofline_first_sample": {
                         "bound": "hbm", "achieved": hot["plain_hbm_GBps"],
                         "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": hot["plain_hbm_frac"],
                         "bytes_per_update": "(3 N + alpha 2 N^2) x 4 B"},
                     "estimated_full_schedule_s": est,
                     "fast_full_schedule_kernel_s": fast_total,
                     "value": R * N * T / est,
                     "speedup": est / fast_total, "identical_results_on_samples": bool(same)}

    # ---------------- CPU oracle on a bounded sample ----------------
    cpu = None
    if not args.no_cpu and saved:
        import oracle
        from concurrent.futures import ThreadPoolExecutor
        info = cpu_info()
        threads = max(1, min(16, info["nproc"] or 1))
        oracle.lib()
        starts = sorted(saved)[::2]                 # every fourth slice
        tasks = [(i, k) for i in starts for k in range(threads)]
        host = {i: saved[i][0].cpu().numpy() for i in starts}
        CS = args.cpu_sweeps

        def run_task(ik):
            i, k = ik
            return oracle.run(inst.D, inst.F, host[i][k:k + 1], inst.beta[i * S:i * S + CS], seed,
                              sweep_offset=i * S, rep_ids=[k]).counters[0, 1]

        t2 = time.perf_counter()
        run_task(tasks[0])
        one_s = time.perf_counter() - t2
        t2 = time.perf_counter()
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(run_task, tasks))
        all_s = time.perf_counter() - t2
        upd = len(tasks) * N * CS
        cpu = {"value": upd / all_s, "unit": "p-dit updates/s", "cores": threads,
               "kind": "oracle", "single_core": N * CS / one_s, "nproc": info["nproc"],
               "cpu_model": info["cpu_model"],
               "sample": f"{threads} replicas x {CS} sweeps from the fast path's states at the "
                         f"starts of slices {starts} ({len(tasks)} tasks, one replica per "
                         f"thread), the schedule's beta and sweep offsets there"}
    ctx.close()

    out = {"metric": METRIC, "value": value, "unit": "p-dit updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
           "data": "synthetic",
           "config": {"workload": "qap_n256_euclid", "N": N, "replicas": R, "sweeps": T,
                      "slice_sweeps": S, "timed_sweeps": f"{args.warmup * S}..{run_sweeps}",
                      "beta": f"geometric 0.5/s -> 2000/s, s = {inst.meta['scale']:.1f}",
                      "sweep_plan": args.sweep, "parallelism": "replicas"},
           "acceptance": alpha_timed, "roofline": roofline, "plain": plain_rec,
           "time_to_target": ttt, "cpu_baseline": cpu,
           "slices": [{k: v for k, v in p.items() if k != "plan"} | {"kernel": p["plan"]["sweep"]}
                      for p in per_slice]}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the replicas of this "
              "workload are independent chains and the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "pt":
        pt_workload(args)
        return
    if args.workload == "cupim":
        cupim_workload(args)
        return
    if args.workload == "clique":
        clique_workload(args)
        return
    if args.workload == "n256":
        n256_workload(args)
        return
    if args.workload == "hrec":
        hrec_workload(args)
        return
    if args.workload == "cupim256":
        cupim256_workload(args)
        return
    if args.workload != "n64":
        if args.ttt_slices:
            ttt_workload(args)
        else:
            other_workload(args)
        return
    n64_workload(args)


def cupim256_workload(args):
    """GPU-CUPIM beyond the on-chip kernel: the N=256 workload (distances to
    141) at its 512 replicas, the first --sweeps (default 200) iterations of
    its schedule, against the sequential sweeps (the register kernel) on the
    same schedule slice from the same start.  Per method the kernel time of
    the run (HIP events), updates/s (N updates per iteration or sweep) and
    the best energy reached; not the benchmark figure."""
    import numpy as np
    import torch

    from paper_2605_24408_amd import pdit as P
    from paper_2605_24408_amd import workloads as W
    dev = torch.device("cuda", 0)
    inst = W.config_n256()
    T = args.sweeps or 200
    D = torch.from_numpy(inst.D).to(dev)
    F = torch.from_numpy(inst.F).to(dev)
    beta = torch.from_numpy(inst.beta[:T].copy()).to(dev)
    out = {"workload": "cupim256", "N": inst.N, "replicas": inst.R, "iterations": T}
    for method in ("cupim", "sweeps"):
        with P.Pdit() as ctx:
            for rep in range(2):   # the first run allocates and builds
                p = torch.from_numpy(inst.perms).to(dev)
                ctx.set_sweep_offset(0)
                ctx.reset()
                (ctx.run_cupim if method == "cupim" else ctx.run_sweeps)(D, F, p, beta,
                                                                      W.PHILOX_SEED)
                torch.cuda.synchronize()
            ms = ctx.last_timing()[1]
            e, _ = ctx.best()
            cnt = ctx.counters()
            out[method] = {"kernel_ms": ms, "updates_per_s": inst.R * inst.N * T / (ms * 1e-3),
                           "best_energy": int(e.min()), "accepted": cnt["accepted"],
                           "plan": ctx.last_plan()}
        print(f"{method}: {ms:.1f} ms, best {out[method]['best_energy']}", file=sys.stderr,
              flush=True)
    print(json.dumps(out), flush=True)


# peaks of MI355X: dense MFMA (bf16 2.5 PFLOP/s, int8 5.0 POP/s), HBM 8 TB/s
PEAK_BF16 = 2.5e15
PEAK_I8 = 5.0e15
PEAK_HBM = 8.0e12


def hrec_workload(args):
    """Step "H recompute" (pdit_h_recompute) on its own, over all replicas of
    the N=256 workload (bf16 MFMA; u8 distances above 127 rule out int8) and
    the N=512 workload (byte-plane split MFMA, int64 H), plus the N=256 shape
    with 7-bit data for the int8 mode.  Per call: the time of the recompute
    (H in the library's buffer and its trace) from HIP events, the MFMA
    operations it issues (2 R N^3 per product; four products in split mode)
    against the dense peak of their type, and the HBM bytes of the H it
    writes against 8 TB/s."""
    import numpy as np
    import torch

    from paper_2605_24408_amd import pdit as P
    from paper_2605_24408_amd import workloads as W
    dev = torch.device("cuda", 0)
    reps = args.steps or 20
    warm = args.warmup if args.warmup is not None else 2
    c4, c5 = W.config_n256(), W.config_n512()
    small = np.minimum(c4.D, 127).astype(np.int32)   # the int8 mode's data at the same shape
    cases = [("qap_n256_euclid", c4.D, c4.F, c4.perms, "bf16", 1),
             ("qap_n256_euclid (D clipped to 127)", small, c4.F, c4.perms, "i8", 1),
             ("qap_n512_uniform1e4", c5.D, c5.F, c5.perms, "split", 4)]
    results = []
    with P.Pdit() as ctx:
        for name, D, F, perms, mode, products in cases:
            Dd = torch.from_numpy(np.ascontiguousarray(D, dtype=np.int32)).to(dev)
            Fd = torch.from_numpy(np.ascontiguousarray(F, dtype=np.int32)).to(dev)
            pd = torch.from_numpy(np.ascontiguousarray(perms, dtype=np.int32)).to(dev)
            R, N = pd.shape
            times = []
            for k in range(warm + reps):
                ctx.h_recompute(Dd, Fd, pd, mode=mode, with_H=False)
                if k >= warm:
                    times.append(ctx.last_timing()[0])
            ms = float(np.median(times))
            h64 = mode == "split"            # the N=512 data need int64 H
            hbytes = R * N * N * (8 if h64 else 4)
            ops = products * 2.0 * R * N ** 3
            peak = PEAK_BF16 if mode == "bf16" else PEAK_I8
            achieved = ops / (ms * 1e-3)
            results.append({"config": name, "N": N, "R": R, "mode": mode, "ms": ms,
                            "mfma_ops": ops, "achieved_ops_per_s": achieved, "peak": peak,
                            "frac_mfma": achieved / peak, "h_bytes": hbytes,
                            "hbm_gbs": hbytes / (ms * 1e-3) / 1e9,
                            "frac_hbm": hbytes / (ms * 1e-3) / PEAK_HBM})
            print(f"{name} {mode}: {ms:.3f} ms, {achieved / 1e12:.1f} T ops/s "
                  f"({100 * achieved / peak:.1f}% of peak), H {hbytes / 1e6:.0f} MB at "
                  f"{hbytes / (ms * 1e-3) / 1e9:.0f} GB/s", file=sys.stderr, flush=True)
    print(json.dumps({"workload": "h_recompute", "steps": reps, "warmup": warm,
                      "unit": "ms per call", "results": results}), flush=True)


def n64_workload(args):
    """The N=64 workload's full schedule as the step (the previous headline
    configuration, kept for comparison); same JSON fields."""
    if args.steps is None:
        args.steps = 5
    if args.warmup is None:
        args.warmup = 1
    import numpy as np
    import torch

    from paper_2605_24408_amd import pdit
    from paper_2605_24408_amd import workloads as W

    dev = torch.device("cuda", 0)
    inst = W.config_n64()
    N, R, T = inst.N, inst.R, inst.T
    D = torch.from_numpy(inst.D).to(dev)
    F = torch.from_numpy(inst.F).to(dev)
    perm0 = torch.from_numpy(inst.perms).to(dev)
    beta = torch.from_numpy(inst.beta).to(dev)
    perm = perm0.clone()
    seed = W.PHILOX_SEED
    upd_per_step = R * N * T

    def one_step(ctx):
        perm.copy_(perm0)
        ctx.set_sweep_offset(0)
        ctx.reset()
        ctx.run_sweeps(D, F, perm, beta, seed)
        return ctx.best()

    if args.copy_probe:
        src = torch.ones(64 << 20, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---------------- fast path (timed) ----------------
    fast = pdit.Pdit(sweep="fast", recompute="i8")
    for _ in range(args.warmup):
        one_step(fast)
    torch.cuda.synchronize()
    sweep_ms, rec_ms = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        Eb, pb = one_step(fast)
        r_ms, s_ms = fast.last_timing()
        rec_ms.append(r_ms)
        sweep_ms.append(s_ms)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = upd_per_step * args.steps / elapsed
    cnt = fast.counters()
    E_fast = fast.energy().cpu().numpy()
    Eb_fast = Eb.cpu().numpy()
    alpha = cnt["accepted"] / cnt["updates"]

    # ---------------- roofline of the sweep kernel ----------------
    sweep_avg_ms = float(np.mean(sweep_ms))
    ops_per_launch = ops_per_update(N, alpha) * upd_per_step
    achieved = ops_per_launch / (sweep_avg_ms * 1e-3)
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        rec = json.load(open(TRAFFIC_FILE))
        if rec.get("kernel_source_sha") == src_hash(FAST_SRC):
            traffic = rec.get("bytes_per_launch")
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": ALU_PEAK_OPS / 1e12,
                "unit": "Tops/s", "frac": achieved / ALU_PEAK_OPS, "traffic": traffic,
                "kernel": "sweep_table_kernel<64, true, true, false>", "kernel_ms": sweep_avg_ms,
                "recompute_ms": float(np.mean(rec_ms)),
                "ops_per_update": ops_per_update(N, alpha),
                "lds_bytes_per_update": 4 * N}

    # ---------------- plain path, target energy, time to target ----------------
    plain_rec = None
    ttt = None
    if not args.no_plain:
        plain = pdit.Pdit(sweep="plain", recompute="plain")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        Ebp, _ = one_step(plain)
        torch.cuda.synchronize()
        plain_s = time.perf_counter() - t1
        _, plain_sweep_ms = plain.last_timing()
        E_plain = plain.energy().cpu().numpy()
        Eb_plain = Ebp.cpu().numpy()
        plain_rec = {"value": upd_per_step / plain_s, "ms_per_step": 1e3 * plain_s,
                     "sweep_kernel_ms": plain_sweep_ms,
                     "speedup": value * plain_s / upd_per_step,
                     "identical_results": bool(np.array_equal(E_plain, E_fast)
                                               and np.array_equal(Eb_plain, Eb_fast))}
        # target: the plain path's best energy over all replicas; sweeps to
        # target from the per-sweep energy trace (identical on both paths)
        target = int(Eb_plain.min())
        trace = torch.zeros((R, T), dtype=torch.int64, device=dev)
        perm.copy_(perm0)
        fast.set_sweep_offset(0)
        fast.reset()
        fast.set_recording(None, trace)
        fast.run_sweeps(D, F, perm, beta, seed)
        tr = trace.min(dim=0).values.cpu().numpy()
        hit = np.nonzero(tr <= target)[0]
        k = int(hit[0]) + 1 if hit.size else T
        # wall time of the first k sweeps, on each path
        bk = beta[:k].contiguous()

        def timed_prefix(ctx):
            perm.copy_(perm0)
            ctx.set_sweep_offset(0)
            ctx.reset()
            torch.cuda.synchronize()
            t = time.perf_counter()
            ctx.run_sweeps(D, F, perm, bk, seed)
            e, _ = ctx.best()
            torch.cuda.synchronize()
            return time.perf_counter() - t, int(e.min())

        tf, ef = timed_prefix(fast)
        tp, ep = timed_prefix(plain)
        ttt = {"target_energy": target, "sweeps_to_target": k,
               "fast_s": tf, "plain_s": tp, "fast_best_at_k": ef, "plain_best_at_k": ep,
               "final_gap": float((Eb_fast.min() - target) / target)}
        plain.close()

    # ---------------- CPU oracle baseline (bounded sample) ----------------
    cpu = None
    if not args.no_cpu:
        import oracle
        from concurrent.futures import ThreadPoolExecutor
        threads = max(1, min(16, os.cpu_count() or 1))
        nrep = min(args.cpu_replicas, R)
        oracle.lib()
        t2 = time.perf_counter()
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(lambda k: oracle.run(inst.D, inst.F, inst.perms[k:k + 1], inst.beta,
                                             seed, rep_ids=[k]), range(nrep)))
        cpu_s = time.perf_counter() - t2
        cpu = {"value": nrep * N * T / cpu_s, "unit": "p-dit updates/s", "cores": threads,
               "kind": "oracle",
               "sample": f"{nrep} of the {R} replicas, full {T}-sweep schedule, "
                         f"one replica per thread"}

    fast.close()
    out = {"metric": METRIC, "value": value, "unit": "p-dit updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
           "data": "synthetic",
           "config": {"workload": "qap_n64_uniform99", "N": N, "replicas": R, "sweeps": T,
                      "beta": "geometric 0.001->1.0", "recompute": "int8 mfma",
                      "sweep_kernel": "fast (table of swap energy changes in LDS, "
                                      "speculative rows)",
                      "parallelism": "replicas"},
           "acceptance": alpha, "ties": cnt["ties"], "roofline": roofline,
           "plain": plain_rec, "time_to_target": ttt, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
