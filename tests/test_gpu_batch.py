"""GPU parity of batched runs (instances of uneven size in persistent,
graph-captured launches): every draw of every (instance, replica) recorded
and replayed on the oracle with the instance's own Philox word (the
protocol of ``parity.py``), graph replays against resumed oracle runs, the
autotuner, and the full-size uneven workload on sampled replicas."""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
from paper_2605_24408_amd import workloads as W
from parity import replay

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).to(DEV)


def small_batch(T=30, R=3):
    """Instances across every kernel class: N <= 16, 32, 64, 128 on chip,
    N > 128 on the plain kernel; zero and nonzero diagonals."""
    rng = np.random.default_rng(77)
    out = []
    for k, (N, zd) in enumerate([(12, True), (20, False), (40, True), (64, True), (70, False),
                                 (100, True), (130, True), (9, True)]):
        D, F = W.random_instance(rng, N, 0, 40, zero_diag=zd)
        perms = W.random_perms(rng, R, N)
        s = W.energy_scale(D, F)
        beta = W.beta_geometric(0.2 / s, 50.0 / s, T)
        out.append((D, F, perms, beta))
    return out


def to_dev(batch, record=True):
    """Device tensors of a batch; with ``record`` every instance also gets
    buffers for its draws and energy trace."""
    out = []
    for D, F, p, b in batch:
        R, N = p.shape
        T = len(b)
        item = (dev(D, torch.int32), dev(F, torch.int32), dev(p, torch.int32),
                dev(b, torch.float32))
        if record:
            item = item + (torch.full((R, T, N), -1, dtype=torch.int32, device=DEV),
                           torch.zeros((R, T), dtype=torch.int64, device=DEV))
        out.append(item)
    return out


def replay_batch(got, batch, seed, sweep_offset=0, start=None, what="batch"):
    """Every replica of every instance replayed draw by draw on the oracle
    (instance index k as Philox word 3); ``start``: per instance the
    previous call's GPU state (perm, E_best, perm_best) to resume from."""
    for k, ((D, F, perms, beta), g) in enumerate(zip(batch, got)):
        if start is not None:
            perms = start[k]["perm"]
        replay(g, D, F, perms, beta, seed, offset=sweep_offset, inst_id=k,
               E_best=None if start is None else start[k]["E_best"],
               perm_best=None if start is None else start[k]["perm_best"],
               what=f"{what}, instance {k} (N={D.shape[0]})")


def gpu_state(ctx, dbatch):
    E = ctx.energy().cpu().numpy()
    Eb, pb = ctx.best()
    Eb, pb = Eb.cpu().numpy(), pb.cpu().numpy()
    cnt = ctx.replica_counters().cpu().numpy()
    out, rb, po = [], 0, 0
    for item in dbatch:
        perm = item[2]
        R, N = perm.shape
        st = dict(perm=perm.cpu().numpy(), E=E[rb:rb + R], E_best=Eb[rb:rb + R],
                  perm_best=pb[po:po + R * N].reshape(R, N), counters=cnt[rb:rb + R])
        if len(item) > 4:
            st["choices"] = item[4].cpu().numpy()
            st["trace"] = item[5].cpu().numpy()
        out.append(st)
        rb += R
        po += R * N
    return out


@pytest.mark.parametrize("sweep", ["auto", "plain"])
def test_batch_matches_oracle(sweep):
    from paper_2605_24408_amd import pdit as P
    batch = small_batch()
    say(f"batch vs oracle, sweep={sweep}")
    dbatch = to_dev(batch)
    with P.Pdit(sweep=sweep) as ctx:
        ctx.run_sweeps_batch(dbatch, 5)
        torch.cuda.synchronize()
        got = gpu_state(ctx, dbatch)
    replay_batch(got, batch, 5, what=f"batch {sweep}")
    assert sum(int(g["counters"][:, 1].sum()) for g in got) > 100
    # without recording (the kernels that skip it): the same results
    plain = to_dev(batch, record=False)
    with P.Pdit(sweep=sweep) as ctx:
        ctx.run_sweeps_batch(plain, 5)
        torch.cuda.synchronize()
        unrec = gpu_state(ctx, plain)
    for g, u in zip(got, unrec):
        for key in ("perm", "E", "E_best", "perm_best", "counters"):
            assert np.array_equal(g[key], u[key]), key


def test_batch_graph_replays_match_resumed_oracle():
    """Three calls with the same shapes: the first captures the graph, the
    next two replay it (seed and sweep offset come from device memory).  Host
    work and synchronisations run between the replays; every call is checked
    against the oracle resumed from the previous state."""
    from paper_2605_24408_amd import pdit as P
    batch = small_batch(T=12, R=2)
    dbatch = to_dev(batch)
    prev = None
    with P.Pdit() as ctx:
        for call in range(3):
            say(f"graph call {call}")
            ctx.run_sweeps_batch(dbatch, 9)
            torch.cuda.synchronize()
            got = gpu_state(ctx, dbatch)
            replay_batch(got, batch, 9, sweep_offset=12 * call, start=prev,
                         what=f"graph call {call}")
            prev = got
            _ = torch.randn(1000, device=DEV).sum().item()  # unrelated eager work
        assert ctx.get_sweep_offset() == 36


def test_batch_instance0_equals_single_run():
    from paper_2605_24408_amd import pdit as P
    batch = small_batch(T=20)
    dbatch = to_dev(batch, record=False)
    with P.Pdit() as ctx:
        ctx.run_sweeps_batch(dbatch, 3)
        torch.cuda.synchronize()
        got = gpu_state(ctx, dbatch)[0]
    D, F, perms, beta = batch[0]
    with P.Pdit() as ctx:
        perm = dev(perms, torch.int32)
        ctx.run_sweeps(dev(D, torch.int32), dev(F, torch.int32), perm, dev(beta, torch.float32), 3)
        E = ctx.energy().cpu().numpy()
        torch.cuda.synchronize()
    assert np.array_equal(perm.cpu().numpy(), got["perm"])
    assert np.array_equal(E, got["E"])


def test_autotune_then_run():
    from paper_2605_24408_amd import pdit as P
    batch = small_batch(T=10, R=2)
    dbatch = to_dev(batch)
    before = [item[2].clone() for item in dbatch]
    with P.Pdit() as ctx:
        t = ctx.autotune(dbatch, 10, 4)
        assert t["blocks_per_cu"] >= 1 and t["seq_threshold"] >= 1 and t["best_ms"] > 0
        for b, item in zip(before, dbatch):
            assert torch.equal(b, item[2])  # the trials ran on private copies
            assert (item[4] == -1).all()   # and recorded nothing
        ctx.run_sweeps_batch(dbatch, 4)
        torch.cuda.synchronize()
        got = gpu_state(ctx, dbatch)
    replay_batch(got, batch, 4, what="after autotune")


def test_autotune_cache(tmp_path, monkeypatch):
    """PDIT_AUTOTUNE_CACHE: the first call runs the trials and appends its
    setting under the batch's key; a second context takes it from the file
    without trials; a batch of another shape misses and adds a line."""
    from paper_2605_24408_amd import pdit as P
    cache = tmp_path / "autotune.txt"
    monkeypatch.setenv("PDIT_AUTOTUNE_CACHE", str(cache))
    dbatch = to_dev(small_batch(T=6, R=2), record=False)
    with P.Pdit() as ctx:
        first = ctx.autotune(dbatch, 6, 4)
    assert not first["cached"]
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and lines[0].split()[1:3] == [str(first["blocks_per_cu"]),
                                                       str(first["seq_threshold"])]
    assert lines[0].split()[0].count("/") == 1 + len(dbatch)   # arch/CUs, then one part per instance
    with P.Pdit() as ctx:
        second = ctx.autotune(dbatch, 6, 4)
        ctx.run_sweeps_batch(dbatch, 4)
        torch.cuda.synchronize()
    assert second["cached"]
    assert (second["blocks_per_cu"], second["seq_threshold"]) == (first["blocks_per_cu"],
                                                                  first["seq_threshold"])
    other = to_dev(small_batch(T=6, R=3), record=False)
    with P.Pdit() as ctx:
        third = ctx.autotune(other, 6, 4)
    assert not third["cached"]
    assert len(cache.read_text().splitlines()) == 2


def test_uneven_workload_full_size_sampled():
    """The uneven workload at full size (256 instances, N in [20, 150], 64
    replicas each, 2000 sweeps) in one batched call, then again with every
    draw recorded (identical results); replica 5 of five sampled instances
    replayed draw by draw on the oracle, properties checked on many more."""
    from paper_2605_24408_amd import pdit as P
    insts = W.config_uneven()
    dbatch = [(dev(i.D, torch.int32), dev(i.F, torch.int32), dev(i.perms, torch.int32),
               dev(i.beta, torch.float32)) for i in insts]
    say("uneven workload on the GPU")
    with P.Pdit() as ctx:
        ctx.run_sweeps_batch(dbatch, W.PHILOX_SEED)
        torch.cuda.synchronize()
        got = gpu_state(ctx, dbatch)
    Ns = [i.N for i in insts]
    sample = [int(np.argmax(Ns)), int(np.argmin(Ns)), 1, 2, 3]
    say("uneven workload, sampled instances recorded")
    rec = [(dev(i.D, torch.int32), dev(i.F, torch.int32), dev(i.perms, torch.int32),
            dev(i.beta, torch.float32))
           + ((torch.full((i.R, i.T, i.N), -1, dtype=torch.int32, device=DEV),
               torch.zeros((i.R, i.T), dtype=torch.int64, device=DEV)) if k in sample else ())
           for k, i in enumerate(insts)]
    with P.Pdit() as ctx:
        ctx.run_sweeps_batch(rec, W.PHILOX_SEED)
        torch.cuda.synchronize()
        grec = gpu_state(ctx, rec)
    for g, r in zip(got, grec):
        for key in ("perm", "E", "E_best", "perm_best", "counters"):
            assert np.array_equal(g[key], r[key]), key
    say("uneven workload: sampled oracle replicas")

    def one(k):
        i = insts[k]
        replay(grec[k], i.D, i.F, i.perms[5:6], i.beta, W.PHILOX_SEED, rows=[5], inst_id=k,
               what=f"uneven instance {k} (N={i.N}) replica 5")

    with ThreadPoolExecutor(5) as ex:
        list(ex.map(one, sample))
    for k in range(0, 256, 17):
        i = insts[k]
        for j in (0, 63):
            assert sorted(got[k]["perm"][j]) == list(range(i.N))
            assert got[k]["E"][j] == oracle.energy(i.D, i.F, got[k]["perm"][j])
            assert got[k]["E_best"][j] == oracle.energy(i.D, i.F, got[k]["perm_best"][j])
            assert got[k]["counters"][j][0] == i.N * 2000


def large_batch(T=3, R=2):
    """Instances that no on-chip class takes (N > 256, or values beyond the
    fast kernels' exact range) beside table-kernel ones: every copy layout
    and product width of the kernel without a stored H, int32 and int64 H."""
    rng = np.random.default_rng(91)
    out = []
    for N, hi in [(300, 40), (40, 40), (140, 100_000), (260, 10_000), (70, 30_000), (512, 99)]:
        D = W.sym_uniform(rng, N, 0, hi)
        F = W.sym_uniform(rng, N, 0, 40 if hi == 100_000 else hi)
        perms = W.random_perms(rng, R, N)
        s = W.energy_scale(D, F)
        beta = W.beta_geometric(0.1 / s, 30.0 / s, T)
        out.append((D, F, perms, beta))
    return out


@pytest.mark.parametrize("sweep", ["auto", "large"])
def test_batch_large_groups(sweep):
    """Batched runs put the instances without an on-chip class on the
    persistent kernel without a stored H (grouped by copy layout, product
    width and H width); every replica matches the oracle, and a second call
    (the captured graph replayed) matches the resumed oracle."""
    from paper_2605_24408_amd import pdit as P
    batch = large_batch()
    dbatch = to_dev(batch)
    say(f"batch large groups sweep={sweep}")
    with P.Pdit(sweep=sweep) as ctx:
        ctx.run_sweeps_batch(dbatch, 21)
        got = gpu_state(ctx, dbatch)
        replay_batch(got, batch, 21, what=f"large groups {sweep}")
        ctx.run_sweeps_batch(dbatch, 21)
        got2 = gpu_state(ctx, dbatch)
    replay_batch(got2, batch, 21, sweep_offset=3, start=got, what=f"large groups {sweep}, replay")
