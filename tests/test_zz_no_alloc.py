"""pdit_run_sweeps_noalloc (the entry point for callers that cannot
allocate device memory) against pdit_run_sweeps, called through the C ABI:
two calls in a row on the library's static scratch, the second on a
smaller input, then a resumed call and a run whose work space exceeds the
scratch; every output bit for bit equal to the context entry point's."""
import numpy as np
import pytest
import torch

from paper_2605_24408_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def say(msg):
    print(msg, flush=True)


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


def with_context(P, D, F, perms, beta, seed, offset, sweep, best=None):
    with P.Pdit(sweep=sweep) as ctx:
        p = dev(perms, torch.int32)
        ctx.set_sweep_offset(offset)
        ctx.run_sweeps(dev(D, torch.int32), dev(F, torch.int32), p, dev(beta, torch.float32), seed)
        Eb, pb = ctx.best()
        out = {"perm": p.cpu().numpy(), "E": ctx.energy().cpu().numpy(),
               "E_best": Eb.cpu().numpy(), "perm_best": pb.cpu().numpy(),
               "counters": ctx.replica_counters().cpu().numpy(), "plan": ctx.last_plan()}
    return out


def without_alloc(P, D, F, perms, beta, seed, offset, sweep, best=None):
    R, N = perms.shape
    p = dev(perms, torch.int32)
    E = torch.zeros(R, dtype=torch.int64, device=DEV)
    if best is None:
        Eb = torch.zeros(R, dtype=torch.int64, device=DEV)
        pb = torch.zeros((R, N), dtype=torch.int32, device=DEV)
    else:
        Eb, pb = dev(best[0], torch.int64), dev(best[1], torch.int32)
    cnt = torch.full((R, 3), -1, dtype=torch.int64, device=DEV)
    P.run_sweeps_noalloc(dev(D, torch.int32), dev(F, torch.int32), p, dev(beta, torch.float32),
                         seed, offset, E, Eb, pb, cnt, init_best=best is None, sweep=sweep)
    torch.cuda.synchronize()
    return {"perm": p.cpu().numpy(), "E": E.cpu().numpy(), "E_best": Eb.cpu().numpy(),
            "perm_best": pb.cpu().numpy(), "counters": cnt.cpu().numpy()}


def same(a, b, what):
    for key in ("perm", "E", "E_best", "perm_best", "counters"):
        assert np.array_equal(a[key], b[key]), f"{what}: {key}"


def test_noalloc_equals_context_entry_point():
    from paper_2605_24408_amd import pdit as P
    rng = np.random.default_rng(12)
    cases = [  # (N, R, T, max value, sweep): the second call is smaller than the first
        (64, 512, 40, 99, "auto"),    # table kernel, 8 MiB of H
        (40, 64, 30, 99, "auto"),     # table kernel, smaller
        (300, 8, 3, 10_000, "auto"),  # no on-chip class: the kernel without a stored H, int64 H
        (24, 16, 20, 9, "plain"),     # H in the scratch, read and rewritten by the plain kernel
    ]
    for N, R, T, vmax, sweep in cases:
        D, F = W.random_instance(rng, N, 0, vmax)
        perms = W.random_perms(rng, R, N)
        s = W.energy_scale(D, F)
        beta = W.beta_geometric(0.2 / s, 50.0 / s, T)
        say(f"noalloc N={N} R={R} T={T} sweep={sweep}")
        ref = with_context(P, D, F, perms, beta, 7, 11, sweep)
        got = without_alloc(P, D, F, perms, beta, 7, 11, sweep)
        same(ref, got, f"N={N}")
        assert got["counters"][:, 0].sum() == R * N * T
        assert got["counters"][:, 1].sum() > 0


def test_noalloc_resume_equals_one_call():
    """Two calls of T sweeps (the second from the first's state, best state
    and sweep offset) equal one context call of 2T sweeps."""
    from paper_2605_24408_amd import pdit as P
    rng = np.random.default_rng(3)
    N, R, T = 48, 32, 25
    D, F = W.random_instance(rng, N, 0, 60)
    perms = W.random_perms(rng, R, N)
    s = W.energy_scale(D, F)
    beta = W.beta_geometric(0.2 / s, 50.0 / s, 2 * T)
    one = with_context(P, D, F, perms, beta, 5, 0, "auto")
    a = without_alloc(P, D, F, perms, beta[:T], 5, 0, "auto")
    b = without_alloc(P, D, F, a["perm"], beta[T:], 5, T, "auto", best=(a["E_best"], a["perm_best"]))
    for key in ("perm", "E", "E_best", "perm_best"):
        assert np.array_equal(one[key], b[key]), key
    assert np.array_equal(one["counters"][:, :2], a["counters"][:, :2] + b["counters"][:, :2])


def test_noalloc_refuses_runs_beyond_its_scratch():
    """N = 256 x 512 replicas needs 128 MiB of H: refused with PDIT_ENOMEM
    and a message, the permutations untouched; a later call still runs."""
    from paper_2605_24408_amd import pdit as P
    inst = W.config_n256(R=512, T=2)
    with pytest.raises(P.PditError) as e:
        without_alloc(P, inst.D, inst.F, inst.perms, inst.beta, 2, 0, "auto")
    assert e.value.status == "PDIT_ENOMEM" and "scratch" in str(e.value)
    rng = np.random.default_rng(1)
    D, F = W.random_instance(rng, 20, 0, 9)
    perms = W.random_perms(rng, 4, 20)
    beta = np.full(5, 0.05, np.float32)
    same(with_context(P, D, F, perms, beta, 3, 0, "auto"),
         without_alloc(P, D, F, perms, beta, 3, 0, "auto"), "after a refusal")
