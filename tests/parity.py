"""GPU-oracle parity protocol shared by the GPU tests.

Both paths evaluate Eq. 5 on the same exact integer energy changes and the
same Philox uniforms; they differ only in how the weights are rounded (the
oracle in double precision, the kernels on integer weights), so a draw may
differ only where the oracle flags a tie (tau within 2^-20 Z of a boundary
between candidates of nonzero weight).

* ``replay``: for runs whose draws the GPU recorded, the oracle replays the
  GPU's draws one by one.  At the first draw that differs from its own it
  checks that its own draw is a tie, adopts the GPU's candidate (re-syncing
  its state to the GPU's at that draw) and goes on; a difference off a tie
  fails at that draw.  The final states, energies, best states, energy
  traces and accepted counts must then be identical, the number of adopted
  draws is printed and bounded by the oracle's tie count, and the GPU's tie
  counter is compared with the oracle's.
* ``chunked``: for launches that do not record, the GPU runs in chunks and
  every chunk is compared replica by replica with an oracle run of the same
  chunk from the same state; a replica that differs must carry an oracle
  tie inside that chunk, and the oracle is re-synced to the GPU's state
  before the next chunk.
"""
from __future__ import annotations

import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def check_ties(gpu_ties: int, oracle_ties: int, what: str):
    """The kernels flag a tie on their own CDF with the same 2^-20 band; their
    boundaries are a subset of the oracle's (a weight they round to 0 is
    tiny but nonzero in double), so their ties are the oracle's except where
    tau sits at the band's edge: allow 2% of them plus 3."""
    assert gpu_ties <= oracle_ties + 0.02 * gpu_ties + 3, (
        f"{what}: the GPU counted {gpu_ties} ties, the oracle {oracle_ties}")


def replay(got, D, F, perms, beta, seed, offset=0, rows=None, rep_ids=None, inst_id=0,
           E_best=None, perm_best=None, threads=1, what="run"):
    """Draw-by-draw parity of a recorded GPU run (``got``: arrays perm, E,
    E_best, perm_best, counters, choices and optionally trace, indexed by
    the GPU's replica rows).  ``perms``: the initial permutations of the
    compared rows; ``rows``: which GPU rows (default all); ``rep_ids``:
    their Philox replica indices (default ``rows``).  Returns the oracle
    result."""
    perms = np.asarray(perms)
    R = perms.shape[0]
    rows = list(range(R)) if rows is None else list(rows)
    rep_ids = rows if rep_ids is None else list(rep_ids)
    forced = np.ascontiguousarray(got["choices"][rows])
    has_trace = got.get("trace") is not None

    def one(i):
        return oracle.run(D, F, perms[i:i + 1], beta, seed, sweep_offset=offset,
                          rep_ids=[rep_ids[i]], inst_id=inst_id,
                          E_best=None if E_best is None else [E_best[i]],
                          perm_best=None if perm_best is None else perm_best[i:i + 1],
                          record_trace=has_trace, forced=forced[i:i + 1])

    if threads > 1 and R > 1:
        with ThreadPoolExecutor(min(threads, R)) as ex:
            parts = list(ex.map(one, range(R)))
    else:
        parts = [one(i) for i in range(R)]
    excused = 0
    o_ties = g_ties = 0
    for i, (k, ref) in enumerate(zip(rows, parts)):
        tag = f"{what}: replica {k}"
        assert np.array_equal(got["perm"][k], ref.perm[0]), tag + " permutation"
        assert got["E"][k] == ref.E[0], tag + " energy"
        assert got["E_best"][k] == ref.E_best[0], tag + " best energy"
        assert np.array_equal(got["perm_best"][k], ref.perm_best[0]), tag + " best state"
        assert np.array_equal(got["counters"][k][:2], ref.counters[0][:2]), tag + " counters"
        if has_trace:
            assert np.array_equal(got["trace"][k], ref.E_trace[0]), tag + " energy trace"
        excused += int(ref.excused[0])
        assert ref.excused[0] <= ref.counters[0][2]
        o_ties += int(ref.counters[0][2])
        g_ties += int(got["counters"][k][2])
    check_ties(g_ties, o_ties, what)
    updates = sum(int(p.counters[0][0]) for p in parts)
    say(f"{what}: {len(rows)} replicas, {updates} draws replayed, {excused} adopted at oracle "
        f"ties; ties: GPU {g_ties}, oracle {o_ties}")
    return parts


def chunked(run_gpu_chunk, run_oracle_chunk, state0, n_chunks, what="run", max_resync=None):
    """Chunk-by-chunk parity for launches that do not record their draws.

    run_gpu_chunk(c) -> dict of per-replica arrays after chunk c (keys perm,
        E, E_best, perm_best, counters, plus any others the oracle side
        returns);
    run_oracle_chunk(c, state) -> (dict of the same arrays, ties per replica
        in that chunk), starting from ``state`` (the same dict layout);
    state0: the common starting state.
    Replica k may differ after a chunk only if the oracle counted a tie for
    it in that chunk; the oracle is then re-synced to the GPU's state.
    Returns the number of re-syncs."""
    state = {k: np.array(v, copy=True) for k, v in state0.items()}
    resync = 0
    for c in range(n_chunks):
        g = run_gpu_chunk(c)
        o, ties = run_oracle_chunk(c, state)
        R = len(o["E"])
        for k in range(R):
            same = all(np.array_equal(g[key][k], o[key][k]) for key in o)
            if not same:
                assert ties[k] > 0, (f"{what}: chunk {c}, replica {k} differs from the oracle "
                                     f"with no oracle tie in the chunk")
                resync += 1
        state = {k: np.array(v, copy=True) for k, v in g.items()}
    if max_resync is not None:
        assert resync <= max_resync, f"{what}: {resync} re-syncs"
    say(f"{what}: {n_chunks} chunks, {resync} replica re-syncs at oracle ties")
    return resync
