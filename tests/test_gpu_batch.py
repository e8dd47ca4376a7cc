"""GPU parity of batched searches (grover_batch_*): many independent instances of Algorithm 5 in one
persistent launch, complex64 states with binary64 update and sums.

Every instance is compared with the oracle's search (binary64) under the tolerance derived in
test_gpu_precision.error_bound for complex64 storage and binary64 sums.  Each instance starts from the
uniform superposition, so its exact state has two values only (marked, unmarked); the device computes every
amplitude of a class from identical inputs, so each class must also be bitwise constant — a property that
holds at any size and is checked at full size below.
"""
from __future__ import annotations

import numpy as np
import pytest

import workloads
from test_gpu_precision import error_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_04635_amd as pkg

    pkg.load()
    return pkg


def small_batch():
    """(n, marks, iterations or None) per instance: sizes that span the register-held form (n <= 14), the
    streamed one, several tiles and ragged tiles, marked lists dense within one tile and degenerate sets."""
    rows = [
        (1, [0], None), (2, [3], None), (3, [5], None), (3, [1, 6], 3), (4, [], None), (4, list(range(16)), None),
        (5, [0, 31], 3), (6, [17], 0), (8, [1, 2, 200], None), (9, [511], None), (10, [5], None),
        (11, [3, 700, 1500, 2047], None), (12, list(range(1000, 1008)), None), (13, [4096, 8191], None),
        (14, [12345], None), (14, [0, 1, 2, 3, 9000], 40), (15, [7], 30), (15, list(range(40, 340)), 12),
        (16, [1, 60000], 25), (16, [65535], 12), (17, [77777], 9), (18, [3, 262143], 6),
    ]
    extra = workloads.BatchWorkload("small", 24, 8, 7, 8, seed=97)
    n, m, mk = extra.instances()
    rows += [(int(n[b]), mk[b].tolist(), None) for b in range(extra.count)]
    return rows


def iterations(orc, rows):
    return [orc.optimal_iterations(n, len(mk)) if k is None else k for n, mk, k in rows]


def make(G, rows):
    iters = [k for _, _, k in rows]
    return G.GroverBatch([r[0] for r in rows], [len(r[1]) for r in rows], [r[1] for r in rows],
                         iterations=None if all(k is None for k in iters) else
                         [G.grover_optimal_iterations(n, len(mk)) if k is None else k for n, mk, k in rows])


@pytest.fixture(scope="module")
def expected(orc):
    rows = small_batch()
    ks = iterations(orc, rows)
    return [orc.search(n, mk, k) for (n, mk, _), k in zip(rows, ks)], ks


def check_against(orc_states, ks, rows, read, team):
    for i, ((n, mk, _), want, k) in enumerate(zip(rows, orc_states, ks)):
        got = read(i).astype(np.complex128)
        err = float(np.max(np.abs(got - want)))
        assert err <= error_bound(n, max(k, 1), "c64", "f64", 1), (i, n, len(mk), k, team, err)


@pytest.mark.parametrize("split,team", [(0, 1), (12, 2), (10, 4), (0, 4), (14, 0)])
def test_small_batch_matches_oracle(G, expected, split, team):
    rows = small_batch()
    b = make(G, rows)
    grid = b.query(G.grover.BQ_GRID)
    b.set_tiling(split, team if team else grid)  # team 0 here: the whole grid per instance
    assert b.query(G.grover.BQ_TEAM) == (team if team else grid)
    b.run()
    b.sync()
    check_against(*expected, rows, b.read_state, team)
    b.close()


def test_batch_runs_are_bitwise_reproducible_and_graph_replays_match(G):
    import torch

    rows = small_batch()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = make(G, rows)
        b.set_tiling(12, 2)
        b.run()
        b.sync()
        first = [b.read_state(i) for i in range(b.count)]
        b.run()
        b.sync()
        for i in range(b.count):
            assert np.array_equal(b.read_state(i).view(np.uint32), first[i].view(np.uint32)), i
        b.capture()
        assert b.query(G.grover.BQ_GRAPH) == 1
        other = torch.zeros(1 << 20, device="cuda")
        for rep in range(3):
            other.add_(1.0)  # eager work of the program between replays
            torch.cuda.synchronize()
            b.run()
            b.sync()
            for i in range(b.count):
                assert np.array_equal(b.read_state(i).view(np.uint32), first[i].view(np.uint32)), (rep, i)
        b.close()


def test_graph_replay_rewrites_the_states(G):
    """A replay must recompute from the uniform start: overwrite states on the device, replay, compare."""
    import ctypes

    import torch

    # by its soname, so that the HIP runtime already in the process (torch's, which libgrover shares) is the
    # one called; another copy of the runtime would not know these device allocations
    hip = ctypes.CDLL("libamdhip64.so.7")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    device_to_device = 3
    rows = small_batch()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = make(G, rows)
        b.run()
        b.sync()
        want = [b.read_state(i) for i in range(b.count)]
        b.capture()
        for i in (0, 14, 20):
            ptr, nbytes = G.grover_batch_state(b.b, i)
            junk = torch.full((nbytes // 4,), 7.0, device="cuda")
            torch.cuda.synchronize()
            assert hip.hipMemcpy(ptr, junk.data_ptr(), nbytes, device_to_device) == 0
            torch.cuda.synchronize()  # a device-to-device copy may return before it is done
            assert not np.array_equal(b.read_state(i).view(np.uint32), want[i].view(np.uint32))
        b.run()
        b.sync()
        for i in range(b.count):
            assert np.array_equal(b.read_state(i).view(np.uint32), want[i].view(np.uint32)), i
        b.close()


def test_batch_tune_selects_a_candidate_and_stays_correct(G, expected):
    rows = small_batch()
    b = make(G, rows)
    split, team, ms = b.tune()
    assert ms > 0.0 and (team == 1 or (split in (18, 19, 20) and team in (2, 4, 8, 16)))
    assert (b.query(G.grover.BQ_SPLIT), b.query(G.grover.BQ_TEAM)) == (split, team)
    b.run()
    b.sync()
    check_against(*expected, rows, b.read_state, team)
    b.close()


def test_batch_queries_and_tiling_limits(G, orc):
    rows = small_batch()
    b = make(G, rows)
    ks = iterations(orc, rows)
    assert b.query(G.grover.BQ_COUNT) == len(rows)
    assert b.query(G.grover.BQ_UPDATES) == sum((1 << n) * k for (n, _, _), k in zip(rows, ks))
    grid = b.query(G.grover.BQ_GRID)
    assert grid >= 1
    with pytest.raises(G.GroverError):
        b.set_tiling(10, 0)
    with pytest.raises(G.GroverError):
        b.set_tiling(10, grid + 1)
    b.set_tiling(15, 2)
    assert b.query(G.grover.BQ_N_TEAM) == sum(1 for n, _, _ in rows if n >= 15)
    ptr, nbytes = G.grover_batch_state(b.b, 3)
    assert ptr % 256 == 0 and nbytes == (1 << rows[3][0]) * 8
    with pytest.raises(G.GroverError):
        G.grover_batch_state(b.b, len(rows))
    with pytest.raises(G.GroverError):
        G.grover_batch_read_state(b.b, 0, 0, 8)
    b.close()


def test_batch_barrier_timeout_is_reported(G, expected, monkeypatch):
    """A wait limit of zero makes every team barrier that has to wait give up; the failure must surface at
    sync, and a fresh batch afterwards must work."""
    monkeypatch.setenv("GROVER_BARRIER_TIMEOUT_MS", "0")
    rows = small_batch()
    b = make(G, rows)
    b.set_tiling(10, 8)
    b.run()
    with pytest.raises(G.GroverError) as e:
        b.sync()
    assert e.value.status == G.grover.GROVER_E_TIMEOUT
    b.close()
    monkeypatch.delenv("GROVER_BARRIER_TIMEOUT_MS")
    b = make(G, rows)
    b.set_tiling(10, 8)
    b.run()
    b.sync()
    check_against(*expected, rows, b.read_state, 8)
    b.close()
