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
    """(n, marks, iterations or None) per instance: sizes that span the form one workgroup holds on chip
    (n <= 15), the team-held and streamed ones, several tiles and ragged tiles, marked lists dense within one tile and degenerate sets."""
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


@pytest.mark.parametrize("split,team,resident", [(0, 1, 0), (12, 2, 0), (10, 4, 0), (0, 4, 0), (14, 0, 0),
                                                 (19, 2, 8), (0, 1, 4), (10, 2, 2), (15, 4, 1), (0, 0, 8),
                                                 (19, 2, 16), (0, 1, 16), (12, 4, 16)])
def test_small_batch_matches_oracle(G, expected, split, team, resident):
    """Streamed tilings (resident = 0) and teams that hold the state on chip (resident vectors per thread r,
    up to 8 in registers and 8 more in LDS: a state of nvec vectors is held by the power of two
    >= nvec / (1024 r) workgroups); team 0 here means the whole grid per streamed instance."""
    rows = small_batch()
    b = make(G, rows)
    grid = b.query(G.grover.BQ_GRID)
    b.set_tiling(split, team if team else grid, resident)
    assert b.query(G.grover.BQ_TEAM) == (team if team else grid)
    assert b.query(G.grover.BQ_RESIDENT) == resident
    # every state here (n <= 18) fits on chip when resident > 0: the kernel without streamed paths runs
    assert b.query(G.grover.BQ_STREAMS) == (0 if resident else 1)
    b.run()
    b.sync()
    check_against(*expected, rows, b.read_state, (team, resident))
    b.close()


@pytest.mark.parametrize("split,team,resident", [(19, 2, 16), (19, 2, 8), (0, 1, 0), (20, 0, 4)])
def test_large_instances_match_oracle(G, orc, split, team, resident):
    """The largest instance sizes (n = 21 ... 24) with a few iterations each, beside small ones: with 16
    vectors per thread they are held by teams of 64, 128 and 256 workgroups (the whole grid) and n = 24
    streams; with 8, n >= 23 streams; (0, 1, 0) streams every large state through one workgroup; team 0 is
    the whole grid per streamed instance."""
    rows = [(24, [1, 16777215], 3), (23, [4194304], 4), (22, [0, 7, 3000000], 3), (21, [2097151], 5),
            (20, [12345], 2), (9, [3], None), (15, [0, 32767], 6)]
    ks = iterations(orc, rows)
    b = make(G, rows)
    grid = b.query(G.grover.BQ_GRID)
    if team == 0 and grid & (grid - 1):
        b.close()
        pytest.skip("a whole-grid streamed team nests inside the resident teams only for a power-of-two grid")
    b.set_tiling(split, team if team else grid, resident)
    assert b.query(G.grover.BQ_STREAMS) == 1  # n = 24 never fits on chip
    b.run()
    b.sync()
    for i, ((n, mk, _), k) in enumerate(zip(rows, ks)):
        want = orc.search(n, mk, k)
        got = b.read_state(i).astype(np.complex128)
        err = float(np.max(np.abs(got - want)))
        assert err <= error_bound(n, max(k, 1), "c64", "f64", 1), (i, n, k, split, team, resident, err)
    b.close()


def test_batch_runs_are_bitwise_reproducible_and_graph_replays_match(G):
    import torch

    rows = small_batch()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = make(G, rows)
        b.set_tiling(12, 2, 4)
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
    split, team, resident, ms = b.tune()
    assert ms > 0.0 and (team == 1 or (split in (18, 19, 20) and team in (2, 4, 8)))
    assert resident in (0, 4, 8, 16)
    assert (b.query(G.grover.BQ_SPLIT), b.query(G.grover.BQ_TEAM), b.query(G.grover.BQ_RESIDENT)) == (split, team,
                                                                                                     resident)
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
    with pytest.raises(G.GroverError):
        b.set_tiling(10, 2, 3)  # resident vectors must be a power of two <= 16
    with pytest.raises(G.GroverError):
        b.set_tiling(10, 2, 32)
    # a streamed team of 3 could not nest inside resident teams of 2, 4, ...; here every state fits on chip
    # in a resident team (n <= 18), so no streamed phase exists and the tiling is accepted
    b.set_tiling(10, 3, 8)
    assert b.query(G.grover.BQ_PHASES) == 1 + len({n for n, _, _ in rows if n >= 16})
    # states of n <= 15 are held by one workgroup whatever the tiling; the rest stream in teams of 2
    b.set_tiling(15, 2)
    assert b.query(G.grover.BQ_N_TEAM) == sum(1 for n, _, _ in rows if n >= 16)
    assert b.query(G.grover.BQ_PHASES) == 2
    # resident teams of 2^k workgroups for n = 16 .. 18 (8 vectors per thread), nothing streamed
    b.set_tiling(15, 2, 8)
    assert b.query(G.grover.BQ_N_TEAM) == sum(1 for n, _, _ in rows if n >= 16)
    assert b.query(G.grover.BQ_PHASES) == 1 + len({n for n, _, _ in rows if n >= 16})
    # 16 vectors per thread: n = 16 on 2 workgroups, 17 on 4, 18 on 8
    b.set_tiling(15, 2, 16)
    assert b.query(G.grover.BQ_PHASES) == 1 + len({n for n, _, _ in rows if n >= 16})
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
    b.set_tiling(10, 8, 2)
    b.run()
    with pytest.raises(G.GroverError) as e:
        b.sync()
    assert e.value.status == G.grover.GROVER_E_TIMEOUT
    b.close()
    monkeypatch.delenv("GROVER_BARRIER_TIMEOUT_MS")
    b = make(G, rows)
    b.set_tiling(10, 8, 2)
    b.run()
    b.sync()
    check_against(*expected, rows, b.read_state, 8)
    b.close()
