"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on the same seeded inputs.

Tolerances (max absolute amplitude error against the binary64 oracle): 1e-12 for binary64 storage
(f64, c128) and 1e-5 for complex64 storage. Integer results (marked lists, sampled indices) must match
exactly.
"""
from __future__ import annotations

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "c128": 1e-12, "c64": 1e-5}


@pytest.fixture(scope="module")
def G():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_04635_amd as pkg

    pkg.load()
    return pkg


def as_c128(psi: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(psi.astype(np.complex128))


def start_state(n: int, dtype: str, seed: int) -> np.ndarray:
    """Random start state, already rounded to the storage type (the oracle starts from the same values)."""
    psi = workloads.random_state(n, seed, real=(dtype == "f64"))
    if dtype == "f64":
        return psi.real.astype(np.float64)
    return psi.astype(np.complex64 if dtype == "c64" else np.complex128)


def assert_close(got: np.ndarray, want: np.ndarray, dtype: str, what: str = ""):
    err = float(np.max(np.abs(as_c128(got) - want))) if want.size else 0.0
    assert err <= TOL[dtype], f"{what} max|err| = {err:.3e} > {TOL[dtype]}"
    return err


# ------------------------------------------------------------------------------ the n = 10 workload
def test_plain_n10_workload_end_to_end(G, orc):
    """n = 10, real binary64, one marked index from a seed, 25 iterations, 10^4 shots."""
    w = workloads.PLAIN_N10
    g = G.Grover(w.n, w.dtype, marks=list(w.marks))
    assert g.query(0) == 2  # resident form
    g.iterate(w.iterations)
    want = orc.search(w.n, list(w.marks), w.iterations)
    got = g.read_state()
    assert_close(got, want, "f64", "state")
    assert abs(g.norm() - 1.0) < 1e-13
    u = workloads.uniforms_u53(w.shot_seed, w.shots)
    shots = g.sample(w.shots, u53=u)
    # bit-exact on identical input: the oracle sampler on the GPU's own state
    assert np.array_equal(shots, orc.sample(as_c128(got), u))
    # end to end: the oracle's state gives the same shots here (state difference ~1e-16)
    assert np.array_equal(shots, orc.sample(want, u))
    assert np.mean(shots == w.marks[0]) > 0.99
    g.close()


# ----------------------------------------------------------------------------- elementwise parity
CASES = []
for form, ns in [("resident", [1, 2, 3, 5, 10, 12, 14]), ("fused", [1, 3, 9, 11, 13, 15, 17, 20]),
                 ("two_pass", [1, 4, 10, 16, 19])]:
    for n in ns:
        for dtype in ["f64", "c64", "c128"]:
            CASES.append((form, n, dtype))
# the held form (complex64 only): one workgroup with fewer vectors than threads (n = 1 .. 9), registers only
# (about 2 vectors per thread on teams of 4 .. 64 workgroups at n = 14 .. 17, up to 8 per thread on 64 and
# 128 workgroups at n = 18 .. 21), 8 more vectors per thread in LDS (n = 22, 23: teams of 128 and 256)
for n in [1, 3, 9, 14, 15, 17, 20, 21, 23]:
    CASES.append(("held", n, "c64"))


@pytest.mark.parametrize("form,n,dtype", CASES)
def test_iterate_matches_oracle(G, orc, form, n, dtype):
    """Random start state (complex unless real storage), several marked-set sizes and iteration counts."""
    N = 1 << n
    for mi, m in enumerate(sorted({0, 1, min(3, N), max(1, N // 3), N})):
        marks = workloads.distinct_marks(n, m, seed=11 * n + m)
        psi0 = start_state(n, dtype, seed=1000 + n + mi)
        g = G.Grover(n, dtype, marks=marks, form=form)
        g.write_state(psi0)
        want = as_c128(psi0)
        done = 0
        for k in (0, 1, 6):
            g.iterate(k)
            orc.iterate(want, marks, k)
            done += k
            assert_close(g.read_state(), want, dtype, f"{form} n={n} m={m} k={done}")
        g.close()


@pytest.mark.parametrize("form,n,dtype", [("resident", 10, "c64"), ("fused", 16, "c64"), ("fused", 18, "c128"),
                                          ("two_pass", 14, "f64"), ("fused", 12, "f64"), ("held", 18, "c64"),
                                          ("held", 22, "c64")])
def test_search_to_optimum_matches_oracle_and_closed_form(G, orc, form, n, dtype):
    m = 3
    marks = workloads.distinct_marks(n, m, seed=n)
    k = orc.optimal_iterations(n, m)
    g = G.Grover(n, dtype, marks=marks, form=form)
    g.iterate(k)
    got = g.read_state()
    assert_close(got, orc.search(n, marks, k), dtype, "state")
    a, b = orc.two_class(n, m, k)
    mask = np.zeros(1 << n, dtype=bool)
    mask[marks.astype(np.int64)] = True
    # two-class structure holds exactly in any precision
    assert np.all(got[mask] == got[mask][0]) and np.all(got[~mask] == got[~mask][0])
    assert abs(complex(got[mask][0]) - a) <= TOL[dtype] and abs(complex(got[~mask][0]) - b) <= TOL[dtype]
    if dtype != "f64":
        assert np.all(got.imag == 0)
    g.close()


@pytest.mark.parametrize("form,n", [("resident", 9), ("fused", 13), ("fused", 19), ("fused", 24), ("two_pass", 12),
                                    ("held", 16), ("held", 21)])
def test_iterate_composes_bitwise(G, form, n):
    """iterate(a); iterate(b) equals iterate(a + b) bit for bit, and reruns are bitwise identical."""
    marks = workloads.distinct_marks(n, 5, seed=3)
    psi0 = start_state(n, "c64", seed=77)
    ga = G.Grover(n, "c64", marks=marks, form=form).write_state(psi0)
    gb = G.Grover(n, "c64", marks=marks, form=form).write_state(psi0)
    ga.iterate(7).iterate(0).iterate(13)
    gb.iterate(20)
    sa, sb = ga.read_state(), gb.read_state()
    assert np.array_equal(sa.view(np.uint32), sb.view(np.uint32))
    gb.write_state(psi0).iterate(20)
    assert np.array_equal(gb.read_state().view(np.uint32), sb.view(np.uint32))
    ga.close()
    gb.close()


def test_fused_grid_shapes(G, orc, monkeypatch):
    """Forced persistent-grid sizes over the 16 tiles of an n = 16 complex128 state (each workgroup holds
    its last 6 tiles on chip, 2 in LDS and then 4 in registers): a single workgroup (10 tiles streamed
    before the held ones), 2 workgroups (8 tiles: 2 streamed), 3 (6, 5 and 5 tiles: none streamed, 2 or 1
    in LDS), 4 (4 tiles: registers only), 7 (3 and 2 tiles), a prime count (ragged shares) and more
    workgroups than tiles (empty shares); sparse marks and marks too many for a tile's registers."""
    n, dtype = 16, "c128"
    psi0 = start_state(n, dtype, seed=8)
    for m in [6, (1 << n) // 3]:
        marks = workloads.distinct_marks(n, m, seed=8)
        want = orc.iterate(as_c128(psi0), marks, 9)
        for grid in ["1", "2", "3", "4", "7", "97", "250"]:
            monkeypatch.setenv("GROVER_FUSED_GRID", grid)
            g = G.Grover(n, dtype, marks=marks, form="fused")
            assert g.query(1) == int(grid)
            g.write_state(psi0).iterate(9)
            assert_close(g.read_state(), want, dtype, f"grid={grid} m={m}")
            g.close()


def test_fused_access_form(G, orc, monkeypatch):
    """Up to 272 MiB of the state per pass streams with ordinary loads and stores (kept in the memory-side
    cache across iterations): the whole of a state that small, else the leading tiles of each workgroup's
    share, the rest with nontemporal accesses.  Every form gives the same results bit for bit: n = 24
    complex64 (8 tiles per workgroup, 2 streamed) all ordinary, all nontemporal and against the oracle;
    n = 26 complex64 (32 tiles per workgroup) split against all nontemporal."""
    budget = 272 << 20
    for n, dtype in [(16, "c64"), (24, "c128"), (25, "c64"), (25, "c128"), (26, "c64")]:
        g = G.Grover(n, dtype, marks=[3], form="fused")
        state = (1 << n) * g.query(G.grover.Q_ELEM_BYTES)
        share = g.query(G.grover.Q_GRID) * 4096 * 16
        want = state if state <= budget else min(state, budget // share * share)
        assert g.query(G.grover.Q_FUSED_TEMPORAL) == want, (n, dtype)
        g.close()

    def run(n, dtype, forced, psi0, marks, k1, k2):
        if forced is None:
            monkeypatch.delenv("GROVER_FUSED_TEMPORAL", raising=False)
        else:
            monkeypatch.setenv("GROVER_FUSED_TEMPORAL", forced)
        g = G.Grover(n, dtype, marks=marks, form="fused")
        state = (1 << n) * g.query(G.grover.Q_ELEM_BYTES)
        if forced is not None:
            assert g.query(G.grover.Q_FUSED_TEMPORAL) == (state if forced == "1" else 0)
        g.write_state(psi0).iterate(k1).iterate(k2)
        out = g.read_state()
        g.close()
        return out

    n, dtype = 24, "c64"
    psi0 = start_state(n, dtype, seed=24)
    marks = workloads.distinct_marks(n, 7, seed=24)
    a, b = run(n, dtype, "0", psi0, marks, 4, 5), run(n, dtype, "1", psi0, marks, 4, 5)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    assert_close(b, orc.iterate(as_c128(psi0), marks, 9), dtype, "n=24 fused")
    n = 26
    psi0 = start_state(n, dtype, seed=26)
    marks = workloads.distinct_marks(n, 9, seed=26)
    a, b = run(n, dtype, "0", psi0, marks, 2, 3), run(n, dtype, None, psi0, marks, 2, 3)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


@pytest.mark.parametrize("n,dtype", [(24, "f64"), (23, "c128"), (24, "c64"), (25, "cbf16")])
def test_fused_nontemporal_stores(G, orc, monkeypatch, n, dtype):
    """128 MiB states, large enough that each workgroup streams tiles besides the six (bfloat16: three) it
    holds on chip, in the kernel variant that streams every tile with nontemporal loads and stores (each
    storage type's own store bits: nt sc1 for binary64 and complex128, nt for complex64 and bfloat16):
    bit for bit the results of ordinary accesses, and for the binary64-sum types within tolerance of the
    oracle."""
    psi0 = workloads.random_state(n, 500 + n, real=(dtype == "f64"))
    if dtype == "f64":
        psi0 = psi0.real.astype(np.float64)
    elif dtype != "cbf16":
        psi0 = psi0.astype(np.complex64 if dtype == "c64" else np.complex128)
    marks = workloads.distinct_marks(n, 5, seed=n)
    out = {}
    for forced in ("0", "1"):
        monkeypatch.setenv("GROVER_FUSED_TEMPORAL", forced)
        g = G.Grover(n, dtype, marks=marks, form="fused")
        state = (1 << n) * g.query(G.grover.Q_ELEM_BYTES)
        assert g.query(G.grover.Q_FUSED_TEMPORAL) == (state if forced == "1" else 0)
        g.write_state(psi0).iterate(3).iterate(4)
        out[forced] = g.read_state()
        g.close()
    monkeypatch.delenv("GROVER_FUSED_TEMPORAL", raising=False)
    assert np.array_equal(out["0"].view(np.uint64), out["1"].view(np.uint64)), (n, dtype)
    if dtype != "cbf16":
        assert_close(out["0"], orc.iterate(as_c128(psi0), marks, 7), dtype, f"n={n} {dtype} nontemporal")


# ----------------------------------------------------------------------------------- hash oracle
@pytest.mark.parametrize("form", ["held", "fused"])
def test_hash_predicate_marks_match_oracle(G, orc, form):
    n, bits = 20, 17
    seed = None
    for s in range(5000, 5200):
        _, c = orc.hash_marks(n, s, bits, cap=0)
        if c == 8:
            seed = s
            break
    assert seed is not None
    want, _ = orc.hash_marks(n, seed, bits, cap=64)
    g = G.Grover(n, "c64", hash_seed=seed, hash_bits=bits, m=8, form=form)
    assert np.array_equal(g.marked(), want)
    k = orc.optimal_iterations(n, 8)
    g.iterate(k)
    assert_close(g.read_state(), orc.search(n, want, k), "c64", "hash search")
    g.close()
    with pytest.raises(G.GroverError) as e:
        G.Grover(n, "c64", hash_seed=seed, hash_bits=bits, m=7)
    assert e.value.status == -6


# ------------------------------------------------------------------------------------- gate path
@pytest.mark.parametrize("n,dtype", [(1, "c128"), (3, "f64"), (6, "c128"), (9, "c64"), (11, "c128")])
def test_gate_level_path_matches_oracle(G, orc, n, dtype):
    marks = workloads.distinct_marks(n, 2 if n > 1 else 1, seed=n)
    psi0 = start_state(n, dtype, seed=60 + n)
    g = G.Grover(n, dtype, marks=marks).write_state(psi0)
    g.hadamard_all()
    want = orc.hadamard_all(as_c128(psi0))
    assert_close(g.read_state(), want, dtype, "H^n")
    g.write_state(psi0).gate_iterate(3)
    want = orc.gate_iterate(as_c128(psi0), marks, 3)
    assert_close(g.read_state(), want, dtype, "gate iterate")
    # the two paths agree (the paper's equivalence), here on the GPU
    g2 = G.Grover(n, dtype, marks=marks).write_state(psi0).iterate(3)
    assert_close(g2.read_state(), want, dtype, "gate vs proposed")
    g.close()
    g2.close()


@pytest.mark.parametrize("dtype", ["c128", "c64", "f64"])
def test_two_pass_form_where_its_grid_wraps(G, orc, dtype):
    """The plain form caps its grid at 2048 x 256 threads, so at n = 22 every thread of its sum and update
    kernels visits 2 (f64, c64) or 8 (c128) vectors: element-wise parity there, several iterations."""
    n = 22
    marks = workloads.distinct_marks(n, 5, seed=2222)
    psi0 = start_state(n, dtype, seed=2200)
    g = G.Grover(n, dtype, marks=marks, form="two_pass").write_state(psi0)
    want = as_c128(psi0)
    for k in (1, 3):
        g.iterate(k)
        orc.iterate(want, marks, k)
        assert_close(g.read_state(), want, dtype, f"two_pass n={n} k={k}")
    g.close()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_single_qubit_gate_passes_where_their_grid_wraps(G, orc, dtype):
    """The single-qubit passes of the gate-level path cap their grid at 4096 x 256 threads: at n = 23 each
    thread visits 4 butterfly pairs per pass.  H^n and one conventional iteration, element by element."""
    n = 23
    marks = workloads.distinct_marks(n, 2, seed=2323)
    psi0 = start_state(n, dtype, seed=2300)
    g = G.Grover(n, dtype, marks=marks, form="fused").write_state(psi0)
    g.hadamard_all()
    assert_close(g.read_state(), orc.hadamard_all(as_c128(psi0)), dtype, "H^n")
    g.write_state(psi0).gate_iterate(1)
    assert_close(g.read_state(), orc.gate_iterate(as_c128(psi0), marks, 1), dtype, "gate iterate")
    g.close()


# ----------------------------------------------------------------------------------- measurement
@pytest.mark.parametrize("n,dtype", [(1, "c64"), (4, "f64"), (12, "c64"), (13, "c128"), (18, "c64")])
def test_sampler_bit_exact_on_identical_input(G, orc, n, dtype):
    psi0 = start_state(n, dtype, seed=5 + n)
    if n > 2:
        psi0[3] = 0  # a zero-probability index
    g = G.Grover(n, dtype, marks=[]).write_state(psi0)
    u = workloads.uniforms_u53(31 + n, 50_000)
    u[:3] = [0, (1 << 53) - 1, 1 << 52]
    host = g.sample(u.size, u53=u)
    want = orc.sample(as_c128(psi0), u)
    assert np.array_equal(host, want)
    dev = g.sample(u.size, u53=u, device_out=True).cpu().numpy().astype(np.uint64)
    assert np.array_equal(dev, want)
    import torch

    ut = torch.from_numpy(u.astype(np.int64)).cuda()
    assert np.array_equal(g.sample(u.size, u53=ut), want)
    # device-generated uniforms: SplitMix64_j(seed) >> 11, the oracle's own generator
    assert np.array_equal(g.sample(20_000, seed=99), orc.sample(as_c128(psi0), orc.uniforms_u53(99, 20_000)))
    if n > 2:
        assert not np.any(host == 3)
    assert g.sample(0, seed=1).size == 0
    g.close()


def test_sampler_zero_state_is_an_error(G):
    g = G.Grover(5, "c64", marks=[]).write_state(np.zeros(32, dtype=np.complex64))
    with pytest.raises(G.GroverError):
        g.sample(10, seed=1)
    g.write_state(np.ones(32, dtype=np.complex64) / np.sqrt(32))
    assert g.sample(10, seed=1).size == 10  # the error state was cleared
    g.close()


@pytest.mark.parametrize("dtype", ["f64", "c64", "c128"])
def test_norm_matches_oracle(G, orc, dtype):
    psi0 = start_state(16, dtype, seed=4)
    g = G.Grover(16, dtype, marks=[]).write_state(psi0)
    assert abs(g.norm() - orc.norm(as_c128(psi0))) < 1e-14
    g.reset()
    assert abs(g.norm() - 1.0) < (1e-14 if dtype != "c64" else 1e-6)
    g.close()


# ------------------------------------------------------------------------------ failure handling
def test_cooperative_grid_too_large_is_reported(G, monkeypatch):
    monkeypatch.setenv("GROVER_FUSED_GRID", str(1 << 24))
    with pytest.raises(G.GroverError) as e:
        G.Grover(16, "c64", marks=[1], form="fused")
    assert e.value.status == -4


def test_barrier_timeout_is_reported_and_recovers(G, orc, monkeypatch):
    """A zero wait limit makes the first grid barrier give up: every workgroup exits, grover_sync reports
    the timeout, and the context works again afterwards."""
    monkeypatch.setenv("GROVER_BARRIER_TIMEOUT_MS", "0")
    monkeypatch.setenv("GROVER_FUSED_GRID", "64")
    g = G.Grover(16, "c64", marks=[5], form="fused")
    g.iterate(3)
    with pytest.raises(G.GroverError) as e:
        g.sync()
    assert e.value.status == -7
    g.close()
    monkeypatch.delenv("GROVER_BARRIER_TIMEOUT_MS")
    g = G.Grover(16, "c64", marks=[5], form="fused").iterate(3)
    g.sync()
    assert_close(g.read_state(), orc.search(16, [5], 3), "c64")
    g.close()


def test_held_form_selection(G):
    """AUTO takes the held form for complex64 states with binary64 sums between the one-workgroup form
    and the largest state that fits on chip; other storage types and larger states keep the fused form."""
    g = G.Grover(18, "c64", marks=[5])
    assert g.query(0) == G.grover.GROVER_FORM_HELD
    assert g.query(1) == 64  # 2^17 vectors spread over 64 workgroups: 2 per thread
    g.close()
    # about 2 vectors per thread up to 64 workgroups, at most 8 per thread up to 128, then 16 (8 in LDS)
    for n, team in [(15, 8), (16, 16), (20, 64), (21, 128), (22, 128), (23, 256)]:
        g = G.Grover(n, "c64", marks=[5])
        assert g.query(0) == G.grover.GROVER_FORM_HELD and g.query(1) == team, n
        g.close()
    assert G.Grover(18, "c128", marks=[5]).query(0) == G.grover.GROVER_FORM_FUSED
    assert G.Grover(18, "c64", marks=[5], accum="f32").query(0) == G.grover.GROVER_FORM_FUSED
    assert G.Grover(12, "c64", marks=[5]).query(0) == G.grover.GROVER_FORM_RESIDENT
    assert G.Grover(12, "c128", marks=[5]).query(0) == G.grover.GROVER_FORM_RESIDENT
    h = G.Grover(14, "c64", marks=[5], form="held")
    assert h.query(1) == 4  # 2^13 vectors, 2 per thread
    h.close()
    with pytest.raises(G.GroverError) as e:
        G.Grover(16, "c128", marks=[5], form="held")
    assert e.value.status == G.grover.GROVER_E_UNSUPPORTED
    cu = G.Grover(10, "c64", marks=[5], form="held")
    assert cu.query(1) == 1
    cu.close()


@pytest.mark.parametrize("n", [18, 22])  # a team of 64 (one slot per lane) and of 128 (slots waited together)
def test_held_barrier_timeout_is_reported_and_recovers(G, orc, monkeypatch, n):
    monkeypatch.setenv("GROVER_BARRIER_TIMEOUT_MS", "0")
    g = G.Grover(n, "c64", marks=[5], form="held")
    g.iterate(3)
    with pytest.raises(G.GroverError) as e:
        g.sync()
    assert e.value.status == -7
    g.close()
    monkeypatch.delenv("GROVER_BARRIER_TIMEOUT_MS")
    g = G.Grover(n, "c64", marks=[5], form="held").iterate(3)
    g.sync()
    assert_close(g.read_state(), orc.search(n, [5], 3), "c64")
    g.close()


def test_caller_buffer_is_adopted_and_size_checked(G):
    import torch

    buf = torch.zeros(1 << 12, dtype=torch.complex64, device="cuda")
    g = G.Grover(12, "c64", marks=[7], state=buf)
    assert G.grover_state_device(g.ctx)[0] == buf.data_ptr()
    g.iterate(4)
    torch.cuda.synchronize()
    assert np.array_equal(buf.cpu().numpy(), g.read_state())
    g.close()
    with pytest.raises(ValueError):
        G.Grover(12, "c64", marks=[7], state=torch.zeros(100, dtype=torch.complex64, device="cuda"))
