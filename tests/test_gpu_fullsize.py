"""Full-size parity: the n = 28 single-large-instance workload in the launch configuration bench.py times
(fused persistent form, default grid, complex64 storage, hash predicate with M = 8, 4549 iterations,
10^6 shots), checked against the oracle where it can compute the outputs (the first iterations element by
element, the two-class value of every amplitude at the end) and through properties that hold at any size.
"""
from __future__ import annotations

import os

import numpy as np
import pytest

import workloads
from conftest import GOLDEN

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_04635_amd as pkg

    pkg.load()
    return pkg


def max_abs_err_chunked(got: np.ndarray, want: np.ndarray, chunk: int = 1 << 24) -> float:
    err = 0.0
    for s in range(0, got.size, chunk):
        d = np.abs(got[s:s + chunk].astype(np.complex128) - want[s:s + chunk])
        err = max(err, float(d.max()))
    return err


def test_n28_hash_workload(G, orc):
    w = workloads.HASH_N28
    N = 1 << w.n
    g = G.Grover(w.n, w.dtype, hash_seed=w.hash_seed, hash_bits=w.hash_bits, m=w.m, form="fused")
    assert g.query(0) == 1
    marks = g.marked()
    with open(os.path.join(GOLDEN, "hash_marks_n28.txt")) as f:
        golden = [int(x) for x in f if x.strip() and not x.startswith("#")]
    assert marks.tolist() == golden  # bit-exact device predicate + compaction

    # first 8 iterations, every amplitude against the full binary64 oracle
    g.iterate(8)
    want = orc.search(w.n, marks, 8)
    err8 = max_abs_err_chunked(g.read_state(), want)
    assert err8 <= 1e-5, err8
    del want

    # the rest of the optimal run (composition is bitwise, so this equals one 4549-iteration call)
    g.iterate(w.iterations - 8)
    got = g.read_state()
    mask = np.zeros(N, dtype=bool)
    mask[marks.astype(np.int64)] = True
    a_gpu, b_gpu = got[int(marks[0])], got[int(np.argmin(mask))]
    assert np.all(got[mask] == a_gpu)          # every marked amplitude bit-identical
    assert np.all(got[~mask] == b_gpu)         # every unmarked amplitude bit-identical
    assert np.all(got.imag == 0)               # standard phases keep the state real
    a, b = orc.two_class(w.n, w.m, w.iterations)
    assert abs(complex(a_gpu) - a) <= 1e-5 and abs(complex(b_gpu) - b) <= 1e-5
    assert abs(g.norm() - 1.0) < 1e-5

    # measurement: bit-exact against the oracle sampler on the same state
    u = workloads.uniforms_u53(w.shot_seed, w.shots)
    shots = g.sample(w.shots, u53=u)
    psi = got.astype(np.complex128)
    del got
    assert np.array_equal(shots, orc.sample(psi, u))
    # end to end against the oracle's own final state (its two-class values): a shot can only differ where
    # U falls within the CDF difference of the two states, ~2e-5 per marked boundary here
    psi[mask] = a
    psi[~mask] = b
    mism = int(np.sum(shots != orc.sample(psi, u)))
    assert mism <= 64, mism
    assert np.isin(shots, marks).all()
    g.close()


def two_class_shots(g, marks, a: complex, b: complex, seed: int, shots: int = 100000):
    """10^5 measurement shots of a two-class state (every marked amplitude a, every other b) from given
    53-bit uniforms, and the sampler's definition evaluated exactly for that state with integers: p = re^2 +
    im^2 in binary64, q = floor(p 2^62), t = floor(U Q_total / 2^53), index = the smallest i with Q_i > t,
    where Q_i counts the unmarked and marked indices up to i."""
    def q_of(z: complex) -> int:
        return int((z.real * z.real + z.imag * z.imag) * 2.0 ** 62)

    qa, qb = q_of(a), q_of(b)
    ms = sorted(int(x) for x in marks)
    total = (g.N - len(ms)) * qb + len(ms) * qa

    def index_of(t: int) -> int:
        acc, p = 0, 0
        for k in ms:
            if qb > 0 and t < acc + (k - p) * qb:
                return p + (t - acc) // qb
            acc += (k - p) * qb
            if t < acc + qa:
                return k
            acc += qa
            p = k + 1
        return p + (t - acc) // qb

    u = workloads.uniforms_u53(seed, shots)
    got = g.sample(shots, u53=u)
    want = np.array([index_of((int(x) * total) >> 53) for x in u], dtype=np.uint64)
    return got, want


def test_large_index_range(G, orc):
    """n = 31 (2^31 complex64 amplitudes, 16 GiB): indices past 2^31 and marks at the very end of the
    state; three iterations against the oracle's two-class values, then measurement shots against the
    sampler's definition evaluated exactly."""
    import torch

    n = 31
    N = 1 << n
    marks = np.array([5, (1 << 31) - 2, (1 << 31) - 1], dtype=np.uint64)
    g = G.Grover(n, "c64", marks=marks, form="fused")
    g.iterate(3)
    torch.cuda.synchronize()
    st = g.state
    a, b = orc.two_class(n, marks.size, 3)
    idx = torch.from_numpy(marks.astype(np.int64)).cuda()
    marked_vals = st[idx]
    assert torch.all(marked_vals == marked_vals[0]).item()
    assert abs(complex(marked_vals[0].item()) - a) <= 1e-5
    unmarked = st[6:N - 2]
    assert torch.all(unmarked == st[0]).item() and torch.all(st[:5] == st[0]).item()
    assert abs(complex(st[0].item()) - b) <= 1e-5
    assert abs(g.norm() - 1.0) < 1e-5

    # measurement over the whole index range (a 16 GiB integer CDF, indices past 2^31)
    shots, want = two_class_shots(g, marks, complex(marked_vals[0].item()), complex(st[0].item()), seed=31)
    assert np.array_equal(shots, want), int(np.sum(shots != want))
    assert shots.max() > (1 << 30)  # the shots reach the upper half of the index range
    g.close()


@pytest.mark.parametrize("n,dtype", [(34, "c64"), (33, "c128")])
def test_maximum_size(G, orc, n, dtype):
    """The largest states the library accepts: n = 34 (2^34 complex64 amplitudes) and complex128 at n = 33,
    128 GiB each on one GPU, byte addresses up to 2^37.  Marks at both ends of the index range; three fused
    iterations from the uniform state against the oracle's two-class values, every amplitude checked on the
    device (each class bitwise constant); at n = 33 also measurement shots against the sampler's
    definition evaluated exactly."""
    import torch

    if torch.cuda.get_device_properties(0).total_memory < (150 << 30):
        pytest.skip("needs a device with at least 150 GiB (the 128 GiB state and a comparison mask)")
    N = 1 << n
    marks = np.array([0, 5, N - 2, N - 1], dtype=np.uint64)
    g = G.Grover(n, dtype, marks=marks, form="fused")
    assert g.query(0) == 1
    g.iterate(3)
    torch.cuda.synchronize()
    st = g.state
    a, b = orc.two_class(n, marks.size, 3)
    tol = 1e-5 if dtype == "c64" else 1e-12
    idx = torch.from_numpy(marks.astype(np.int64)).cuda()
    marked_vals = st[idx]
    assert torch.all(marked_vals == marked_vals[0]).item()
    assert abs(complex(marked_vals[0].item()) - a) <= tol
    ref = st[1]
    assert abs(complex(ref.item()) - b) <= tol
    assert torch.all(st[1:5] == ref).item() and torch.all(st[6:N - 2] == ref).item()
    assert abs(g.norm() - 1.0) < 1e-5
    if dtype == "c128":  # its 64 GiB integer CDF fits beside the state (complex64 at n = 34 would need 128 GiB)
        shots, want = two_class_shots(g, marks, complex(marked_vals[0].item()), complex(ref.item()), seed=n)
        assert np.array_equal(shots, want), int(np.sum(shots != want))
        assert shots.max() > (1 << 32)  # indices past 2^32
    g.close()
    del g, st, marked_vals, ref
    torch.cuda.empty_cache()  # the 128 GiB state goes back to the device before the next case


@pytest.mark.parametrize("storage,accum", [(s, a) for s in ("c128", "c64", "cbf16")
                                           for a in ("f64", "f32", "f32_kahan")])
def test_n26_precision_sweep(G, orc, storage, accum):
    """The precision workload (n = 26, M = 4, 3216 iterations) in every storage x accumulator setting:
    the two-class structure holds exactly; binary64-accumulated settings match the oracle's two-class
    values (complex128: 1e-12, complex64: 1e-5) and, for bfloat16, its stored-precision iteration; the
    binary32-accumulated ones stay within the bound derived from the arithmetic (test_gpu_precision.py)
    where that bound is informative."""
    from test_gpu_precision import BITS, error_bound

    w = workloads.PRECISION_N26
    marks = np.array(w.marks, dtype=np.uint64)
    g = G.Grover(w.n, storage, marks=marks, accum=accum, form="fused")
    g.iterate(w.iterations)
    got = g.read_state()
    mask = np.zeros(1 << w.n, dtype=bool)
    mask[marks.astype(np.int64)] = True
    a_gpu, b_gpu = complex(got[int(marks[0])]), complex(got[int(np.argmin(mask))])
    assert np.all(got[mask] == got[int(marks[0])]) and np.all(got[~mask] == got[int(np.argmin(mask))])
    assert a_gpu.imag == 0 and b_gpu.imag == 0
    a, b = orc.two_class(w.n, w.m, w.iterations)
    err = max(abs(a_gpu - a), abs(b_gpu - b))
    if accum == "f64" and storage == "c128":
        assert err <= 1e-12
    elif accum == "f64" and storage == "c64":
        assert err <= 1e-5
    elif accum == "f64":
        sa, sb = orc.two_class_stored(w.n, w.m, w.iterations, BITS[storage])
        ulp = 2.0 ** (1 - BITS[storage])
        assert abs(a_gpu.real - sa) <= 2 * ulp * abs(sa) and abs(b_gpu.real - sb) <= 2 * ulp * abs(sb)
    bound = error_bound(w.n, w.iterations, storage, accum, g.query(1))
    if bound < 1.0:
        assert err <= bound, (err, bound)
    g.close()


def test_batch4096_workload(G, orc):
    """The 4096-instance batch at full size, in the configuration the benchmark times (the autotuned tiling,
    replayed from a captured graph): every amplitude of every instance is checked — each class (marked,
    unmarked) bitwise constant, and its value within the complex64 bound of the oracle's two-class result."""
    import torch

    from test_gpu_precision import error_bound

    w = workloads.BATCH_4096
    n, m, marks = w.instances()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = G.GroverBatch(n, m, marks)
        split, team, resident, ms = b.tune()
        b.capture()
        b.run()
        b.sync()
        print(f"tiling split={split} team={team} resident={resident} tuned {ms:.1f} ms", flush=True)
        worst = 0.0
        for i in range(w.count):
            ni, mi = int(n[i]), int(m[i])
            k = orc.optimal_iterations(ni, mi)
            a, u = orc.two_class(ni, mi, k)  # marked, unmarked amplitude (binary64)
            got = b.read_state(i)
            mask = np.zeros(1 << ni, dtype=bool)
            mask[marks[i].astype(np.int64)] = True
            gm, gu = got[mask], got[~mask]
            assert np.all(gm.view(np.uint64) == gm.view(np.uint64)[0]), i
            assert np.all(gu.view(np.uint64) == gu.view(np.uint64)[0]), i
            err = max(abs(complex(gm[0]) - a), abs(complex(gu[0]) - u))
            worst = max(worst, err / error_bound(ni, k, "c64", "f64", 1))
            assert err <= error_bound(ni, k, "c64", "f64", 1), (i, ni, mi, k, err)
        print(f"worst error / bound = {worst:.3g}", flush=True)
        b.close()


def test_phase_n20_workload(G, orc):
    """The differentiable workload at full size (n = 20, M = 3, K = 64, 64 schedules, phases N(pi, 0.1)), in
    the configuration the benchmark times: losses of 8 schedules and the final states' two-class structure
    against the oracle, gradients of 2 schedules against the oracle's stored-state adjoint."""
    import torch

    from test_gpu_phase import forward_bound, grad_bound, loss_bound

    w = workloads.PHASE_N20
    marks = w.marks()
    phi, theta = w.schedules()
    eng = G.GroverPhase(w.n, marks, w.K, batch=w.batch)
    every = eng.query(G.grover.PQ_EVERY)
    assert every == 8 and eng.query(G.grover.PQ_CHECKPOINTS) == 7
    ph = torch.tensor(phi, dtype=torch.float64, device="cuda")
    th = torch.tensor(theta, dtype=torch.float64, device="cuda")
    loss = eng.forward(ph, th)
    eng.sync()
    loss = loss.cpu().numpy()
    mask = np.zeros(1 << w.n, dtype=bool)
    mask[marks.astype(np.int64)] = True
    for b in range(0, w.batch, 9):
        got = eng.read_state(b)
        gm, gu = got[mask], got[~mask]
        assert np.all(gm.view(np.uint64) == gm.view(np.uint64)[0]) and np.all(gu.view(np.uint64) == gu.view(np.uint64)[0])
        want = orc.phase_search(w.n, marks, phi[b], theta[b])
        assert np.max(np.abs(got.astype(np.complex128) - want)) <= forward_bound(w.K), b
        assert abs(loss[b] - orc.phase_loss(want, marks)) <= loss_bound(w.K), b
    g = np.linspace(1.0, 2.0, w.batch)
    dphi, dtheta = eng.backward(torch.tensor(g, dtype=torch.float64, device="cuda"))
    eng.sync()
    dphi, dtheta = dphi.cpu().numpy(), dtheta.cpu().numpy()
    for b in (0, w.batch - 1):
        wphi, wtheta = orc.phase_grad_adjoint(w.n, marks, phi[b], theta[b])
        tol = grad_bound(w.K, every, g[b])
        err = max(np.max(np.abs(dphi[b] - g[b] * wphi)), np.max(np.abs(dtheta[b] - g[b] * wtheta)))
        print(f"schedule {b}: max gradient error {err:.3g} (bound {tol:.3g}), |grad| max "
              f"{max(np.max(np.abs(wphi)), np.max(np.abs(wtheta))):.3g}", flush=True)
        assert err <= tol, b
    eng.close()


def test_n28_blocked_gate_iterations(G, orc):
    """The blocked Walsh-Hadamard gate path at n = 28 (3 passes per H^n): three conventional iterations of
    the hash workload from the uniform state against the oracle's two-class values."""
    w = workloads.HASH_N28
    g = G.Grover(w.n, w.dtype, hash_seed=w.hash_seed, hash_bits=w.hash_bits, m=w.m, form="fused")
    marks = g.marked()
    g.reset().gate_iterate_blocked(3)
    got = g.read_state()
    mask = np.zeros(1 << w.n, dtype=bool)
    mask[marks.astype(np.int64)] = True
    a, b = orc.two_class(w.n, w.m, 3)
    assert np.max(np.abs(got[mask].astype(np.complex128) - a)) <= 1e-5
    un = got[~mask]
    for s in range(0, un.size, 1 << 24):
        assert np.max(np.abs(un[s:s + (1 << 24)].astype(np.complex128) - b)) <= 1e-5
    g.close()


def two_class_check(got: np.ndarray, mask: np.ndarray, a: float, b: float, tol: float) -> None:
    """Every marked amplitude bitwise equal to every other, likewise every unmarked one, and both values
    within tol of the oracle's two-class values (a, b); chunked so that the 2 and 4 GiB states stay cheap."""
    view = np.uint64 if got.dtype == np.complex64 else np.complex128
    gm = got[mask]
    assert np.all(gm.view(view) == gm.view(view)[0])
    assert abs(complex(gm[0]) - a) <= tol
    idx = np.flatnonzero(~mask[:64])[0]
    ref = got[idx:idx + 1].view(view)[0]
    assert abs(complex(got[idx]) - b) <= tol
    chunk = 1 << 24
    for s in range(0, got.size, chunk):
        part = got[s:s + chunk]
        keep = ~mask[s:s + chunk]
        assert np.all(part[keep].view(view) == ref), s


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_n28_two_pass_form(G, orc, dtype):
    """The plain form as the benchmark times it (n = 28, the hash workload's marks; its sum and update
    kernels stride over 128 or 512 vectors per thread): three iterations from the uniform state against the
    oracle's two-class values, with each class bitwise constant."""
    w = workloads.HASH_N28
    g = G.Grover(w.n, dtype, hash_seed=w.hash_seed, hash_bits=w.hash_bits, m=w.m, form="two_pass")
    marks = g.marked()
    g.iterate(3)
    got = g.read_state()
    mask = np.zeros(1 << w.n, dtype=bool)
    mask[marks.astype(np.int64)] = True
    a, b = orc.two_class(w.n, w.m, 3)
    two_class_check(got, mask, a, b, 1e-5 if dtype == "c64" else 1e-12)
    g.close()


def test_n28_fused_complex128(G, orc):
    """The fused kernel on the largest state of these tests, 2^28 16-byte vectors (complex128, 4 GiB: byte
    addresses beyond 2^32, each tile through its own buffer resource): five iterations from the uniform
    state against the oracle's two-class values, each class bitwise constant, so an amplitude the kernel
    skipped or misplaced would show."""
    w = workloads.HASH_N28
    g = G.Grover(w.n, "c128", hash_seed=w.hash_seed, hash_bits=w.hash_bits, m=w.m, form="fused")
    assert g.query(0) == 1
    marks = g.marked()
    g.iterate(5)
    got = g.read_state()
    mask = np.zeros(1 << w.n, dtype=bool)
    mask[marks.astype(np.int64)] = True
    a, b = orc.two_class(w.n, w.m, 5)
    two_class_check(got, mask, a, b, 1e-12)
    g.close()


def test_n28_single_qubit_gate_iteration(G, orc):
    """The per-qubit gate path at n = 28 (58 passes, each thread over 128 butterfly pairs): one conventional
    iteration from the uniform state against the oracle's two-class values.  Rounding in the passes depends
    on the index's bits, so the classes are checked by value, not bitwise."""
    w = workloads.HASH_N28
    g = G.Grover(w.n, w.dtype, hash_seed=w.hash_seed, hash_bits=w.hash_bits, m=w.m, form="fused")
    marks = g.marked()
    g.reset().gate_iterate(1)
    got = g.read_state()
    mask = np.zeros(1 << w.n, dtype=bool)
    mask[marks.astype(np.int64)] = True
    a, b = orc.two_class(w.n, w.m, 1)
    assert np.max(np.abs(got[mask].astype(np.complex128) - a)) <= 1e-5
    chunk = 1 << 24
    for s in range(0, got.size, chunk):
        part = got[s:s + chunk][~mask[s:s + chunk]]
        assert np.max(np.abs(part.astype(np.complex128) - b)) <= 1e-5, s
    g.close()
