"""GPU parity of the reduced-precision forms: amplitudes stored as complex128, complex64 or complex bfloat16,
the sum behind the mean accumulated in binary64, binary32 or Kahan-compensated binary32 (fused form).

Tolerance, derived from the arithmetic: in one iteration the stored amplitudes are rounded (error vector of
2-norm <= sqrt(2) u_s for a unit state, u_s the storage's unit roundoff) and the sum S carries an error
<= gamma * sum_i |c_i| <= gamma sqrt(N), which the update spreads over all N amplitudes as 2 dS / N each
(2-norm <= 2 gamma); gamma = (additions on the longest path of the reduction) * u_a.  The iteration is
unitary, so these per-iteration errors add without growth in the 2-norm, which bounds the largest
amplitude error: k (sqrt(2) u_s + 2 gamma), used here with a factor 2 of margin.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

SETTINGS = [(s, a) for s in ("c128", "c64", "cbf16") for a in ("f64", "f32", "f32_kahan")]
U_STORE = {"c128": 2.0 ** -53, "c64": 2.0 ** -24, "cbf16": 2.0 ** -8}
U_ACC = {"f64": 2.0 ** -53, "f32": 2.0 ** -24, "f32_kahan": 2.0 ** -24}
EPV = {"c128": 1, "c64": 2, "cbf16": 4}
BITS = {"c128": 53, "c64": 24, "cbf16": 8}


@pytest.fixture(scope="module")
def G():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_04635_amd as pkg

    pkg.load()
    return pkg


def rounded_start(n: int, storage: str, seed: int) -> np.ndarray:
    """A random unit state already rounded to the storage type, as complex128."""
    from paper_2005_04635_amd.grover import bf16_pairs_to_complex, complex_to_bf16_pairs

    psi = workloads.random_state(n, seed)
    if storage == "c64":
        return psi.astype(np.complex64).astype(np.complex128)
    if storage == "cbf16":
        return bf16_pairs_to_complex(complex_to_bf16_pairs(psi))
    return psi


def error_bound(n: int, k: int, storage: str, accum: str, grid: int) -> float:
    N = 1 << n
    per_thread = math.ceil(N / EPV[storage] / (1024 * grid)) * EPV[storage]
    seq = 2 if accum == "f32_kahan" else per_thread
    depth = seq + 16 + math.ceil(math.log2(max(grid, 1))) + 1
    return 2.0 * k * (math.sqrt(2.0) * U_STORE[storage] + 2.0 * depth * U_ACC[accum]) + 1e-15


@pytest.mark.parametrize("storage,accum", SETTINGS)
@pytest.mark.parametrize("n", [11, 16])
def test_precision_setting_matches_oracle(G, orc, storage, accum, n):
    marks = workloads.distinct_marks(n, 3, seed=n + 7)
    psi0 = rounded_start(n, storage, seed=40 + n)
    g = G.Grover(n, storage, marks=marks, accum=accum, form="fused")
    assert g.query(0) == 1
    g.write_state(psi0)
    assert np.array_equal(g.read_state().astype(np.complex128), psi0)  # exact round trip
    want = psi0.copy()
    done = 0
    for k in (1, 4):
        g.iterate(k)
        orc.iterate(want, marks, k)
        done += k
        err = float(np.max(np.abs(g.read_state().astype(np.complex128) - want)))
        assert err <= error_bound(n, done, storage, accum, g.query(1)), (storage, accum, n, done, err)
    g.close()


@pytest.mark.parametrize("storage,accum", SETTINGS)
def test_precision_setting_two_class_and_composition(G, storage, accum):
    """From the uniform state every marked amplitude stays bit-identical to every other, and so do the
    unmarked ones, in any precision; calls compose bit for bit."""
    n = 16
    marks = workloads.distinct_marks(n, 4, seed=3)
    ga = G.Grover(n, storage, marks=marks, accum=accum, form="fused")
    gb = G.Grover(n, storage, marks=marks, accum=accum, form="fused")
    ga.iterate(7).iterate(13)
    gb.iterate(20)
    sa, sb = ga.read_state(), gb.read_state()
    assert np.array_equal(np.asarray(sa).view(np.uint8), np.asarray(sb).view(np.uint8))
    mask = np.zeros(1 << n, dtype=bool)
    mask[marks.astype(np.int64)] = True
    assert np.all(sa[mask] == sa[mask][0]) and np.all(sa[~mask] == sa[~mask][0])
    ga.close()
    gb.close()


@pytest.mark.parametrize("storage", ["c64", "cbf16"])
def test_stored_two_class_prediction(G, orc, storage):
    """With binary64 sums, the GPU's two amplitude values track the oracle's two-class iteration with
    storage rounding (the sums differ only in summation order): within two storage ulps."""
    n, m = 20, 2
    marks = workloads.distinct_marks(n, m, seed=20)
    k = orc.optimal_iterations(n, m)
    g = G.Grover(n, storage, marks=marks, accum="f64", form="fused")
    g.iterate(k)
    got = g.read_state().astype(np.complex128)
    mask = np.zeros(1 << n, dtype=bool)
    mask[marks.astype(np.int64)] = True
    a, b = orc.two_class_stored(n, m, k, BITS[storage])
    ulp = 2.0 ** (1 - BITS[storage])
    assert abs(got[mask][0].real - a) <= 2 * ulp * abs(a)
    assert abs(got[~mask][0].real - b) <= 2 * ulp * abs(b) + 1e-300
    g.close()


@pytest.mark.parametrize("accum", ["f64", "f32_kahan"])
def test_bf16_sampler_and_norm(G, orc, accum):
    n = 14
    psi0 = rounded_start(n, "cbf16", seed=9)
    g = G.Grover(n, "cbf16", marks=[3], accum=accum).write_state(psi0)
    u = workloads.uniforms_u53(123, 20000)
    assert np.array_equal(g.sample(u.size, u53=u), orc.sample(psi0, u))
    assert abs(g.norm() - orc.norm(psi0)) < 1e-14
    g.close()


@pytest.mark.parametrize("n", [2, 3])
def test_bf16_smallest_states(G, orc, n):
    """One and two 16-byte vectors of complex bfloat16 (N = 4, 8): the fill, the iteration, the norm and the
    sampler against the oracle.  Every sum here is exact in binary64 (at most 8 values of 8 significant bits),
    so the device's state equals the oracle's stored two-class iteration bit for bit, every iteration."""
    g = G.Grover(n, "cbf16", marks=[1], form="fused")
    mask = np.zeros(1 << n, dtype=bool)
    mask[1] = True
    u = workloads.uniforms_u53(77 + n, 4000)
    for k in range(0, 5):
        got = g.read_state().astype(np.complex128)
        a, b = orc.two_class_stored(n, 1, k, BITS["cbf16"])
        assert np.all(got[mask] == a) and np.all(got[~mask] == b), (n, k, got, a, b)
        assert abs(g.norm() - orc.norm(got)) < 1e-15
        assert np.array_equal(g.sample(u.size, u53=u), orc.sample(got, u)), (n, k)
        g.iterate(1)
    g.close()


def test_bf16_one_qubit_is_unsupported(G):
    with pytest.raises(G.GroverError) as e:
        G.Grover(1, "cbf16", marks=[1], form="fused")
    assert e.value.status == -5


def test_bf16_gate_path_is_unsupported(G):
    g = G.Grover(8, "cbf16", marks=[1])
    with pytest.raises(G.GroverError) as e:
        g.gate_iterate(1)
    assert e.value.status == -5
    g.close()
