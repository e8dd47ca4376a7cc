"""GPU parity of the binary32 update (complex64 storage, binary64 sums): c' = fl32(fl32(2S/N) - s c), in the
one-workgroup, held, fused and batched forms, against the oracle's stored iteration with binary32 storage and
a binary32 update (orc_grover_iterate_stored / orc_two_class_stored_update, p_store = p_update = 24).

Device and oracle then perform the same roundings; they differ only in the order of the binary64 sum's
additions (a tree on the device, pairwise in the oracle), which moves the binary64 value of 2S/N by a few
units of 2^-53 and changes fl32(2S/N) only when it lies that close to a binary32 rounding boundary.  So the
states agree bit for bit almost everywhere, and the bound allows one such event per iteration: four
binary32 ulps of a unit amplitude per iteration.  The binary32 and binary64 updates end only a few ulps apart,
so the test that tells them apart is bitwise: at n = 12 from the uniform state every sum is exact in any
order and the device must reproduce the binary32-update model exactly.
"""
from __future__ import annotations

import numpy as np
import pytest

import workloads
from test_gpu_batch import small_batch

pytestmark = pytest.mark.gpu

ULP = 2.0 ** -24


@pytest.fixture(scope="module")
def G():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_04635_amd as pkg

    pkg.load()
    return pkg


FORM_CODE = {"fused": 1, "resident": 2, "held": 4}
CASES = [("resident", 1), ("resident", 9), ("resident", 12), ("resident", 14), ("held", 15), ("held", 18),
         ("held", 21), ("held", 22), ("fused", 3), ("fused", 16), ("fused", 20), ("fused", 24)]


@pytest.mark.parametrize("form,n", CASES)
def test_binary32_update_matches_the_stored_oracle(G, orc, form, n):
    """Random complex64 start state and several marked-set sizes: element by element against the oracle's
    stored iteration; nearly every amplitude equal bit for bit."""
    N = 1 << n
    for m in sorted({0, 1, min(3, N), max(1, N // 5)}):
        marks = workloads.distinct_marks(n, m, seed=17 * n + m)
        psi0 = workloads.random_state(n, seed=700 + n + m).astype(np.complex64)
        g = G.Grover(n, "c64", marks=marks, form=form, update="f32").write_state(psi0)
        assert g.query(0) == FORM_CODE[form]
        want = psi0.astype(np.complex128)
        done = 0
        for k in (1, 6):
            g.iterate(k)
            orc.iterate_stored(want, marks, k, 24, 24)
            done += k
            got = g.read_state().astype(np.complex128)
            err = float(np.max(np.abs(got - want)))
            same = float(np.mean(got == want))
            assert err <= 4 * ULP * done, (form, n, m, done, err)
            assert same >= 0.99, (form, n, m, done, same)
        g.close()


@pytest.mark.parametrize("form", ["resident", "held", "fused"])
def test_binary32_update_bitwise_from_uniform(G, orc, form):
    """n = 12 from the uniform state: every stored value is a binary32 number and the state has two values,
    so every partial sum of the binary64 sum, in the device's order as in the oracle's, is an integer
    combination of the two that fits 53 bits: all sums are exact, and the device must equal the oracle's
    stored two-class iteration with the binary32 update bit for bit after every one of the 35 iterations of
    the search.  The binary64 update ends elsewhere, so this tells the two updates apart."""
    n, m = 12, 2
    N = 1 << n
    marks = workloads.distinct_marks(n, m, seed=12)
    k_opt = orc.optimal_iterations(n, m)
    g = G.Grover(n, "c64", marks=marks, form=form, update="f32")
    assert g.query(0) == FORM_CODE[form]
    mask = np.zeros(N, dtype=bool)
    mask[marks.astype(np.int64)] = True
    for k in range(1, k_opt + 1):
        g.iterate(1)
        got = g.read_state()
        a, b = orc.two_class_stored_update(n, m, k, 24, 24)
        assert np.all(got[mask] == np.complex64(a)) and np.all(got[~mask] == np.complex64(b)), (form, k)
    a64, b64 = orc.two_class_stored_update(n, m, k_opt, 24, 53)
    assert (np.complex64(a64), np.complex64(b64)) != (got[mask][0], got[~mask][0])
    g.close()


@pytest.mark.parametrize("form,n,m", [("held", 18, 3), ("held", 20, 1), ("fused", 20, 4)])
def test_binary32_update_search_from_uniform(G, orc, form, n, m):
    """A whole search from the uniform state at sizes where the sums may round: each class bitwise constant,
    its value within a few binary32 ulps of the oracle's stored two-class iteration with the binary32
    update (usually equal: the sums differ only in their order)."""
    N = 1 << n
    marks = workloads.distinct_marks(n, m, seed=n + 5 * m)
    k = orc.optimal_iterations(n, m)
    g = G.Grover(n, "c64", marks=marks, form=form, update="f32")
    g.iterate(k)
    got = g.read_state()
    mask = np.zeros(N, dtype=bool)
    mask[marks.astype(np.int64)] = True
    gm, gu = got[mask], got[~mask]
    assert np.all(gm.view(np.uint64) == gm.view(np.uint64)[0]) and np.all(gu.view(np.uint64) == gu.view(np.uint64)[0])
    a32, b32 = orc.two_class_stored_update(n, m, k, 24, 24)
    da, db = abs(complex(gm[0]) - a32), abs(complex(gu[0]) - b32)
    print(f"{form} n={n}: |device - oracle| marked {da:.3g}, unmarked {db:.3g}", flush=True)
    assert da <= 4 * ULP * abs(a32) and db <= 4 * ULP * abs(b32) + 1e-300, (da, db)
    g.close()


@pytest.mark.parametrize("form,n", [("resident", 11), ("held", 17), ("fused", 19)])
def test_binary32_update_composes_bitwise(G, form, n):
    marks = workloads.distinct_marks(n, 3, seed=n)
    ga = G.Grover(n, "c64", marks=marks, form=form, update="f32")
    gb = G.Grover(n, "c64", marks=marks, form=form, update="f32")
    ga.iterate(7).iterate(13)
    gb.iterate(20)
    assert np.array_equal(ga.read_state().view(np.uint64), gb.read_state().view(np.uint64))
    ga.close()
    gb.close()


@pytest.mark.parametrize("split,team,resident", [(19, 2, 16), (0, 1, 0), (12, 2, 0), (10, 2, 2)])
def test_batch_binary32_update(G, orc, split, team, resident):
    """Every instance of the small batch with the binary32 update, held on chip or streamed: each class
    bitwise constant, its value the stored two-class iteration with the binary32 update."""
    rows = small_batch()
    ns, ms, mks = [r[0] for r in rows], [len(r[1]) for r in rows], [r[1] for r in rows]
    ks = [orc.optimal_iterations(n, len(mk)) if k is None else k for n, mk, k in rows]
    b = G.GroverBatch(ns, ms, mks, iterations=ks, update="f32")
    b.set_tiling(split, team, resident)
    b.run()
    b.sync()
    for i, (n, mk, k) in enumerate(zip(ns, mks, ks)):
        got = b.read_state(i)
        mask = np.zeros(1 << n, dtype=bool)
        mask[np.asarray(mk, dtype=np.int64)] = True
        a, u = orc.two_class_stored_update(n, len(mk), k, 24, 24)
        for sel, want in ((mask, a), (~mask, u)):
            part = got[sel]
            if part.size:
                assert np.all(part.view(np.uint64) == part.view(np.uint64)[0]), i
                assert abs(complex(part[0]) - want) <= 4 * ULP * max(k, 1), (i, n, len(mk), k)
    b.close()
