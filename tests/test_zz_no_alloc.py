"""The allocation-free entry point grover_iterate_static against grover_iterate on a fused-form context.

grover_iterate_static runs the same kernel on the same grid with its barrier memory in a fixed device array
of the library, so its states must equal the context's bit for bit.  Two (three) calls in a row, each on a
smaller state than the one before, share that array; then the rejections.
"""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_04635_amd as pkg

    pkg.load()
    return pkg


def _device_marks(marks: np.ndarray):
    import torch

    return torch.from_numpy(np.ascontiguousarray(marks.astype(np.uint64)).view(np.int64)).cuda()


def _static(G, state, n, dtype, marks_t, m, k, status):
    import torch

    lib = G.load()
    rc = lib.grover_iterate_static(torch.cuda.current_stream().cuda_stream or None, state.data_ptr(), n, dtype,
                                   marks_t.data_ptr() if m else None, m, k, status.data_ptr())
    torch.cuda.current_stream().synchronize()
    return rc


def test_static_iterate_equals_context_iterate(G, orc):
    import torch

    # 512 MiB (nontemporal split, 256 workgroups), then 8 MiB (256 workgroups, ordinary accesses), then
    # 32 KiB (one workgroup): each call smaller than the one before
    for n, dtype, m, k in [(26, "c64", 6, 5), (20, "c128", 3, 11), (12, "c64", 2, 9)]:
        print(f"static iterate n={n} {dtype} m={m} k={k}", flush=True)
        code = G.grover.DTYPES[dtype]
        marks = np.sort(workloads.distinct_marks(n, m, seed=n * 31 + m))
        psi0 = workloads.random_state(n, seed=500 + n).astype(np.complex64 if dtype == "c64" else np.complex128)
        g = G.Grover(n, dtype, marks=marks, form="fused").write_state(psi0).iterate(k)
        want = g.read_state()
        g.close()
        state = torch.from_numpy(psi0.copy()).cuda()
        status = torch.full((1,), 7, dtype=torch.int32, device="cuda")
        assert _static(G, state, n, code, _device_marks(marks), m, k, status) == 0
        assert int(status.item()) == 0
        got = state.cpu().numpy()
        assert np.array_equal(got.view(np.uint8), want.view(np.uint8)), (n, dtype)
        if n <= 20:
            ref = psi0.astype(np.complex128)
            orc.iterate(ref, marks, k)
            tol = 1e-5 if dtype == "c64" else 1e-12
            assert float(np.max(np.abs(got.astype(np.complex128) - ref))) <= tol


def test_static_iterate_rejections(G):
    import torch

    lib = G.load()
    n = 10
    psi0 = workloads.random_state(n, seed=9).astype(np.complex64)
    state = torch.from_numpy(psi0.copy()).cuda()
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream().cuda_stream or None
    assert lib.grover_iterate_static(s, state.data_ptr(), 0, 1, None, 0, 1, None) == -1
    assert lib.grover_iterate_static(s, state.data_ptr(), 35, 1, None, 0, 1, None) == -1
    assert lib.grover_iterate_static(s, state.data_ptr(), 1, 3, None, 0, 1, None) == -5
    assert lib.grover_iterate_static(s, state.data_ptr() + 8, n, 1, None, 0, 1, None) == -1
    assert lib.grover_iterate_static(s, state.data_ptr(), n, 1, None, 2, 1, None) == -1
    assert lib.grover_iterate_static(s, state.data_ptr(), n, 1, None, 0, 1 << 32, None) == -1
    assert b"2^32" in lib.grover_last_error(None)
    # a marked list that is not strictly increasing, or reaches past the state: rejected on the device,
    # the state untouched
    for bad in ([5, 3], [4, 4], [7, 1 << n]):
        arr = np.array(bad, dtype=np.uint64)
        status.fill_(9)
        assert _static(G, state, n, 1, _device_marks(arr), arr.size, 4, status) == 0
        assert int(status.item()) == 2, bad
        assert np.array_equal(state.cpu().numpy(), psi0)
    # and a good call on the same scratch afterwards runs normally
    assert _static(G, state, n, 1, _device_marks(np.array([3], dtype=np.uint64)), 1, 4, status) == 0
    assert int(status.item()) == 0
    assert not np.array_equal(state.cpu().numpy(), psi0)
