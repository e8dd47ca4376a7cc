"""The bandwidth probe (grover_stream_probe, a measurement helper): what each mode does to the buffer, on
buffers that end inside a tile and shorter than one tile, and the argument checks."""
from __future__ import annotations

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_04635_amd as pkg

    pkg.load()
    return pkg


def _probe(G, buf, nbytes, passes, mode):
    import torch

    ms = G.grover_stream_probe(torch.cuda.current_stream().cuda_stream, buf.data_ptr(), nbytes, passes, mode)
    assert ms >= 0.0
    return buf.cpu().numpy()


@pytest.mark.parametrize("nbytes", [16, 48, 65536 * 3 + 400, (1 << 22) + 24])
def test_probe_modes_on_the_buffer(G, nbytes):
    """In place: every whole 16-byte vector negated per pass (an even count restores it); read-only: no change;
    write-only: every whole vector set to (p, 0, p, 0) of the last pass p; bytes past the last whole vector never
    touched.  Per-pass launches do the same."""
    import torch

    g = G.grover
    n = nbytes // 4 + 4  # floats, with a guard beyond nbytes
    x0 = np.random.default_rng(nbytes).standard_normal(n).astype(np.float32)
    whole = (nbytes // 16) * 4  # floats in whole vectors
    for mode in (0, g.GROVER_PROBE_LAUNCH_PER_PASS):
        buf = torch.from_numpy(x0.copy()).cuda()
        got = _probe(G, buf, nbytes, 3, mode)
        assert np.array_equal(got[:whole], -x0[:whole]) and np.array_equal(got[whole:], x0[whole:])
        got = _probe(G, buf, nbytes, 1, mode)
        assert np.array_equal(got, x0)
    buf = torch.from_numpy(x0.copy()).cuda()
    assert np.array_equal(_probe(G, buf, nbytes, 5, g.GROVER_PROBE_READ_ONLY), x0)
    got = _probe(G, buf, nbytes, 3, g.GROVER_PROBE_WRITE_ONLY)
    want = x0.copy()
    want[:whole] = np.tile(np.array([2.0, 0.0, 2.0, 0.0], dtype=np.float32), whole // 4)
    assert np.array_equal(got, want)
    buf = torch.from_numpy(x0.copy()).cuda()
    got = _probe(G, buf, nbytes, 2, g.GROVER_PROBE_NARROW | g.GROVER_PROBE_LAUNCH_PER_PASS)
    assert np.array_equal(got, x0)


def test_probe_rejections(G):
    import torch

    g = G.grover
    lib = G.load()
    buf = torch.zeros(64, dtype=torch.float32, device="cuda")
    ms = g.ctypes.c_float()
    s = torch.cuda.current_stream().cuda_stream or None
    assert lib.grover_stream_probe(s, None, 256, 1, 0, g.ctypes.byref(ms)) == -1
    assert lib.grover_stream_probe(s, buf.data_ptr() + 4, 128, 1, 0, g.ctypes.byref(ms)) == -1
    assert lib.grover_stream_probe(s, buf.data_ptr(), 8, 1, 0, g.ctypes.byref(ms)) == -1
    assert lib.grover_stream_probe(s, buf.data_ptr(), 256, 1, 16, g.ctypes.byref(ms)) == -1
    both = g.GROVER_PROBE_READ_ONLY | g.GROVER_PROBE_WRITE_ONLY
    assert lib.grover_stream_probe(s, buf.data_ptr(), 256, 1, both, g.ctypes.byref(ms)) == -1
    assert lib.grover_stream_probe(s, buf.data_ptr(), 256, 1, 0, None) == -1
