"""The C-ABI library loads and exports what include/grover.h declares; host-only paths (no GPU needed)."""
from __future__ import annotations

import ctypes
import os
import re
import subprocess

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "grover.h")
LIB = os.path.join(ROOT, "paper_2005_04635_amd", "libgrover.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(grover_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2005_04635_amd import build

        build.build()
    import paper_2005_04635_amd as pkg

    return pkg.load()


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ["grover_init", "grover_iterate", "grover_sample", "grover_sample_u53", "grover_gate_iterate",
                 "grover_apply_hadamard_all", "grover_norm", "grover_optimal_iterations", "grover_destroy"]:
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2005_04635_amd import EXPORTS

    names = declared_functions()
    assert sorted(EXPORTS) == names, "binding and header disagree"
    for name in names:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (grover_\w+)", out))
    assert set(names) <= exported


def test_library_is_gfx950_device_code():
    """The shared object embeds a gfx950 code object bundle."""
    data = open(LIB, "rb").read()
    assert b"gfx950" in data


def test_optimal_iterations_host_only(lib):
    from paper_2005_04635_amd import grover_optimal_iterations as k

    assert k(3, 1) == 2 and k(10, 1) == 25 and k(28, 8) == 4549 and k(26, 4) == 3216 and k(20, 3) == 464
    assert k(10, 0) == 0 and k(3, 9) == 0 and k(64, 1) == 0
    assert k(1, 1) == 1 and k(1, 2) == 0  # N = 2: one marked -> floor(pi/4 * sqrt 2) = 1


def test_status_strings_and_null_handling(lib):
    assert lib.grover_status_str(0) == b"ok"
    for code in range(-7, 0):
        assert lib.grover_status_str(code) not in (b"", b"unknown status")
    assert lib.grover_status_str(-99) == b"unknown status"
    assert lib.grover_last_error(None) == b"no context"
    assert lib.grover_iterate(None, 5) == -1
    assert lib.grover_gate_iterate_blocked(None, 1) == -1
    assert lib.grover_apply_hadamard_all_blocked(None) == -1
    assert lib.grover_sync(None) == -1
    lib.grover_destroy(None)


@pytest.mark.parametrize("field,value", [("n", 0), ("n", 35), ("dtype", 4), ("oracle_kind", 2), ("form", 5),
                                         ("flags", 1), ("hash_bits", 65), ("accum", 3), ("update", 2)])
def test_init_rejects_invalid_config_before_touching_the_device(lib, field, value):
    from paper_2005_04635_amd.grover import grover_config

    cfg = grover_config()
    cfg.n = 10
    setattr(cfg, field, value)
    ctx = ctypes.c_void_p()
    assert lib.grover_init(ctypes.byref(ctx), ctypes.byref(cfg), None, None, 0) == -1
    assert not ctx.value


def test_init_rejects_bad_marked_lists(lib):
    from paper_2005_04635_amd.grover import grover_config

    def init_with(marks, n=4):
        arr = (ctypes.c_uint64 * max(len(marks), 1))(*marks)
        cfg = grover_config()
        cfg.n = n
        cfg.m = len(marks)
        cfg.marked = ctypes.cast(arr, ctypes.POINTER(ctypes.c_uint64))
        ctx = ctypes.c_void_p()
        return lib.grover_init(ctypes.byref(ctx), ctypes.byref(cfg), None, None, 0)

    assert init_with([3, 3]) == -1       # duplicate: the oracle would flip it twice
    assert init_with([16]) == -1         # out of range for n = 4
    assert init_with(list(range(17))) == -1  # m > N
    cfg = grover_config()
    cfg.n = 4
    cfg.m = 2  # list kind with a null list
    ctx = ctypes.c_void_p()
    assert lib.grover_init(ctypes.byref(ctx), ctypes.byref(cfg), None, None, 0) == -1
    assert lib.grover_init(None, ctypes.byref(cfg), None, None, 0) == -1
    assert lib.grover_init(ctypes.byref(ctx), None, None, None, 0) == -1


def test_resident_form_limit(lib):
    from paper_2005_04635_amd.grover import grover_config

    cfg = grover_config()
    cfg.n = 15
    cfg.form = 2  # resident holds at most 2^14 amplitudes
    ctx = ctypes.c_void_p()
    assert lib.grover_init(ctypes.byref(ctx), ctypes.byref(cfg), None, None, 0) == -5


@pytest.mark.parametrize("dtype,accum", [(0, 0), (2, 0), (3, 0), (1, 1), (1, 2)])
def test_held_form_is_complex64_with_binary64_sums(lib, dtype, accum):
    """The held form exists for complex64 storage and binary64 sums only; rejected before device work."""
    from paper_2005_04635_amd.grover import grover_config

    cfg = grover_config()
    cfg.n, cfg.dtype, cfg.accum, cfg.form = 16, dtype, accum, 4
    ctx = ctypes.c_void_p()
    assert lib.grover_init(ctypes.byref(ctx), ctypes.byref(cfg), None, None, 0) == -5


@pytest.mark.parametrize("dtype,accum,form", [(0, 0, 1), (2, 0, 1), (3, 0, 1), (1, 1, 1), (1, 2, 0), (1, 0, 3),
                                               (2, 0, 2)])
def test_binary32_update_needs_complex64_binary64_sums(lib, dtype, accum, form):
    """The binary32 update exists for complex64 storage with binary64 sums, in the fused, one-workgroup and
    held forms; anything else is rejected before device work."""
    from paper_2005_04635_amd.grover import grover_config

    cfg = grover_config()
    cfg.n, cfg.dtype, cfg.accum, cfg.form, cfg.update = 10, dtype, accum, form, 1
    ctx = ctypes.c_void_p()
    assert lib.grover_init(ctypes.byref(ctx), ctypes.byref(cfg), None, None, 0) == -5


@pytest.mark.parametrize("dtype,accum,form", [(3, 0, 2), (3, 0, 3), (1, 1, 2), (1, 2, 3), (2, 1, 3)])
def test_reduced_precision_needs_the_fused_form(lib, dtype, accum, form):
    """bfloat16 storage and binary32 sums exist in the fused form only."""
    from paper_2005_04635_amd.grover import grover_config

    cfg = grover_config()
    cfg.n, cfg.dtype, cfg.accum, cfg.form = 10, dtype, accum, form
    ctx = ctypes.c_void_p()
    assert lib.grover_init(ctypes.byref(ctx), ctypes.byref(cfg), None, None, 0) == -5


def test_state_smaller_than_one_vector_is_rejected(lib):
    """Every kernel moves the state in whole 16-byte vectors; complex bfloat16 at n = 1 (two amplitudes, 8
    bytes) is less than one and is rejected before any device work; every other type fits at n = 1."""
    from paper_2005_04635_amd.grover import grover_config

    cfg = grover_config()
    cfg.n, cfg.dtype, cfg.form = 1, 3, 1
    ctx = ctypes.c_void_p()
    assert lib.grover_init(ctypes.byref(ctx), ctypes.byref(cfg), None, None, 0) == -5
    assert not ctx.value


def test_bf16_host_conversions_round_once_to_nearest_even():
    import numpy as np

    from paper_2005_04635_amd.grover import bf16_pairs_to_complex, complex_to_bf16_pairs

    x = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8) + 0.25j, 1 / 3, 2.0 ** -13])
    back = bf16_pairs_to_complex(complex_to_bf16_pairs(x))
    assert back[0] == 1.0 and back[1] == 1 + 2.0 ** -6 and back[2] == -1.0 + 0.25j
    assert abs(back[3] - 1 / 3) <= 2.0 ** -9 / 3 * 2 and back[4] == 2.0 ** -13
    # one correct rounding from binary64 even where rounding through binary32 first would differ:
    # 1 + 2^-8 + 2^-30 lies just above the tie, binary32 would round it onto the tie, then to even
    y = np.array([1 + 2.0 ** -8 + 2.0 ** -30])
    assert bf16_pairs_to_complex(complex_to_bf16_pairs(y))[0] == 1 + 2.0 ** -7


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    import paper_2005_04635_amd.grover as g

    monkeypatch.setattr(g, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        g.load(str(tmp_path / "nope.so"))


def _batch_cfg(n, m, marks, dtype=1):
    from paper_2005_04635_amd.grover import grover_batch_config

    keep = [(ctypes.c_uint32 * len(n))(*n), (ctypes.c_uint64 * len(m))(*m),
            (ctypes.c_uint64 * max(len(marks), 1))(*marks)]
    cfg = grover_batch_config()
    cfg.count = len(n)
    cfg.n = ctypes.cast(keep[0], ctypes.POINTER(ctypes.c_uint32))
    cfg.m = ctypes.cast(keep[1], ctypes.POINTER(ctypes.c_uint64))
    if marks:
        cfg.marked = ctypes.cast(keep[2], ctypes.POINTER(ctypes.c_uint64))
    cfg.dtype = dtype
    return cfg, keep


@pytest.mark.parametrize("n,m,marks,status", [
    ([4], [1], [16], -1),            # index out of range
    ([4], [2], [3, 3], -1),          # duplicate
    ([0], [0], [], -1),              # no qubits
    ([25], [1], [0], -1),            # above the batch size limit
    ([3], [9], list(range(9)), -1),  # m > N
    ([3, 4], [1, 1], [2], -1),       # marks given for fewer than sum(m): passed as a null list
])
def test_batch_init_rejects_invalid_configs(lib, n, m, marks, status):
    cfg, keep = _batch_cfg(n, m, marks)
    if len(marks) < sum(m):
        cfg.marked = None
    b = ctypes.c_void_p()
    assert lib.grover_batch_init(ctypes.byref(b), ctypes.byref(cfg), None) == status
    assert not b.value


def test_batch_init_rejects_other_fields(lib):
    b = ctypes.c_void_p()
    cfg, keep = _batch_cfg([4], [1], [3], dtype=2)
    assert lib.grover_batch_init(ctypes.byref(b), ctypes.byref(cfg), None) == -5  # complex128 batches
    cfg, keep = _batch_cfg([4], [1], [3])
    cfg.flags = 1
    assert lib.grover_batch_init(ctypes.byref(b), ctypes.byref(cfg), None) == -1
    cfg.flags, cfg.reserved = 0, 1
    assert lib.grover_batch_init(ctypes.byref(b), ctypes.byref(cfg), None) == -1
    cfg.reserved, cfg.update = 0, 2
    assert lib.grover_batch_init(ctypes.byref(b), ctypes.byref(cfg), None) == -1
    cfg.update, cfg.count = 0, 0
    assert lib.grover_batch_init(ctypes.byref(b), ctypes.byref(cfg), None) == -1
    assert lib.grover_batch_init(None, ctypes.byref(cfg), None) == -1
    assert lib.grover_batch_init(ctypes.byref(b), None, None) == -1
    assert not b.value


def test_batch_null_handles(lib):
    assert lib.grover_batch_run(None) == -1
    assert lib.grover_batch_sync(None) == -1
    assert lib.grover_batch_capture(None) == -1
    assert lib.grover_batch_set_tiling(None, 10, 2, 0) == -1
    assert lib.grover_batch_tune(None, None, None, None, None) == -1
    assert lib.grover_batch_last_error(None) == b"no batch"
    lib.grover_batch_destroy(None)


def test_batch_workload_statistics():
    """The 4096-instance workload: n spans [8, 20], M spans [1, 8], marks distinct and in range."""
    import math

    import numpy as np

    import workloads

    n, m, marks = workloads.BATCH_4096.instances()
    assert n.size == 4096 and n.min() == 8 and n.max() == 20 and m.min() == 1 and m.max() == 8
    for b in range(0, 4096, 97):
        mk = marks[b]
        assert mk.size == m[b] and np.unique(mk).size == mk.size and int(mk.max()) < (1 << int(n[b]))
    N = np.ldexp(1.0, n.astype(int))
    updates = float(np.sum(N * np.floor(math.pi / 4 * np.sqrt(N / m))))
    assert 2.2e11 < updates < 2.3e11


def _phase_cfg(**kw):
    from paper_2005_04635_amd.grover import grover_phase_config

    cfg = grover_phase_config()
    cfg.n, cfg.batch, cfg.iterations, cfg.dtype = 6, 2, 8, 1
    keep = (ctypes.c_uint64 * 3)(3, 17, 40)
    cfg.marked = ctypes.cast(keep, ctypes.POINTER(ctypes.c_uint64))
    cfg.m = 3
    for k, v in kw.items():
        setattr(cfg, k, v)
    return cfg, keep


@pytest.mark.parametrize("field,value,status", [("n", 0, -1), ("n", 31, -1), ("batch", 0, -1),
                                                ("iterations", 0, -1), ("flags", 1, -1), ("m", 65, -1),
                                                ("dtype", 2, -5), ("dtype", 0, -5)])
def test_phase_init_rejects_invalid_configs(lib, field, value, status):
    cfg, keep = _phase_cfg(**{field: value})
    p = ctypes.c_void_p()
    assert lib.grover_phase_init(ctypes.byref(p), ctypes.byref(cfg), None) == status
    assert not p.value


def test_phase_init_rejects_bad_marks_and_nulls(lib):
    p = ctypes.c_void_p()
    for marks in ([3, 3], [64]):
        arr = (ctypes.c_uint64 * len(marks))(*marks)
        cfg, keep = _phase_cfg(m=len(marks), marked=ctypes.cast(arr, ctypes.POINTER(ctypes.c_uint64)))
        assert lib.grover_phase_init(ctypes.byref(p), ctypes.byref(cfg), None) == -1
    cfg, keep = _phase_cfg(marked=None)
    assert lib.grover_phase_init(ctypes.byref(p), ctypes.byref(cfg), None) == -1
    assert lib.grover_phase_init(None, ctypes.byref(cfg), None) == -1
    assert lib.grover_phase_init(ctypes.byref(p), None, None) == -1
    assert lib.grover_phase_forward(None, None, None, None) == -1
    assert lib.grover_phase_backward(None, None, None, None) == -1
    assert lib.grover_phase_sync(None) == -1
    assert lib.grover_phase_set_form(None, 0) == -1
    assert lib.grover_phase_set_team(None, 1) == -1
    assert lib.grover_phase_last_error(None) == b"no phase context"
    lib.grover_phase_destroy(None)


def test_stream_probe_rejects_bad_arguments_before_touching_the_device(lib):
    ms = ctypes.c_float()
    assert lib.grover_stream_probe(None, None, 256, 1, 0, ctypes.byref(ms)) == -1
    assert lib.grover_stream_probe(None, ctypes.c_void_p(0x1004), 256, 1, 0, ctypes.byref(ms)) == -1
    assert lib.grover_stream_probe(None, ctypes.c_void_p(0x1000), 8, 1, 0, ctypes.byref(ms)) == -1
    assert lib.grover_stream_probe(None, ctypes.c_void_p(0x1000), 256, 1, 32, ctypes.byref(ms)) == -1
    assert lib.grover_stream_probe(None, ctypes.c_void_p(0x1000), 256, 1, 5, ctypes.byref(ms)) == -1
    assert lib.grover_stream_probe(None, ctypes.c_void_p(0x1000), 256, 1, 0, None) == -1


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU (a search's state is not sharded): --gpus above 1 exits with status 2 and
    a message, before anything touches a device."""
    import sys

    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)
