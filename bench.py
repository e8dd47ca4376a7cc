"""Benchmark of the Grover hot path on one MI355X: amplitude-updates/s and fraction of peak HBM bandwidth
per Grover iteration at n = 28, against the plain binary64 form.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-forms]
    python bench.py --sweep table1      (the paper's Table 1 sizes: proposed vs gate-level, one line each)
    python bench.py --sweep precision   (storage x accumulator of the mean at n = 26, one line each)
    python bench.py --sweep batch       (4096 independent searches: tilings, the tuned graph, one-by-one)
    python bench.py --sweep adjoint     (generalized iteration with phases: forward + adjoint gradient)
    python bench.py --sweep update      (element update in binary32 against binary64: on-chip forms, batch)
    python bench.py --sweep scaling     (one full search per n = 14 ... 28: the N^(3/2) growth of a search)

Workload (synthetic by construction; the paper uses no dataset): the single large instance, n = 28
(2^28 complex64 amplitudes, 2 GiB), M = 8 marked indices defined by the hash predicate
(SplitMix64_i(seed) mod 2^25 == 0), floor(pi/4 sqrt(N/M)) = 4549 iterations, 10^6 measurement shots.

One step is one pass of the whole hot path on inputs already resident in HBM: the uniform superposition
is written, 4549 fused iterations run (one persistent cooperative kernel), the norm is taken, and 10^6
shots are sampled with device-resident uniforms.  `value` = N * 4549 / (wall time of one step).

The process talks to the GPU only through libgrover's C ABI and the HIP runtime it links (events, device
buffers, a stream); no framework is loaded.

Printed JSON line (last line of stdout):
  roofline      the fused iterate kernel: algorithmic bytes per launch (16 B per amplitude-update plus the
                8 B-per-amplitude prologue read) / its mean duration measured with HIP events on the
                stream it runs on, against MI355X's 8 TB/s; `traffic` is the counter-measured HBM bytes per
                launch from the committed rocprofv3 summary (null when the kernel source changed since)
  forms         the plain binary64 comparator (complex128, oracle / sum / update kernels per iteration)
                and other forms, timed on a bounded number of iterations
  cpu_baseline  the CPU oracle (single thread, binary64) on a bounded sample of the same workload
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, public datasheet
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "fused_iterate_n28_c64_traffic.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2005_04635_amd", "csrc", f) for f in ("k_fused.hip", "internal.h")]
PAPER_CPU_N20_UPDATES_PER_S = 1048576 * 804 / 20.005  # Table 1, proposed simulator, n = 20, i3-5005U 1 thread


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def committed_traffic():
    """HBM bytes per fused-iterate launch from the committed counter summary, if it matches this source."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    text = open(TRAFFIC_SUMMARY).read()
    sha = re.search(r"^source_sha:\s*(\S+)", text, re.M)
    val = re.search(r"^hbm_bytes_per_launch:\s*([0-9.eE+]+)", text, re.M)
    if not sha or not val or sha.group(1) != kernel_source_sha():
        return None
    return float(val.group(1))


class Hip:
    """The few HIP runtime calls the benchmark needs (the runtime libgrover itself links)."""

    def __init__(self):
        self.lib = ctypes.CDLL("libamdhip64.so.7")
        self.events = []  # every event created and not yet destroyed
        P = ctypes.c_void_p
        for name, args in {
            "hipSetDevice": [ctypes.c_int], "hipDeviceSynchronize": [], "hipStreamCreate": [ctypes.POINTER(P)],
            "hipStreamSynchronize": [P], "hipStreamDestroy": [P], "hipEventCreate": [ctypes.POINTER(P)],
            "hipEventDestroy": [P], "hipEventRecord": [P, P],
            "hipEventSynchronize": [P], "hipEventElapsedTime": [ctypes.POINTER(ctypes.c_float), P, P],
            "hipMalloc": [ctypes.POINTER(P), ctypes.c_size_t], "hipFree": [P],
            "hipMemcpy": [P, P, ctypes.c_size_t, ctypes.c_int],
            "hipMemcpyAsync": [P, P, ctypes.c_size_t, ctypes.c_int, P],
            "hipDeviceGetName": [ctypes.c_char_p, ctypes.c_int, ctypes.c_int],
        }.items():
            fn = getattr(self.lib, name)
            fn.restype = ctypes.c_int
            fn.argtypes = args

    def ok(self, rc, what):
        if rc != 0:
            raise RuntimeError(f"{what} failed with HIP error {rc}")

    def event(self):
        e = ctypes.c_void_p()
        self.ok(self.lib.hipEventCreate(ctypes.byref(e)), "hipEventCreate")
        self.events.append(e)
        return e

    def destroy_events(self, *evs) -> None:
        for e in evs:
            if any(e is x for x in self.events):
                self.events = [x for x in self.events if x is not e]
                self.lib.hipEventDestroy(e)

    def close(self, stream) -> None:
        """Wait for the device, then release every event still held and the stream."""
        self.lib.hipDeviceSynchronize()
        self.destroy_events(*list(self.events))
        if stream is not None and stream.value:
            self.lib.hipStreamDestroy(stream)

    def elapsed_ms(self, e0, e1) -> float:
        ms = ctypes.c_float()
        self.ok(self.lib.hipEventSynchronize(e1), "hipEventSynchronize")
        self.ok(self.lib.hipEventElapsedTime(ctypes.byref(ms), e0, e1), "hipEventElapsedTime")
        return ms.value

    def malloc(self, nbytes: int):
        p = ctypes.c_void_p()
        self.ok(self.lib.hipMalloc(ctypes.byref(p), nbytes), "hipMalloc")
        return p

    def name(self) -> str:
        buf = ctypes.create_string_buffer(256)
        self.lib.hipDeviceGetName(buf, 256, 0)
        return buf.value.decode(errors="replace")


def make_config(pkg, n, dtype, marks=None, hash_seed=None, hash_bits=0, m=0, form="fused", update="f64"):
    import numpy as np

    g = pkg.grover
    cfg = g.grover_config()
    cfg.n, cfg.dtype, cfg.form, cfg.flags = n, g.DTYPES[dtype], g.FORMS[form], 0
    cfg.update = g.UPDATES[update]
    keep = None
    if hash_seed is not None:
        cfg.oracle_kind, cfg.hash_seed, cfg.hash_bits, cfg.m = g.GROVER_ORACLE_HASH, hash_seed, hash_bits, m
    else:
        keep = np.ascontiguousarray(np.asarray(marks, dtype=np.uint64))
        cfg.oracle_kind, cfg.m = g.GROVER_ORACLE_LIST, keep.size
        cfg.marked = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    return cfg, keep


def time_form(pkg, hip, stream, n, dtype, form, marks, iters, bytes_per_update, prologue_bytes):
    """Amplitude-updates/s of one form on a resident state, HIP events on its stream."""
    cfg, keep = make_config(pkg, n, dtype, marks=marks, form=form)
    ctx = pkg.grover_init(cfg, stream.value, 0, 0)
    try:
        pkg.grover_iterate(ctx, 2)
        pkg.grover_sync(ctx)
        e0, e1 = hip.event(), hip.event()
        hip.lib.hipEventRecord(e0, stream)
        pkg.grover_iterate(ctx, iters)
        hip.lib.hipEventRecord(e1, stream)
        ms = hip.elapsed_ms(e0, e1)
        pkg.grover_sync(ctx)
    finally:
        pkg.grover_destroy(ctx)
    N = 1 << n
    gbs = (bytes_per_update * N * iters + prologue_bytes * N) / (ms / 1e3) / 1e9
    return {"form": form, "storage": dtype, "iterations": iters, "ms": round(ms, 3),
            "amplitude_updates_per_s": N * iters / (ms / 1e3), "algorithmic_gbs": round(gbs, 1),
            "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}


def cpu_baseline(w, marks, iters):
    import oracle

    orc = oracle.default()
    N = 1 << w.n
    t0 = time.perf_counter()
    psi = orc.init_uniform(w.n)
    t1 = time.perf_counter()
    orc.iterate(psi, marks, iters)
    t2 = time.perf_counter()
    del psi
    return {"value": N * iters / (t2 - t1), "unit": "amplitude-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"n={w.n} M={w.m} hash marks, {iters} iterations of the binary64 CPU oracle from the uniform "
                      f"state ({t2 - t1:.1f} s, plus {t1 - t0:.1f} s untimed initialisation), one host thread",
            "host_cpus": os.cpu_count()}


def cpu_worker(spec: str) -> int:
    """One process of the all-core CPU baseline (no GPU is touched): the binary64 oracle from the uniform
    state of the n = 28 workload for a few iterations; prints its own time as one JSON line."""
    import numpy as np

    import oracle
    import workloads

    iters = int(spec)
    w = workloads.HASH_N28
    marks = np.loadtxt(os.path.join(ROOT, "tests", "golden", "hash_marks_n28.txt"), dtype=np.uint64, comments="#")
    orc = oracle.default()
    psi = orc.init_uniform(w.n)
    t1 = time.perf_counter()
    orc.iterate(psi, marks, iters)
    t2 = time.perf_counter()
    print(json.dumps({"iterations": iters, "s": t2 - t1}), flush=True)
    return 0


def cpu_baseline_all_cores(w, iters, single):
    """The same oracle on every host core at once: one child process per core (bench.py --cpu-worker; the
    oracle is single-threaded and unchanged), each iterating its own copy of the n = 28 state from the
    uniform superposition; the aggregate rate is the sum of the processes' updates over the longest one's
    time.  Returned as the baseline, with the single-thread figure beside it."""
    import subprocess

    procs = min(os.cpu_count() or 1, 16)  # at most 16: one GPU's share of a shared host
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-worker", str(iters)]
    children = [subprocess.Popen(cmd, stdout=subprocess.PIPE, text=True) for _ in range(procs)]
    times = []
    for c in children:
        out, _ = c.communicate()
        if c.returncode != 0:
            raise RuntimeError(f"CPU baseline worker failed with status {c.returncode}")
        times.append(json.loads(out.strip().splitlines()[-1])["s"])
    N = 1 << w.n
    rate = procs * N * iters / max(times)
    return {"value": rate, "unit": "amplitude-updates/s", "cores": procs, "kind": "oracle",
            "sample": f"n={w.n} M={w.m} hash marks: {procs} concurrent processes of the single-threaded binary64 "
                      f"oracle, each {iters} iterations from the uniform state on its own 4 GiB state "
                      f"(slowest {max(times):.1f} s, fastest {min(times):.1f} s); rate = all updates / slowest",
            "single_thread": single, "host_cpus": os.cpu_count()}


PAPER_TABLE1_S = {  # Table 1: seconds on an Intel i3-5005U, one thread (conventional, proposed)
    10: (0.010, 0.025), 16: (3.768, 0.349), 18: (37.708, 2.579), 20: (357.029, 20.005)}


def cpu_table1_times(n: int, mark, k: int) -> dict:
    """The binary64 CPU oracle on this host, one thread, at one of Table 1's sizes: the proposed search
    (uniform state, then k iterations of Algorithms 3 and 4) and the conventional one (Algorithm 2's
    iteration: H^n by n applications of Algorithm 1, the phase shift, H^n).  The conventional search runs in
    full up to n = 16; above, 4 of its iterations are timed and scaled to k (labelled)."""
    import oracle

    orc = oracle.default()
    t0 = time.perf_counter()
    orc.search(n, mark, k)
    t_prop = time.perf_counter() - t0
    k_conv = k if n <= 16 else 4
    psi = orc.init_uniform(n)
    t0 = time.perf_counter()
    orc.gate_iterate(psi, mark, k_conv)
    t_conv = (time.perf_counter() - t0) * k / k_conv
    return {"proposed": t_prop, "conventional": t_conv, "speedup": t_conv / t_prop,
            "conventional_basis": "full search" if k_conv == k else f"{k_conv} iterations timed, scaled to {k}",
            "host_cpus": os.cpu_count()}


def sweep_table1(pkg, hip, stream) -> None:
    """The paper's Table 1 on this GPU: a full single-solution search (the optimal number of iterations from
    the uniform superposition) with the proposed iteration and with the gate-level one (H^n as n single-qubit
    passes, and as the blocked Walsh-Hadamard transform), at the paper's sizes; then three iterations of
    each at n = 28.  One JSON line per size."""
    import workloads

    for n in (10, 16, 18, 20, 28):
        mark = [workloads.marked_index_from_seed(n, 1000 + n)]
        cfg, keep = make_config(pkg, n, "c64", marks=mark, form="auto")
        ctx = pkg.grover_init(cfg, stream.value, 0, 0)
        k_full = pkg.grover_optimal_iterations(n, 1)
        k = k_full if n <= 20 else 3
        res = {"sweep": "table1", "n": n, "iterations": k, "storage": "c64",
               "form": ["", "fused", "resident", "two_pass", "held"][pkg.grover_query(ctx, 0)]}
        for path, fn in (("proposed", pkg.grover_iterate), ("gate_level", pkg.grover_gate_iterate),
                         ("gate_level_blocked", pkg.grover_gate_iterate_blocked)):
            pkg.grover_reset(ctx)
            fn(ctx, 1)  # warm
            pkg.grover_reset(ctx)
            pkg.grover_sync(ctx)
            e0, e1 = hip.event(), hip.event()
            hip.lib.hipEventRecord(e0, stream)
            fn(ctx, k)
            hip.lib.hipEventRecord(e1, stream)
            ms = hip.elapsed_ms(e0, e1)
            pkg.grover_sync(ctx)
            res[path + "_s"] = ms / 1e3
            res[path + "_amplitude_iterations_per_s"] = (1 << n) * k / (ms / 1e3)
        if res["form"] == "held":
            # the fused form of the same search, for comparison with the held form AUTO chose
            fcfg, fkeep = make_config(pkg, n, "c64", marks=mark, form="fused")
            fctx = pkg.grover_init(fcfg, stream.value, 0, 0)
            pkg.grover_iterate(fctx, 1)
            pkg.grover_reset(fctx)
            pkg.grover_sync(fctx)
            e0, e1 = hip.event(), hip.event()
            hip.lib.hipEventRecord(e0, stream)
            pkg.grover_iterate(fctx, k)
            hip.lib.hipEventRecord(e1, stream)
            ms = hip.elapsed_ms(e0, e1)
            pkg.grover_sync(fctx)
            pkg.grover_destroy(fctx)
            res["proposed_fused_s"] = ms / 1e3
        res["speedup_proposed_over_gate"] = res["gate_level_s"] / res["proposed_s"]
        res["speedup_proposed_over_blocked_gate"] = res["gate_level_blocked_s"] / res["proposed_s"]
        if n in PAPER_TABLE1_S:
            conv, prop = PAPER_TABLE1_S[n]
            res["paper_i3_1thread_s"] = {"conventional": conv, "proposed": prop, "speedup": conv / prop}
            res["cpu_oracle_1thread_s"] = cpu_table1_times(n, mark, k)
        pkg.grover_destroy(ctx)
        print(json.dumps(res), flush=True)


def sweep_scaling(pkg, hip, stream, runs: int) -> None:
    """The paper's complexity statement on this GPU: each iteration is one O(N) pass and a single-solution
    search takes floor(pi/4 sqrt(N)) of them, so a search costs O(N^(3/2)) and grows about 8x for two more
    qubits (Table 1's own ratio from n = 18 to n = 20 is 20.005 / 2.579 = 7.76).  One full search per
    n = 14 ... 28 (complex64, one solution, the form AUTO picks), the median of `runs` searches below n = 26
    and one above; one JSON line per n, with the ratio to the search two qubits smaller."""
    import workloads

    by_n = {}
    for n in range(14, 29):
        mark = [workloads.marked_index_from_seed(n, 2000 + n)]
        cfg, keep = make_config(pkg, n, "c64", marks=mark, form="auto")
        ctx = pkg.grover_init(cfg, stream.value, 0, 0)
        k = pkg.grover_optimal_iterations(n, 1)
        pkg.grover_iterate(ctx, 1)  # warm
        times = []
        for _ in range(runs if n < 26 else 1):
            pkg.grover_reset(ctx)
            pkg.grover_sync(ctx)
            e0, e1 = hip.event(), hip.event()
            hip.lib.hipEventRecord(e0, stream)
            pkg.grover_iterate(ctx, k)
            hip.lib.hipEventRecord(e1, stream)
            times.append(hip.elapsed_ms(e0, e1))
            hip.destroy_events(e0, e1)
            pkg.grover_sync(ctx)
        ms = sorted(times)[len(times) // 2]
        res = {"sweep": "scaling", "n": n, "iterations": k, "storage": "c64",
               "form": ["", "fused", "resident", "two_pass", "held"][pkg.grover_query(ctx, 0)],
               "search_ms": ms, "us_per_iteration": ms * 1e3 / k,
               "ns_per_amplitude_iteration": ms * 1e6 / (k * (1 << n))}
        if n - 2 in by_n:
            res["ratio_to_n_minus_2"] = ms / by_n[n - 2]
        by_n[n] = ms
        pkg.grover_destroy(ctx)
        print(json.dumps(res), flush=True)


def sweep_precision(pkg, hip, stream) -> None:
    """Storage {complex128, complex64, complex bfloat16} x accumulator of the mean {binary64, binary32,
    Kahan binary32} on the precision workload (n = 26, M = 4, 3216 iterations from the uniform state):
    error of the two amplitude values against the binary64 oracle and against Grover's closed form, time per
    iteration and its ratio to the plain binary64 form (complex128, separate oracle / sum / update kernels).
    One JSON line per setting; the state is read back to check the two-class structure."""
    import numpy as np

    import oracle
    import workloads

    orc = oracle.default()
    w = workloads.PRECISION_N26
    marks = np.array(w.marks, dtype=np.uint64)
    N = 1 << w.n
    a_ref, b_ref = orc.two_class(w.n, w.m, w.iterations)
    theta = math.asin(math.sqrt(w.m / N))
    a_cf = math.sin((2 * w.iterations + 1) * theta) / math.sqrt(w.m)
    b_cf = math.cos((2 * w.iterations + 1) * theta) / math.sqrt(N - w.m)
    plain = time_form(pkg, hip, stream, w.n, "c128", "two_pass", marks, 300, 48, 0)
    plain_ms = plain["ms"] / plain["iterations"]
    print(json.dumps({"sweep": "precision", "storage": "c128", "accum": "f64", "form": "two_pass (plain FP64)",
                      "ms_per_iteration": plain_ms, "amplitude_updates_per_s": plain["amplitude_updates_per_s"],
                      "algorithmic_gbs": plain["algorithmic_gbs"]}), flush=True)
    for storage in ("c128", "c64", "cbf16"):
        eb = pkg.grover.ELEM_BYTES[pkg.grover.DTYPES[storage]]
        for accum in ("f64", "f32", "f32_kahan"):
            cfg, keep = make_config(pkg, w.n, storage, marks=marks, form="fused")
            cfg.accum = pkg.grover.ACCUMS[accum]
            ctx = pkg.grover_init(cfg, stream.value, 0, 0)
            e0, e1 = hip.event(), hip.event()
            hip.lib.hipEventRecord(e0, stream)
            pkg.grover_iterate(ctx, w.iterations)
            hip.lib.hipEventRecord(e1, stream)
            ms = hip.elapsed_ms(e0, e1)
            pkg.grover_sync(ctx)
            raw = np.empty(N * eb, dtype=np.uint8)
            pkg.grover_read_state(ctx, raw.ctypes.data, raw.nbytes)
            pkg.grover_destroy(ctx)
            if storage == "cbf16":
                psi = pkg.grover.bf16_pairs_to_complex(raw.view(np.uint16))
            else:
                psi = raw.view(np.complex128 if storage == "c128" else np.complex64)
            a, b = complex(psi[int(marks[0])]), complex(psi[0 if 0 not in marks else 1])
            two_class = bool(np.all(psi[marks.astype(np.int64)] == psi[int(marks[0])]))
            del psi, raw
            gbs = (2 * eb * N * w.iterations + eb * N) / (ms / 1e3) / 1e9
            print(json.dumps({
                "sweep": "precision", "n": w.n, "m": w.m, "iterations": w.iterations, "storage": storage,
                "accum": accum, "form": "fused",
                "marked_amplitude": a.real, "unmarked_amplitude": b.real,
                "p_marked": w.m * abs(a) ** 2,
                "max_abs_err_vs_fp64_oracle": max(abs(a - a_ref), abs(b - b_ref)),
                "max_abs_err_vs_closed_form": max(abs(a - a_cf), abs(b - b_cf)),
                "marked_equal": two_class, "ms_per_iteration": ms / w.iterations,
                "amplitude_updates_per_s": N * w.iterations / (ms / 1e3), "algorithmic_gbs": round(gbs, 1),
                "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
                "speedup_vs_plain_fp64": plain_ms / (ms / w.iterations)}), flush=True)


def batch_config(pkg, n, m, marks, update="f64"):
    import numpy as np

    g = pkg.grover
    keep = [np.ascontiguousarray(n, dtype=np.uint32), np.ascontiguousarray(m, dtype=np.uint64),
            np.ascontiguousarray(np.concatenate(marks), dtype=np.uint64)]
    cfg = g.grover_batch_config()
    cfg.count = keep[0].size
    cfg.n = keep[0].ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
    cfg.m = keep[1].ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    cfg.marked = keep[2].ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    cfg.dtype = g.GROVER_C64
    cfg.update = g.UPDATES[update]
    return cfg, keep


def sweep_batch(pkg, hip, stream, runs: int) -> None:
    """The 4096-instance batch: every candidate tiling timed (one JSON line each), then the fastest replayed
    from a captured graph `runs` times; against running the instances one by one, with the plain binary64
    form (complex128, separate oracle / sum / update kernels) and with the best single-instance form
    (complex64, `auto`), both timed on every 8th instance and scaled by amplitude-updates."""
    import numpy as np

    import workloads

    g = pkg.grover
    w = workloads.BATCH_4096
    n, m, marks = w.instances()
    cfg, keep = batch_config(pkg, n, m, marks)
    b = pkg.grover_batch_init(cfg, stream.value)
    updates = pkg.grover_batch_query(b, g.BQ_UPDATES)
    state_bytes = pkg.grover_batch_query(b, g.BQ_BYTES)
    alg_bytes = 16.0 * updates + 8.0 * float(np.sum(np.ldexp(1.0, n.astype(int))))
    grid = pkg.grover_batch_query(b, g.BQ_GRID)
    log(f"[bench] batch {w.name}: {w.count} instances, {updates:.4g} updates, {state_bytes / 2**30:.2f} GiB, "
        f"grid {grid}")

    def timed_run():
        e0, e1 = hip.event(), hip.event()
        hip.lib.hipEventRecord(e0, stream)
        pkg.grover_batch_run(b)
        hip.lib.hipEventRecord(e1, stream)
        ms = hip.elapsed_ms(e0, e1)
        pkg.grover_batch_sync(b)
        return ms

    cands = [(0, 1, 0)] + [(s, t, 0) for s in (18, 19, 20) for t in (2, 4, 8) if t <= grid]
    cands += [(19, 2, r) for r in (16, 8, 4, 2)]
    best = None
    for split, team, res in cands:
        pkg.grover_batch_set_tiling(b, split, team, res)
        timed_run()  # warm
        ms = min(timed_run() for _ in range(2))
        log(f"[bench] tiling split={split} team={team} resident={res}: {ms:.1f} ms")
        print(json.dumps({"sweep": "batch_tiling", "split_n": split, "team": team, "resident": res,
                          "in_teams": pkg.grover_batch_query(b, g.BQ_N_TEAM),
                          "phases": pkg.grover_batch_query(b, g.BQ_PHASES), "ms": round(ms, 3),
                          "amplitude_updates_per_s": updates / (ms / 1e3)}), flush=True)
        if best is None or ms < best[3]:
            best = (split, team, res, ms)
    pkg.grover_batch_set_tiling(b, best[0], best[1], best[2])
    pkg.grover_batch_capture(b)
    pkg.grover_batch_run(b)
    pkg.grover_batch_sync(b)
    hip.ok(hip.lib.hipDeviceSynchronize(), "hipDeviceSynchronize")
    e0, e1 = hip.event(), hip.event()
    t0 = time.perf_counter()
    hip.lib.hipEventRecord(e0, stream)
    for _ in range(runs):
        pkg.grover_batch_run(b)
    hip.lib.hipEventRecord(e1, stream)
    ms = hip.elapsed_ms(e0, e1) / runs
    pkg.grover_batch_sync(b)
    wall_ms = (time.perf_counter() - t0) * 1e3 / runs
    pkg.grover_batch_destroy(b)

    # one by one, on every 8th instance
    sample = list(range(0, w.count, 8))
    one_by_one = {}
    for dtype, form in (("c128", "two_pass"), ("c64", "auto")):
        t_ms, upd = 0.0, 0.0
        for i in sample:
            cfgi, keepi = make_config(pkg, int(n[i]), dtype, marks=marks[i], form=form)
            ctx = pkg.grover_init(cfgi, stream.value, 0, 0)
            k = pkg.grover_optimal_iterations(int(n[i]), int(m[i]))
            pkg.grover_sync(ctx)
            a0, a1 = hip.event(), hip.event()
            hip.lib.hipEventRecord(a0, stream)
            pkg.grover_reset(ctx)
            pkg.grover_iterate(ctx, k)
            hip.lib.hipEventRecord(a1, stream)
            t_ms += hip.elapsed_ms(a0, a1)
            pkg.grover_sync(ctx)
            pkg.grover_destroy(ctx)
            upd += float(1 << int(n[i])) * k
        one_by_one[f"{dtype}_{form}"] = {"amplitude_updates_per_s": upd / (t_ms / 1e3),
                                        "sample": f"every 8th instance ({len(sample)}), reset + iterate each, "
                                                  f"{t_ms:.0f} ms of device time"}
        log(f"[bench] one by one {dtype} {form}: {upd / (t_ms / 1e3):.4g} updates/s")
    rate = updates / (ms / 1e3)
    gbs = alg_bytes / (ms / 1e3) / 1e9
    print(json.dumps({
        "sweep": "batch", "workload": w.name, "instances": w.count, "amplitude_updates": updates,
        "state_bytes": state_bytes, "split_n": best[0], "team": best[1], "resident": best[2], "graph": True,
        "runs": runs,
        "ms_per_run": round(ms, 3), "wall_ms_per_run": round(wall_ms, 3), "amplitude_updates_per_s": rate,
        "algorithmic_gbs": round(gbs, 1), "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
        "one_by_one": one_by_one,
        "speedup_vs_plain_fp64_one_by_one": rate / one_by_one["c128_two_pass"]["amplitude_updates_per_s"],
        "speedup_vs_best_single_form_one_by_one": rate / one_by_one["c64_auto"]["amplitude_updates_per_s"],
    }), flush=True)


def sweep_update(pkg, hip, stream, runs: int) -> None:
    """The element update in binary32 (from 2S/N rounded to binary32) against binary64, complex64 storage and
    binary64 sums, where the update's instruction count bounds the time: one workgroup holding the state
    (n = 12), a held team (n = 16, 20, 22), the batch of 4096 searches (each update with its own tuned
    tiling, replayed from a captured graph); and the fused form at n = 28 (bound by HBM, for contrast; 400
    iterations).  For each: device time of one search (median of `runs`), amplitude-updates/s, and the error
    of the final state against the exact iteration (the binary64 oracle's two-class values) and against the
    oracle's model of that update.  One JSON line per case."""
    import numpy as np

    import oracle
    import workloads

    orc = oracle.default()
    g = pkg.grover
    for n, m, form in ((12, 2, "auto"), (16, 1, "auto"), (20, 1, "auto"), (22, 3, "auto"), (28, 8, "fused")):
        marks = np.sort(workloads.distinct_marks(n, m, seed=4000 + n))
        k = orc.optimal_iterations(n, m) if n < 28 else 400
        N = 1 << n
        a_ex, b_ex = orc.two_class(n, m, k)
        res = {"sweep": "update", "n": n, "m": m, "iterations": k, "storage": "c64", "accum": "f64"}
        for update in ("f64", "f32"):
            cfg, keep = make_config(pkg, n, "c64", marks=marks, form=form, update=update)
            ctx = pkg.grover_init(cfg, stream.value, 0, 0)
            res["form"] = ["", "fused", "resident", "two_pass", "held"][pkg.grover_query(ctx, 0)]
            pkg.grover_iterate(ctx, 1)
            times = []
            for _ in range(runs):
                pkg.grover_reset(ctx)
                e0, e1 = hip.event(), hip.event()
                hip.lib.hipEventRecord(e0, stream)
                pkg.grover_iterate(ctx, k)
                hip.lib.hipEventRecord(e1, stream)
                times.append(hip.elapsed_ms(e0, e1))
                hip.destroy_events(e0, e1)
            pkg.grover_sync(ctx)
            ms = sorted(times)[len(times) // 2]
            psi = np.empty(N, dtype=np.complex64)
            pkg.grover_read_state(ctx, psi.ctypes.data, psi.nbytes)
            pkg.grover_destroy(ctx)
            a = complex(psi[int(marks[0])])
            b = complex(psi[0 if 0 not in marks else int(np.setdiff1d(np.arange(8), marks)[0])])
            del psi
            a_md, b_md = orc.two_class_stored_update(n, m, k, 24, 24 if update == "f32" else 53)
            res[update] = {"ms": round(ms, 4), "amplitude_updates_per_s": N * k / (ms / 1e3),
                           "max_abs_err_vs_exact": max(abs(a - a_ex), abs(b - b_ex)),
                           "max_abs_err_vs_oracle_model": max(abs(a - a_md), abs(b - b_md))}
        res["speedup_f32_update"] = res["f64"]["ms"] / res["f32"]["ms"]
        print(json.dumps(res), flush=True)
        log(f"[bench] update n={n}: f64 {res['f64']['ms']:.3f} ms, f32 {res['f32']['ms']:.3f} ms")

    w = workloads.BATCH_4096
    n, m, marks = w.instances()
    res = {"sweep": "update", "workload": w.name, "instances": w.count, "storage": "c64", "accum": "f64"}
    for update in ("f64", "f32"):
        cfg, keep = batch_config(pkg, n, m, marks, update=update)
        b = pkg.grover_batch_init(cfg, stream.value)
        updates = pkg.grover_batch_query(b, g.BQ_UPDATES)
        split, team, resident, tuned_ms = pkg.grover_batch_tune(b)
        pkg.grover_batch_capture(b)
        pkg.grover_batch_run(b)
        pkg.grover_batch_sync(b)
        times = []
        for _ in range(runs):
            e0, e1 = hip.event(), hip.event()
            hip.lib.hipEventRecord(e0, stream)
            pkg.grover_batch_run(b)
            hip.lib.hipEventRecord(e1, stream)
            times.append(hip.elapsed_ms(e0, e1))
            hip.destroy_events(e0, e1)
        pkg.grover_batch_sync(b)
        ms = sorted(times)[len(times) // 2]
        worst_ex, worst_md = 0.0, 0.0
        for i in range(w.count):
            ni, mi = int(n[i]), int(m[i])
            ki = orc.optimal_iterations(ni, mi)
            psi = np.empty(1 << ni, dtype=np.complex64)
            pkg.grover_batch_read_state(b, i, psi.ctypes.data, psi.nbytes)
            mk = marks[i].astype(np.int64)
            a = complex(psi[mk[0]])
            um = np.ones(1 << ni, dtype=bool)
            um[mk] = False
            u = complex(psi[int(np.argmax(um))])
            a_ex, u_ex = orc.two_class(ni, mi, ki)
            a_md, u_md = orc.two_class_stored_update(ni, mi, ki, 24, 24 if update == "f32" else 53)
            worst_ex = max(worst_ex, abs(a - a_ex), abs(u - u_ex))
            worst_md = max(worst_md, abs(a - a_md), abs(u - u_md))
        pkg.grover_batch_destroy(b)
        res[update] = {"tiling": {"split_n": split, "team": team, "resident": resident}, "ms_per_run": round(ms, 3),
                       "amplitude_updates_per_s": updates / (ms / 1e3), "max_abs_err_vs_exact": worst_ex,
                       "max_abs_err_vs_oracle_model": worst_md}
        log(f"[bench] update batch {update}: {ms:.2f} ms (tiling {split}/{team}/{resident})")
    res["speedup_f32_update"] = res["f64"]["ms_per_run"] / res["f32"]["ms_per_run"]
    print(json.dumps(res), flush=True)


def sweep_adjoint(pkg, hip, stream, runs: int) -> None:
    """The differentiable workload (n = 20, M = 3, K = 64 iterations, 64 phase schedules ~ N(pi, 0.1)) in
    both forms of the library (states held on chip for all steps, the default at this size; states
    streamed from memory every step): forward runs (loss) and adjoint runs (gradient) timed with HIP events
    on the context's stream, their amplitude rates, memory traffic, accuracy against the binary64 oracle on
    two schedules, and the plain binary64 GPU form (standard iteration, complex128, separate kernels) at
    the same n for comparison.  One JSON line."""
    import numpy as np

    import oracle
    import workloads

    g = pkg.grover
    w = workloads.PHASE_N20
    marks = np.ascontiguousarray(w.marks(), dtype=np.uint64)
    phi, theta = w.schedules()
    cfg = g.grover_phase_config()
    cfg.n, cfg.batch, cfg.iterations, cfg.dtype = w.n, w.batch, w.K, g.GROVER_C64
    cfg.m = marks.size
    cfg.marked = marks.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    p = pkg.grover_phase_init(cfg, stream.value)
    every, nck = pkg.grover_phase_query(p, g.PQ_EVERY), pkg.grover_phase_query(p, g.PQ_CHECKPOINTS)
    team, grid = pkg.grover_phase_query(p, g.PQ_TEAM), pkg.grover_phase_query(p, g.PQ_GRID)
    held_teams = (pkg.grover_phase_query(p, g.PQ_HELD_TEAM_F), pkg.grover_phase_query(p, g.PQ_HELD_TEAM_A))
    B, K, N = w.batch, w.K, 1 << w.n
    nbytes = B * K * 8
    bufs = {name: hip.malloc(size) for name, size in
            (("phi", nbytes), ("theta", nbytes), ("loss", B * 8), ("dloss", B * 8), ("dphi", nbytes),
             ("dtheta", nbytes))}
    ones = np.ones(B)
    for name, arr in (("phi", phi), ("theta", theta), ("dloss", ones)):
        a = np.ascontiguousarray(arr, dtype=np.float64)
        hip.ok(hip.lib.hipMemcpy(bufs[name], ctypes.c_void_p(a.ctypes.data), a.nbytes, 1), "hipMemcpy H2D")

    def fwd():
        pkg.grover_phase_forward(p, bufs["phi"].value, bufs["theta"].value, bufs["loss"].value)

    def bwd():
        pkg.grover_phase_backward(p, bufs["dloss"].value, bufs["dphi"].value, bufs["dtheta"].value)

    def measure(form):
        pkg.grover_phase_set_form(p, form)
        fwd()
        bwd()
        pkg.grover_phase_sync(p)
        f_ms, b_ms = [], []
        for _ in range(runs):
            e = [hip.event() for _ in range(3)]
            hip.lib.hipEventRecord(e[0], stream)
            fwd()
            hip.lib.hipEventRecord(e[1], stream)
            bwd()
            hip.lib.hipEventRecord(e[2], stream)
            f_ms.append(hip.elapsed_ms(e[0], e[1]))
            b_ms.append(hip.elapsed_ms(e[1], e[2]))
            pkg.grover_phase_sync(p)
        fm, bm = sorted(f_ms)[len(f_ms) // 2], sorted(b_ms)[len(b_ms) // 2]
        # results of one more pair
        fwd()
        pkg.grover_phase_sync(p)
        loss = np.empty(B)
        hip.ok(hip.lib.hipMemcpy(ctypes.c_void_p(loss.ctypes.data), bufs["loss"], B * 8, 2), "hipMemcpy D2H")
        bwd()
        pkg.grover_phase_sync(p)
        dphi, dtheta = np.empty((B, K)), np.empty((B, K))
        hip.ok(hip.lib.hipMemcpy(ctypes.c_void_p(dphi.ctypes.data), bufs["dphi"], nbytes, 2), "hipMemcpy D2H")
        hip.ok(hip.lib.hipMemcpy(ctypes.c_void_p(dtheta.ctypes.data), bufs["dtheta"], nbytes, 2), "hipMemcpy D2H")
        return fm, bm, loss, dphi, dtheta

    runs_by_form = {"held": measure(g.GROVER_PHASE_FORM_HELD), "streamed": measure(g.GROVER_PHASE_FORM_STREAMED)}
    pkg.grover_phase_destroy(p)
    for b_ in bufs.values():
        hip.lib.hipFree(b_)
    orc = oracle.default()
    want = {}
    for b in (0, B - 1):
        want[b] = (orc.phase_loss(orc.phase_search(w.n, marks, phi[b], theta[b]), marks),
                   orc.phase_grad_adjoint(w.n, marks, phi[b], theta[b]))
    plain = time_form(pkg, hip, stream, w.n, "c128", "two_pass", marks, 300, 48, 0)
    updates = float(B) * K * N
    # memory traffic per run: streamed, every step reads and writes the state (and the adjoint state);
    # held, only the checkpoints and the final states
    traffic = {"streamed": (B * (8.0 * N + 16.0 * N * K + 8.0 * N * nck), B * (8.0 * N + 32.0 * N * K)),
               "held": (B * (8.0 * N * nck + 8.0 * N), B * (8.0 * N + 8.0 * N * nck + 8.0 * N))}
    forms = {}
    for form, (fm, bm, loss, dphi, dtheta) in runs_by_form.items():
        fb, bb = traffic[form]
        acc = []
        for b in (0, B - 1):
            want_loss, (wphi, wtheta) = want[b]
            acc.append({"schedule": b, "loss": loss[b], "loss_abs_err": abs(loss[b] - want_loss),
                        "grad_max_abs_err": float(max(np.max(np.abs(dphi[b] - wphi)),
                                                      np.max(np.abs(dtheta[b] - wtheta)))),
                        "grad_max_abs": float(max(np.max(np.abs(wphi)), np.max(np.abs(wtheta))))})
        forms[form] = {
            "teams": {"forward": held_teams[0], "adjoint": held_teams[1]} if form == "held" else team,
            "forward_ms": round(fm, 3), "adjoint_ms": round(bm, 3),
            "forward_amplitude_updates_per_s": updates / (fm / 1e3),
            "adjoint_amplitude_steps_per_s": updates / (bm / 1e3),
            "forward_memory_bytes": fb, "adjoint_memory_bytes": bb,
            "forward_memory_gbs": round(fb / (fm / 1e3) / 1e9, 1),
            "adjoint_memory_gbs": round(bb / (bm / 1e3) / 1e9, 1),
            "forward_vs_plain_fp64": (updates / (fm / 1e3)) / plain["amplitude_updates_per_s"],
            "forward_plus_adjoint_vs_plain_fp64_forward_only":
                (updates / ((fm + bm) / 1e3)) / plain["amplitude_updates_per_s"],
            "accuracy_vs_fp64_oracle": acc}
    s_fm, s_bm = forms["streamed"]["forward_ms"], forms["streamed"]["adjoint_ms"]
    sf, sb = traffic["streamed"]
    print(json.dumps({
        "sweep": "adjoint", "workload": w.name, "n": w.n, "m": w.m, "K": K, "batch": B, "storage": "complex64",
        "arithmetic": "f64", "checkpoint_every": every, "checkpoints_per_schedule": nck, "grid": grid,
        "default_form": "held", "forward_ms": forms["held"]["forward_ms"], "adjoint_ms": forms["held"]["adjoint_ms"],
        "streamed_forward_frac_of_hbm_peak": round(sf / (s_fm / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "streamed_adjoint_frac_of_hbm_peak": round(sb / (s_bm / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "plain_fp64_amplitude_updates_per_s": plain["amplitude_updates_per_s"],
        "forms": forms, "runs": runs}), flush=True)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=40)
    ap.add_argument("--cpu-all-iters", type=int, default=4,
                    help="iterations per process of the all-core CPU baseline (one oracle process per host core)")
    ap.add_argument("--cpu-worker", type=str, default=None, help=argparse.SUPPRESS)
    ap.add_argument("--sweep", choices=["table1", "precision", "batch", "adjoint", "update", "scaling"], default=None,
                    help="instead of the headline line, print one JSON line per point of a sweep")
    args = ap.parse_args()
    if args.cpu_worker:
        return cpu_worker(args.cpu_worker)
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the state of a search is not sharded across GPUs; use --gpus 1",
              file=sys.stderr)
        return 2

    import paper_2005_04635_amd as pkg

    pkg.load()
    hip = Hip()
    hip.ok(hip.lib.hipSetDevice(0), "hipSetDevice")
    stream = ctypes.c_void_p()
    hip.ok(hip.lib.hipStreamCreate(ctypes.byref(stream)), "hipStreamCreate")
    try:
        return run(args, pkg, hip, stream)
    finally:
        hip.close(stream)


def run(args, pkg, hip, stream) -> int:
    import numpy as np

    import workloads

    if args.sweep == "table1":
        sweep_table1(pkg, hip, stream)
        return 0
    if args.sweep == "precision":
        sweep_precision(pkg, hip, stream)
        return 0
    if args.sweep == "batch":
        sweep_batch(pkg, hip, stream, max(args.steps, 1))
        return 0
    if args.sweep == "adjoint":
        sweep_adjoint(pkg, hip, stream, max(args.steps, 1))
        return 0
    if args.sweep == "update":
        sweep_update(pkg, hip, stream, max(args.steps, 3))
        return 0
    if args.sweep == "scaling":
        sweep_scaling(pkg, hip, stream, max(args.steps, 3))
        return 0
    w = workloads.HASH_N28
    N = 1 << w.n
    log(f"[bench] device {hip.name()}; workload {w.name}")
    cfg, _ = make_config(pkg, w.n, w.dtype, hash_seed=w.hash_seed, hash_bits=w.hash_bits, m=w.m, form="fused")
    ctx = pkg.grover_init(cfg, stream.value, 0, 0)
    marks = pkg.grover_marked(ctx, w.m)
    grid, block = pkg.grover_query(ctx, 1), pkg.grover_query(ctx, 2)
    # measurement uniforms, resident on the device before timing
    u = np.ascontiguousarray(workloads.uniforms_u53(w.shot_seed, w.shots))
    u_dev = hip.malloc(u.nbytes)
    out_dev = hip.malloc(w.shots * 8)
    hip.ok(hip.lib.hipMemcpy(u_dev, ctypes.c_void_p(u.ctypes.data), u.nbytes, 1), "hipMemcpy H2D")
    e_it = [(hip.event(), hip.event()) for _ in range(args.steps)]
    norms = []

    def step(i_timed):
        pkg.grover_reset(ctx)
        if i_timed is not None:
            hip.lib.hipEventRecord(e_it[i_timed][0], stream)
        pkg.grover_iterate(ctx, w.iterations)
        if i_timed is not None:
            hip.lib.hipEventRecord(e_it[i_timed][1], stream)
        norms.append(pkg.grover_norm(ctx))
        pkg.grover_sample_u53(ctx, u_dev.value, True, w.shots, out_dev.value, True)

    for i in range(args.warmup):
        step(None)
        pkg.grover_sync(ctx)
        log(f"[bench] warmup step {i + 1}/{args.warmup} done")
    hip.ok(hip.lib.hipDeviceSynchronize(), "hipDeviceSynchronize")
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i)
        log(f"[bench] step {i + 1}/{args.steps} enqueued")
    hip.ok(hip.lib.hipDeviceSynchronize(), "hipDeviceSynchronize")
    t1 = time.perf_counter()
    pkg.grover_sync(ctx)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    it_ms = [hip.elapsed_ms(a, b) for a, b in e_it]
    it_ms_mean = sum(it_ms) / len(it_ms)
    shots = np.empty(w.shots, dtype=np.uint64)
    hip.ok(hip.lib.hipMemcpy(ctypes.c_void_p(shots.ctypes.data), out_dev, shots.nbytes, 2), "hipMemcpy D2H")
    marked_frac = float(np.isin(shots, marks).mean())
    log(f"[bench] {ms_per_step:.1f} ms/step, iterate kernel {it_ms_mean:.1f} ms, norm {norms[-1]:.9f}, "
        f"marked shot fraction {marked_frac:.6f}")

    alg_bytes = 16.0 * N * w.iterations + 8.0 * N
    achieved = alg_bytes / (it_ms_mean / 1e3) / 1e9
    traffic = committed_traffic()
    # the measured ceiling of the fused kernel's access pattern: the bandwidth probe (same grid, tiles and
    # nontemporal accesses, no arithmetic) over a buffer of the state's size, in-place read + write and
    # read-only; and the runtime's own device-to-device copy of the same bytes, for context
    state_ptr, state_bytes = pkg.grover_state_device(ctx)
    dst = hip.malloc(state_bytes)
    hip.ok(hip.lib.hipMemcpy(dst, ctypes.c_void_p(state_ptr), state_bytes, 3), "hipMemcpy D2D")
    probe_passes = 20
    g = pkg.grover
    probe = {}
    pkg.grover_stream_probe(stream.value, dst.value, state_bytes, 2)  # warm
    for name, mode, rw in (("in_place", 0, 2.0), ("in_place_launch_per_pass", g.GROVER_PROBE_LAUNCH_PER_PASS, 2.0),
                           ("in_place_narrow", g.GROVER_PROBE_NARROW, 2.0),
                           ("read_only", g.GROVER_PROBE_READ_ONLY, 1.0),
                           ("read_only_launch_per_pass", g.GROVER_PROBE_READ_ONLY | g.GROVER_PROBE_LAUNCH_PER_PASS,
                            1.0)):
        ms_p = pkg.grover_stream_probe(stream.value, dst.value, state_bytes, probe_passes, mode)
        probe[name] = round(rw * state_bytes * probe_passes / (ms_p / 1e3) / 1e9, 1)
    ceiling_gbs = max(probe["in_place"], probe["in_place_launch_per_pass"])
    log(f"[bench] probe GB/s: {probe}")
    c0, c1 = hip.event(), hip.event()
    hip.lib.hipMemcpyAsync(dst, ctypes.c_void_p(state_ptr), state_bytes, 3, stream)
    hip.lib.hipEventRecord(c0, stream)
    for _ in range(5):
        hip.lib.hipMemcpyAsync(dst, ctypes.c_void_p(state_ptr), state_bytes, 3, stream)
    hip.lib.hipEventRecord(c1, stream)
    copy_gbs = 5 * 2 * state_bytes / (hip.elapsed_ms(c0, c1) / 1e3) / 1e9
    hip.destroy_events(c0, c1)
    hip.lib.hipFree(dst)
    hip.lib.hipFree(u_dev)
    hip.lib.hipFree(out_dev)
    pkg.grover_destroy(ctx)

    forms = None
    if not args.no_forms:
        log("[bench] timing the plain binary64 comparator and the other forms")
        forms = [
            time_form(pkg, hip, stream, w.n, "c128", "two_pass", marks, 200, 48, 0),
            time_form(pkg, hip, stream, w.n, "c128", "fused", marks, 400, 32, 16),
            time_form(pkg, hip, stream, w.n, "c64", "two_pass", marks, 400, 24, 0),
        ]

    cpu = None
    if not args.no_cpu_baseline:
        log(f"[bench] CPU oracle baseline: {args.cpu_iters} iterations at n={w.n}, one thread")
        cpu = cpu_baseline(w, marks, args.cpu_iters)
        log(f"[bench] CPU oracle baseline on all host cores: {args.cpu_all_iters} iterations per process")
        cpu = cpu_baseline_all_cores(w, args.cpu_all_iters, cpu)

    value = N * w.iterations / (ms_per_step / 1e3)
    plain = forms[0]["amplitude_updates_per_s"] if forms else None
    line = {
        "metric": "amplitude-updates/s per Grover iteration, n=28 (and % of peak HBM GB/s), vs plain FP64",
        "value": value,
        "unit": "amplitude-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "m": w.m, "marks": "hash predicate, 25 zero bits",
                   "iterations": w.iterations, "shots": w.shots, "storage": "complex64",
                   "accumulate_and_update": "f64", "form": "fused persistent cooperative", "grid": grid,
                   "block": block, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "frac_basis": "algorithmic bytes (16 B per amplitude-update + 8 B per amplitude for the "
                                   "prologue sum) per launch / kernel time; includes the bytes the kernel keeps on "
                                   "chip (6 of each workgroup's tiles) and those the memory-side cache serves "
                                   "(272 MiB of each pass)",
                     "traffic": traffic, "kernel": "fused_iterate_kernel<C64>",
                     "kernel_ms_per_launch": round(it_ms_mean, 3),
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "counter_gbs": round(traffic / (it_ms_mean / 1e3) / 1e9, 1) if traffic else None,
                     "counter_frac": round(traffic / (it_ms_mean / 1e3) / 1e9 / HBM_PEAK_GBS, 4) if traffic else None,
                     "ceiling_gbs": ceiling_gbs, "frac_of_ceiling": round(achieved / ceiling_gbs, 4),
                     "ceiling": "bandwidth probe in the same run: the fused kernel's grid, workgroup shape, tiles "
                                "and nontemporal 16-byte loads and stores without its arithmetic over 2 GiB, "
                                f"{probe_passes} passes; ceiling_gbs = the faster in-place form of that shape "
                                "(in_place_narrow: 1024 threads of 4 vectors, for context)",
                     "probe_gbs": probe},
        "runtime_copy_gbs": round(copy_gbs, 1),
        "vs_plain_fp64": (value / plain) if plain else None,
        "forms": forms,
        "cpu_baseline": cpu,
        "norm": norms[-1],
        "marked_shot_fraction": marked_frac,
        "paper_context_updates_per_s": {"value": PAPER_CPU_N20_UPDATES_PER_S,
                                        "what": "paper Table 1, proposed simulator, n=20, Intel i3-5005U, 1 thread"},
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
