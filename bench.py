"""Benchmark of the Grover hot path on one MI355X: amplitude-updates/s and fraction of peak HBM bandwidth
per Grover iteration at n = 28, against the plain binary64 form.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-forms]

Workload (synthetic by construction; the paper uses no dataset): the single large instance, n = 28
(2^28 complex64 amplitudes, 2 GiB), M = 8 marked indices defined by the hash predicate
(SplitMix64_i(seed) mod 2^25 == 0), floor(pi/4 sqrt(N/M)) = 4549 iterations, 10^6 measurement shots.

One step is one pass of the whole hot path on inputs already resident in HBM: the uniform superposition
is written, 4549 fused iterations run (one persistent cooperative kernel), the norm is taken, and 10^6
shots are sampled with device-resident uniforms.  `value` = N * 4549 / (wall time of one step).

Printed JSON line (last line of stdout):
  roofline      the fused iterate kernel: algorithmic bytes per launch (16 B per amplitude-update plus the
                8 B-per-amplitude prologue read) / its mean duration measured with HIP events on the
                stream it runs on, against MI355X's 8 TB/s; `traffic` is the counter-measured HBM bytes per
                launch from the committed rocprofv3 summary (null when the kernel source changed since)
  forms         the plain binary64 comparator (complex128, oracle / sum / update kernels per iteration)
                and the fused complex128 form, timed on a bounded number of iterations
  cpu_baseline  the CPU oracle (single thread, binary64) on a bounded sample of the same workload
"""
from __future__ import annotations

import argparse
import hashlib
import json
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


def time_form(pkg, torch, n, dtype, form, marks, iters, bytes_per_update, prologue_bytes):
    """Iterations/s of one form on a resident state, HIP events on its stream."""
    g = pkg.Grover(n, dtype, marks=marks, form=form)
    g.iterate(2)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g.iterate(iters)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    N = 1 << n
    ups = N * iters / (ms / 1e3)
    gbs = (bytes_per_update * N * iters + prologue_bytes * N) / (ms / 1e3) / 1e9
    g.close()
    return {"form": form, "storage": dtype, "iterations": iters, "ms": round(ms, 3),
            "amplitude_updates_per_s": ups, "algorithmic_gbs": round(gbs, 1),
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


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=8)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the Grover iteration's state is not sharded across GPUs in "
              "this build (see DESIGN.md for how it would shard); use --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2005_04635_amd as pkg
    import workloads

    w = workloads.HASH_N28
    N = 1 << w.n
    torch.cuda.set_device(0)
    log(f"[bench] device {torch.cuda.get_device_name(0)}; workload {w.name}")
    g = pkg.Grover(w.n, w.dtype, hash_seed=w.hash_seed, hash_bits=w.hash_bits, m=w.m, form="fused")
    marks = g.marked()
    grid, block = g.query(pkg.grover.Q_GRID), g.query(pkg.grover.Q_BLOCK)
    u_dev = torch.from_numpy(workloads.uniforms_u53(w.shot_seed, w.shots).astype(np.int64)).cuda()
    out_dev = None
    e_it0 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    e_it1 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    norms = []

    def step(i_timed):
        nonlocal out_dev
        g.reset()
        if i_timed is not None:
            e_it0[i_timed].record()
        g.iterate(w.iterations)
        if i_timed is not None:
            e_it1[i_timed].record()
        norms.append(g.norm())
        out_dev = g.sample(w.shots, u53=u_dev, device_out=True)

    for i in range(args.warmup):
        step(None)
        torch.cuda.synchronize()
        log(f"[bench] warmup step {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i)
        log(f"[bench] step {i + 1}/{args.steps} enqueued")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    it_ms = [a.elapsed_time(b) for a, b in zip(e_it0, e_it1)]
    it_ms_mean = sum(it_ms) / len(it_ms)
    shots = out_dev.cpu().numpy().astype(np.uint64)
    marked_frac = float(np.isin(shots, marks).mean())
    log(f"[bench] {ms_per_step:.1f} ms/step, iterate kernel {it_ms_mean:.1f} ms, norm {norms[-1]:.9f}, "
        f"marked shot fraction {marked_frac:.6f}")

    alg_bytes = 16.0 * N * w.iterations + 8.0 * N
    achieved = alg_bytes / (it_ms_mean / 1e3) / 1e9
    traffic = committed_traffic()
    # practical ceiling: a device-to-device copy of the same 2 GiB (read + write)
    src = g.state.view(torch.float32)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(5):
        dst.copy_(src)
    c1.record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * src.numel() * 4 / (c0.elapsed_time(c1) / 1e3) / 1e9
    del dst
    g.close()
    del g

    forms = None
    if not args.no_forms:
        log("[bench] timing the plain binary64 comparator and the fused complex128 form")
        forms = [
            time_form(pkg, torch, w.n, "c128", "two_pass", marks, 200, 48, 0),
            time_form(pkg, torch, w.n, "c128", "fused", marks, 400, 32, 16),
            time_form(pkg, torch, w.n, "c64", "two_pass", marks, 400, 24, 0),
        ]
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        log(f"[bench] CPU oracle baseline: {args.cpu_iters} iterations at n={w.n}")
        cpu = cpu_baseline(w, marks, args.cpu_iters)

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
                     "traffic": traffic, "kernel": "fused_iterate_kernel<C64>",
                     "kernel_ms_per_launch": round(it_ms_mean, 3),
                     "algorithmic_bytes_per_launch": alg_bytes},
        "copy_ceiling_gbs": round(copy_gbs, 1),
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
