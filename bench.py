"""Benchmark of the Helmholtz solve on one MI355X.

A step is one pass of the hot path on the 160x96x80-element box cavity at
250 Hz (1,264,977 unknowns, 33.5M nonzeros, complex128): form A(k) on the
device (set_frequency) and solve A p = f with right-Jacobi BiCGStab to a
true relative residual of 1e-8.  The inputs (mesh, admittances, forcing)
are assembled and resident in HBM before the timed region.

Printed as one JSON line: the solve time (value, s), the sparse product's
achieved algorithmic bandwidth against the 8 TB/s HBM peak (roofline), the
oracle's CPU time on a bounded sample (cpu_baseline), and secondary numbers
(GMRES(50), mixed precision, the batched frequency sweep when available).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
# HBM bytes per launch of the complex128 product on this workload, from the
# FETCH_SIZE / WRITE_SIZE passes recorded in profiles/ (calibrated against a
# 1 GiB device copy); set to None whenever the kernel changes until re-measured.
MEASURED_TRAFFIC = {"k_spmv<double>": 717.9e6}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def spmv_bytes(n, nnz):
    # values (16 B) + column index (4 B) per nonzero, row/slice pointers,
    # x read once and y written once (16 B each)
    return 20 * nnz + 4 * (n + 1) + 32 * n


def cpu_baseline(wl, gpu_iters, iters):
    """The oracle's BiCGStab (complex128 CSR, SciPy matvec, one thread) timed
    on `iters` iterations of the same system, scaled to the GPU's count."""
    from oracle import helmholtz as H, krylov
    import workloads as W
    t = time.perf_counter()
    S = H.System(wl["mesh"], wl["beta"])
    A = S.operator(W.wavenumber(wl["freqs"][0]))
    f = S.load(wl["g"])
    log(f"cpu baseline: oracle assembly {time.perf_counter() - t:.1f}s")
    t = time.perf_counter()
    r = krylov.bicgstab(A, f, tol=1e-8, max_iters=iters)
    dt = time.perf_counter() - t
    per_iter = dt / max(r.iters, 1)
    return {"value": per_iter * gpu_iters, "unit": "s", "cores": 1, "kind": "oracle",
            "host_cpus": os.cpu_count(),
            "sample": f"{r.iters} BiCGStab iterations of the same system timed ({dt:.1f} s, "
                      f"{per_iter * 1e3:.1f} ms/iteration), scaled to the GPU's {gpu_iters} iterations"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-iters", type=int, default=40)
    ap.add_argument("--no-extra", action="store_true", help="only the headline solve and the roofline")
    ap.add_argument("--spmv-reps", type=int, default=200)
    ap.add_argument("--spmv-only", action="store_true",
                    help="skip the solves (hardware-counter runs of the product kernel)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a 1 GiB device copy (reference for the traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU sharding "
              "of this solver is a design, not a built path", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_2112_00087_amd import Helmholtz

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    wl = W.workload(1)
    freq = float(wl["freqs"][0])
    t = time.perf_counter()
    model = Helmholtz(wl["mesh"], wl["beta"])
    sizes = model.sizes()
    log(f"assembled {wl['name']}: n={sizes['n_nodes']} nnz={sizes['nnz']} in {time.perf_counter() - t:.1f}s")
    g = torch.as_tensor(wl["g"], device="cuda")
    f = model.load(g)
    opts = dict(method="bicgstab", tol=1e-8, max_matvec=100000)

    def step():
        model.set_frequency(freq)
        return model.solve(f, **opts)

    if args.calib_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.spmv_only:
        model.set_frequency(freq)
        args.steps = 0
    for _ in range(args.warmup if not args.spmv_only else 0):
        _, info = step()
        log(f"warmup: {info}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [dict(iters=0, relres_true=None)]
    for _ in range(args.steps):
        _, info = step()
        infos.append(info)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(args.steps, 1)
    log(f"timed: {dt:.4f} s/solve, {infos[-1]}")

    n, nnz = sizes["n_nodes"], sizes["nnz"]
    ms = model.time_spmv(args.spmv_reps, "fp64")
    byts = spmv_bytes(n, nnz)
    gbs = byts / (ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "traffic": MEASURED_TRAFFIC.get("k_spmv<double>"),
            "kernel": "k_spmv<double> (complex128 sliced-ELL product)",
            "avg_kernel_ms": ms, "algorithmic_bytes": byts}
    log(f"spmv: {ms * 1e3:.1f} us, {gbs:.0f} GB/s ({100 * gbs / HBM_PEAK_GBS:.1f}% of HBM peak)")

    extra = {}
    if not args.no_extra and not args.spmv_only:
        ms32 = model.time_spmv(args.spmv_reps, "mixed")
        b32 = 12 * nnz + 4 * (n + 1) + 16 * n
        extra["spmv_c64_GBs"] = b32 / (ms32 * 1e-3) / 1e9
        for label, o in (("gmres50", dict(method="gmres", restart=50)),
                         ("bicgstab_mixed", dict(method="bicgstab", precision="mixed")),
                         ("gmres50_mixed", dict(method="gmres", restart=50, precision="mixed"))):
            model.set_frequency(freq)
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, inf = model.solve(f, tol=1e-8, max_matvec=30000, **o)
            torch.cuda.synchronize()
            extra[label] = {"s": time.perf_counter() - t, "status": inf["status"], "iters": inf["iters"],
                            "matvecs": inf["matvecs"], "inner_matvecs": inf["inner_matvecs"],
                            "relres_true": inf["relres_true"]}
            log(f"{label}: {extra[label]}")

    cpu = None
    if not args.no_cpu and not args.spmv_only:
        cpu = cpu_baseline(wl, infos[-1]["iters"], args.cpu_iters)
        log(f"cpu baseline: {cpu}")

    out = {
        "metric": "solve time to relres 1e-8 (s) + SpMV HBM GB/s; mixed-batched vs FP64 sweep speedup",
        "value": dt, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": False, "scaling": "strong",
        "vs_baseline": None, "dtype": "complex128", "data": "synthetic",
        "config": {"workload": wl["name"], "n_nodes": n, "nnz": nnz, "freq_hz": freq,
                   "solver": "bicgstab, right Jacobi", "tol": 1e-8,
                   "iters": infos[-1]["iters"], "relres_true": infos[-1]["relres_true"]},
        "spmv_GBs": gbs,
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
