"""Benchmark of the Helmholtz solve on one MI355X.

A step is one pass of the hot path on the 160x96x80-element box cavity at
250 Hz (1,264,977 unknowns, 33.5M nonzeros, complex128): form A(k) on the
device (set_frequency) and solve A p = f with right-Jacobi BiCGStab to a
true relative residual of 1e-8.  The inputs (mesh, admittances, forcing)
are assembled and resident in HBM before the timed region.

Printed as one JSON line: the solve time (value, s), the sparse product's
achieved algorithmic bandwidth against the 8 TB/s HBM peak (roofline), the
oracle's CPU time on a bounded sample (cpu_baseline: one thread and all host
cores, plus direct solves), and secondary numbers (GMRES(50), the paper's
other Krylov methods, mixed precision, the batched 64-frequency sweep
against 64 per-frequency FP64 solves with the errors of sampled columns
against the oracle, the 24-subdomain Schwarz solve and the 16-frequency
adjoint gradient).  Two CPU-side processes (the oracle's direct solve of the
80x48x40 mesh and its reference solutions of two sweep columns) start before
the GPU is touched and run beside the GPU legs.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
# HBM bytes per launch of the FP64 product on this workload, per storage form,
# from the FETCH_SIZE / WRITE_SIZE passes recorded in profiles/ (calibrated
# against a 1 GiB device copy); None until measured for the current kernel.
MEASURED_TRAFFIC = {"stencil": 350.9e6, "split": None, "complex": 732.8e6}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def best_solve(t_bicgstab, extra):
    """Fastest converged solve of the headline system among the methods run
    (BiCGStab is the value; the paper's other Krylov methods are extras)."""
    best = {"method": "bicgstab", "s": t_bicgstab}
    for label, v in extra.items():
        if isinstance(v, dict) and v.get("status") == 0 and "s" in v and v["s"] < best["s"]:
            best = {"method": label, "s": v["s"], "matvecs": v.get("matvecs"),
                    "inner_matvecs": v.get("inner_matvecs"), "relres_true": v.get("relres_true")}
    return best


def host_cores():
    """Cores this process may run on, capped at a one-GPU machine's share (16)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(wl, gpu_iters, iters, side=None):
    """The oracle's BiCGStab (complex128 CSR, SciPy product) timed on `iters`
    iterations of the same system, scaled to the GPU's count: on one thread,
    and on all host cores (the product cut into row blocks, one per thread;
    bitwise the same iterates).  Plus the oracle's direct solves: SuperLU on
    the 20x12x10 workload here, and the 80x48x40 sweep mesh from the CPU-side
    process that ran beside the GPU work (`side`)."""
    from oracle import direct, helmholtz as H, krylov
    from oracle.parallel import RowBlockOperator
    import workloads as W
    t = time.perf_counter()
    S = H.System(wl["mesh"], wl["beta"])
    A = S.operator(W.wavenumber(wl["freqs"][0])).tocsr()
    f = S.load(wl["g"])
    log(f"cpu baseline: oracle assembly {time.perf_counter() - t:.1f}s")
    t = time.perf_counter()
    r = krylov.bicgstab(A, f, tol=1e-8, max_iters=iters)
    dt1 = time.perf_counter() - t
    per1 = dt1 / max(r.iters, 1)
    cores = host_cores()
    B = RowBlockOperator(A, cores)
    t = time.perf_counter()
    rm = krylov.bicgstab(B, f, tol=1e-8, max_iters=iters)
    dtm = time.perf_counter() - t
    B.close()
    perm = dtm / max(rm.iters, 1)
    out = {"value": perm * gpu_iters, "unit": "s", "cores": cores, "kind": "oracle",
           "host_cpus": os.cpu_count(),
           "sample": f"{r.iters} BiCGStab iterations of the same system timed on {cores} threads "
                     f"({dtm:.1f} s, {perm * 1e3:.1f} ms/iteration; product in row blocks) and on 1 thread "
                     f"({dt1:.1f} s, {per1 * 1e3:.1f} ms/iteration), scaled to the GPU's {gpu_iters} iterations",
           "one_thread": {"value": per1 * gpu_iters, "unit": "s", "cores": 1}}
    # direct solve of the small workload (oracle SuperLU, one thread)
    w0 = W.workload(0)
    S0 = H.System(w0["mesh"], w0["beta"])
    A0 = S0.operator(W.wavenumber(w0["freqs"][0]))
    f0 = S0.load(w0["g"])
    t = time.perf_counter()
    x0 = direct.SparseLU(A0).solve(f0)
    out["direct_20x12x10_s"] = time.perf_counter() - t
    out["direct_20x12x10_relres"] = H.relres(A0, x0, f0)
    if side:
        out.update({k: v for k, v in side.items() if k.startswith("direct_") or k.startswith("oracle_sweep")})
    return out


def cpu_side_direct(outdir):
    """CPU-side process: the oracle's SuperLU solve (minimum-degree column
    ordering on the symmetric pattern, one thread) of the 80x48x40 sweep
    mesh at 250 Hz, timed."""
    from oracle import direct, helmholtz as H
    import workloads as W
    wl = W.workload(2)
    S = H.System(wl["mesh"], wl["beta"])
    A = S.operator(W.wavenumber(250.0))
    f = S.load(wl["g"])
    t = time.perf_counter()
    lu = direct.SparseLU(A, ordering="MMD_AT_PLUS_A")
    x = lu.solve(f)
    dt = time.perf_counter() - t
    res = {"direct_80x48x40_s": dt, "direct_80x48x40_relres": H.relres(A, x, f),
           "direct_80x48x40_ordering": "MMD_AT_PLUS_A"}
    with open(os.path.join(outdir, "direct.json"), "w") as fh:
        json.dump(res, fh)


SWEEP_REF_COLS = (0, 63)


def cpu_side_sweep_ref(outdir):
    """CPU-side process: the oracle's TFQMR (complex128 CSR, one thread) to
    relres 1e-12 on sweep columns 0 and 63 (20 and 300 Hz), timed; the
    solutions are the FP64 references the sweep leg's errors are stated
    against."""
    from oracle import helmholtz as H, krylov
    import workloads as W
    wl = W.workload(2)
    S = H.System(wl["mesh"], wl["beta"])
    f = S.load(wl["g"])
    res = {}
    for j in SWEEP_REF_COLS:
        A = S.operator(W.wavenumber(wl["freqs"][j])).tocsr()
        t = time.perf_counter()
        r = krylov.tfqmr(A, f, tol=1e-12, max_matvec=60000)
        res[f"oracle_sweep_col{j}"] = {"freq_hz": float(wl["freqs"][j]), "s": time.perf_counter() - t,
                                       "matvecs": r.matvecs, "relres": H.relres(A, r.x, f)}
        np.save(os.path.join(outdir, f"ref{j}.npy"), r.x)
    with open(os.path.join(outdir, "sweep_ref.json"), "w") as fh:
        json.dump(res, fh)


def start_cpu_side(no_cpu):
    """Starts the CPU-side processes before this process touches the GPU
    (they run on other host cores while the GPU legs run)."""
    import subprocess
    import tempfile
    if no_cpu:
        return None
    outdir = tempfile.mkdtemp(prefix="hz_bench_cpu_")
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-side", kind, outdir],
                              env=env, stdout=subprocess.DEVNULL, stderr=subprocess.PIPE)
             for kind in ("direct", "sweep-ref")]
    return {"dir": outdir, "procs": procs, "t0": time.perf_counter()}


def collect_cpu_side(side, wait_s):
    """Results of the CPU-side processes; a process still running after
    wait_s more seconds is stopped and its result reported as missing."""
    if side is None:
        return {}
    out = {}
    deadline = time.perf_counter() + wait_s
    for p in side["procs"]:
        try:
            p.wait(timeout=max(1.0, deadline - time.perf_counter()))
        except Exception:
            p.kill()
            p.wait()
    for name in ("direct.json", "sweep_ref.json"):
        path = os.path.join(side["dir"], name)
        if os.path.exists(path):
            with open(path) as fh:
                out.update(json.load(fh))
        else:
            out[f"missing_{name}"] = f"not finished within the bench's wait ({wait_s:.0f} s after the GPU legs)"
    out["refs"] = {j: os.path.join(side["dir"], f"ref{j}.npy") for j in SWEEP_REF_COLS
                   if os.path.exists(os.path.join(side["dir"], f"ref{j}.npy"))}
    log(f"cpu side: {({k: v for k, v in out.items() if k != 'refs'})}")
    return out


def sweep_leg(log_fn, precisions=("fp64", "mixed"), method="tfqmr", ell=8):
    """Workload 2: 64 frequencies, 80x48x40.  T_A = 64 x (set_frequency + FP64
    solve); T_B[precision] = one batched sweep; all use the same Krylov method."""
    import torch
    import workloads as W
    from paper_2112_00087_amd import Helmholtz
    wl = W.workload(2)
    m = Helmholtz(wl["mesh"], wl["beta"])
    f = m.load(torch.as_tensor(wl["g"], device="cuda"))
    freqs = wl["freqs"]
    F = f[:, None].repeat(1, freqs.size).contiguous()
    opts = dict(method=method, tol=1e-8, max_matvec=200000, restart=ell if method == "bicgstabl" else 30)
    label = {"bicgstabl": f"bicgstab({ell})"}.get(method, method)
    # warm-up of every path the timed sweeps take (the product autotuner runs
    # once per column count a context meets, compaction included; graph
    # capture; allocations): one untimed pass of each batched sweep
    def mixed_opts(o):
        # complex64 inner solves to 1e-5: the fastest of the inner tolerances
        # 1e-3 .. 1e-6 (2.14, 1.68, 1.75, 1.16, 1.01, 1.08, 1.04 s for 1e-3,
        # 3e-4, 1e-4, 3e-5, 1e-5, 3e-6, 1e-6, each with every column
        # converged); the cap bounds a column that stalls
        return dict(o, max_matvec=20000, inner_tol=1e-5)

    for prec in precisions:
        m.solve_sweep(freqs, F, precision=prec, **(mixed_opts(opts) if prec == "mixed" else opts))
        log_fn(f"  sweep warm-up {prec} done")
    m.set_frequency(freqs[0])
    m.solve(f, **opts)
    torch.cuda.synchronize()
    t = time.perf_counter()
    a_ok, a_iters = 0, []
    for j, fr in enumerate(freqs):
        m.set_frequency(fr)
        _, inf = m.solve(f, **opts)
        a_ok += inf["status"] == 0
        a_iters.append(inf["iters"])
        if j % 16 == 15:
            log_fn(f"  sweep A: {j + 1}/64 frequencies, {time.perf_counter() - t:.1f}s")
    torch.cuda.synchronize()
    T_A = time.perf_counter() - t
    log_fn(f"sweep A (64 x FP64 {method}): {T_A:.2f}s, converged {a_ok}/64")
    out = {"workload": wl["name"], "method": label,
           "T_A_s": T_A, "converged_A": a_ok, "iters_A": a_iters}
    sols = {}
    for prec in precisions:
        t = time.perf_counter()
        o = mixed_opts(opts) if prec == "mixed" else opts
        Pb, infos = m.solve_sweep(freqs, F, precision=prec, **o)
        torch.cuda.synchronize()
        T_B = time.perf_counter() - t
        sols[prec] = Pb
        b_ok = sum(i["status"] == 0 for i in infos)
        worst = max(i["relres_true"] for i in infos)
        log_fn(f"sweep B (batched {prec} {method}): {T_B:.2f}s, converged {b_ok}/64, worst relres {worst:.2e}")
        out[f"batched_{prec}"] = {"T_B_s": T_B, "speedup": T_A / T_B, "converged": b_ok, "worst_relres": worst,
                                  "iters": [i["iters"] for i in infos]}
    if "fp64" in sols and "mixed" in sols:
        # per-column relative difference of the mixed solution from the FP64
        # batched one (both to relres 1e-8); the error of each against the
        # oracle is added on the sampled columns once the CPU side is done
        d = torch.linalg.norm(sols["mixed"] - sols["fp64"], dim=0) / torch.linalg.norm(sols["fp64"], dim=0)
        out["batched_mixed"]["reldiff_vs_fp64"] = [float(v) for v in d.cpu()]
        log_fn(f"mixed vs FP64 batched: max column relative difference {float(d.max()):.2e}")
    out["_columns"] = {prec: {j: sols[prec][:, j].cpu().numpy() for j in SWEEP_REF_COLS} for prec in sols}
    m.close()
    return out


def sweep_errors(sweep, side):
    """Relative errors of the sampled batched columns against the oracle's
    FP64 references (relres 1e-12) computed by the CPU-side process."""
    cols = sweep.pop("_columns", {})
    refs = (side or {}).get("refs", {})
    for prec, byj in cols.items():
        errs = {}
        for j, x in byj.items():
            if j in refs:
                ref = np.load(refs[j])
                errs[f"col{j}"] = float(np.linalg.norm(x - ref) / np.linalg.norm(ref))
        if errs:
            sweep[f"batched_{prec}"]["relerr_vs_oracle"] = errs
            log(f"sweep {prec}: relative error vs the oracle on sampled columns {errs}")


def spmm_leg(log_fn, reps=50):
    """The sweep's multi-vector product at workload 2 (80x48x40, 64
    columns), FP64 and complex64, timed with HIP events on the context's
    stream (hz_time_spmm), against the CSR algorithmic bytes."""
    import workloads as W
    from paper_2112_00087_amd import Helmholtz
    wl = W.workload(2)
    m = Helmholtz(wl["mesh"], wl["beta"])
    out = {"workload": wl["name"], "columns": int(wl["freqs"].size)}
    for prec in ("fp64", "mixed"):
        ms, b, v = m.time_spmm(wl["freqs"], reps, prec)
        gbs = b / (ms * 1e-3) / 1e9
        out[prec] = {"us": ms * 1e3, "bytes": b, "GBs": gbs, "frac": gbs / HBM_PEAK_GBS, "variant": v}
        log_fn(f"multi-vector product {prec}: {ms * 1e3:.1f} us, {b / 1e6:.1f} MB, {gbs:.0f} GB/s "
               f"({100 * gbs / HBM_PEAK_GBS:.1f}% of HBM peak), variant {v}")
    m.close()
    return out


def schwarz_leg(log_fn, max_matvec=300):
    """Workload 3: 24 subdomains on one GPU, interface GMRES(300) in complex128
    with batched local solves (FP64, and complex64 with FP64 refinement), next
    to global solves of the same system."""
    import torch
    import workloads as W
    from paper_2112_00087_amd import Helmholtz
    wl = W.workload(3)
    m = Helmholtz(wl["mesh"], wl["beta"], parts=wl["parts"])
    f = m.load(torch.as_tensor(wl["g"], device="cuda"))
    out = {"workload": wl["name"]}
    # one-sided optimised coefficient for the comparison (the default is the two-sided pair)
    from paper_2112_00087_amd import dd_alpha
    nx, ny, nz = wl["mesh"]["elems"]
    sp = [1.8 / nx, 1.2 / ny, 1.0 / nz]
    H = min(sp[d] * (wl["mesh"]["elems"][d] // wl["parts"][d]) for d in range(3))
    a1, _ = dd_alpha(W.wavenumber(wl["freqs"][0]), H, min(sp), sides=1)
    out["alpha_one_sided"] = [a1.real, a1.imag]
    loc = dict(dd_inner="bicgstabl", inner_restart=4)
    # complex128 local solves to 1e-12 (at 1e-10 their error stalls the
    # interface GMRES); the mixed refinement overshoots 1e-10 by itself
    runs = (("schwarz_two_sided_fp64", dict(loc, precision="fp64", inner_tol=1e-12)),
            ("schwarz_two_sided_mixed", dict(loc, precision="mixed", inner_tol=1e-10)),
            ("schwarz_one_sided_fp64", dict(loc, precision="fp64", inner_tol=1e-12, dd_alpha=a1)))
    for label, o in runs:
        m.set_frequency(wl["freqs"][0])
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, inf = m.solve(f, method="schwarz", tol=1e-8, restart=300, max_matvec=max_matvec, **o)
        torch.cuda.synchronize()
        out[label] = dict(s=time.perf_counter() - t, **inf)
        log_fn(f"{label}: {out[label]}")
    for label, o in (("global_bicgstab", dict(method="bicgstab")), ("global_bicgstabl4", dict(method="bicgstabl",
                                                                                            restart=4))):
        m.set_frequency(wl["freqs"][0])
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, inf = m.solve(f, tol=1e-8, max_matvec=200000, **o)
        torch.cuda.synchronize()
        out[label] = dict(s=time.perf_counter() - t, **inf)
        log_fn(f"{label} on the same system: {out[label]}")
    ms = m.time_spmv(50, "fp64", "complex")
    b = m.spmv_bytes("fp64", "complex")
    out["spmv_complex128_GBs"] = b / (ms * 1e-3) / 1e9
    log_fn(f"workload 3 complex128 product: {ms * 1e3:.1f} us, {out['spmv_complex128_GBs']:.0f} GB/s")
    m.close()
    return out


def adjoint_leg(log_fn):
    import torch
    import workloads as W
    from paper_2112_00087_amd import Helmholtz
    from paper_2112_00087_amd.autograd import HelmholtzEnergy
    wl = W.workload(4)
    m = Helmholtz(wl["mesh"], wl["beta"], wl["eta"])
    beta = torch.tensor(np.stack([wl["beta"].real, wl["beta"].imag], 1), dtype=torch.float64, device="cuda",
                        requires_grad=True)
    eta = torch.tensor(wl["eta"], dtype=torch.float64, device="cuda", requires_grad=True)
    rec = torch.as_tensor(wl["receivers"], device="cuda")
    g = torch.as_tensor(wl["g"], device="cuda")
    torch.cuda.synchronize()
    t = time.perf_counter()
    J = HelmholtzEnergy.apply(beta, eta, m, wl["freqs"], g, rec, dict(method="bicgstabl", restart=4, tol=1e-8,
                                                                      max_matvec=200000))
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t
    J.backward()
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t
    out = {"workload": wl["name"], "J": J.item(), "forward_s": t_fwd, "forward_backward_s": t_all,
           "grad_beta_norm": beta.grad.norm().item(), "grad_eta_norm": eta.grad.norm().item()}
    log_fn(f"adjoint: {out}")
    m.close()
    return out


def unstructured_leg(log_fn, layouts=(("given", 0), ("rcm", 0), ("rcm", 256)), solves=True, cfg=5):
    layouts = tuple(layouts)
    """Workload 5 (unstructured hexahedra) or 6 (unstructured P1
    tetrahedra), random node ids: the sparse product under each internal
    numbering (caller's order, reverse Cuthill-McKee, RCM + length sort of
    the 64-row slices), and solves."""
    import torch
    import workloads as W
    from paper_2112_00087_amd import Helmholtz
    wl = W.workload(cfg)
    freq = float(wl["freqs"][0])
    out = {"workload": wl["name"], "n_nodes": int(wl["mesh"]["n_nodes"]), "n_elems": int(wl["mesh"]["n_elems"])}
    g = torch.as_tensor(wl["g"], device="cuda")
    for order, sigma in layouts:
        t = time.perf_counter()
        m = Helmholtz(wl["mesh"], wl["beta"], order=order, sigma=sigma)
        t_asm = time.perf_counter() - t
        m.set_frequency(freq)
        lay = m.layout()
        nnz = m.sizes()["nnz"]
        r = {"assemble_s": t_asm, "nnz": nnz, "padding": lay["slots"] / nnz, "bandwidth": lay["bandwidth"],
             "n_imag": lay["n_imag"]}
        for prec, form in (("fp64", "solver"), ("fp64", "complex"), ("mixed", "solver")):
            ms = m.time_spmv(100, prec, form)
            b = m.spmv_bytes(prec, form)
            r[f"spmv_{prec}_{form}"] = {"us": ms * 1e3, "GBs": b / (ms * 1e-3) / 1e9, "bytes": b}
        f = m.load(g)
        want_solves = solves
        solves = (("bicgstab", dict(method="bicgstab")), ("tfqmr", dict(method="tfqmr")),
                  ("bicgstabl4", dict(method="bicgstabl", restart=4)))
        for label, o in solves if want_solves and (order, sigma) in (layouts[0], layouts[-1]) else ():
            m.set_frequency(freq)
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, inf = m.solve(f, tol=1e-8, max_matvec=60000, **o)
            torch.cuda.synchronize()
            r[label] = {"s": time.perf_counter() - t, "status": inf["status"], "iters": inf["iters"],
                        "matvecs": inf["matvecs"], "relres_true": inf["relres_true"]}
            log_fn(f"{wl['name']} {order}/{sigma} {label}: {r[label]}")
        key = f"{order}_sigma{sigma}"
        out[key] = r
        log_fn(f"{wl['name']} {key}: {r}")
        m.close()
    return out


FORM_ID = {"complex": 0, "split": 1, "stencil": 2}


def solver_form(model):
    """Storage form the solvers use on this context (matched by its bytes)."""
    from paper_2112_00087_amd import HzError
    b = model.spmv_bytes("fp64", "solver")
    for f in ("stencil", "split"):
        try:
            if model.spmv_bytes("fp64", f) == b:
                return f
        except HzError:
            pass
    return "complex"


def _calib_copy():
    """A 1 GiB device fill and copy of known traffic (reference for the
    hardware traffic counters)."""
    import torch
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def _copy_rate(total_bytes, reps=50):
    """A plain device copy moving about total_bytes (half read, half
    written), timed on torch's stream: the bandwidth a streaming kernel of
    that size reaches on this GPU, as context for the roofline fraction."""
    import torch
    half = max(1 << 20, int(total_bytes) // 2 // (1 << 20) * (1 << 20))
    src = torch.ones(half // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    gbs = 2 * half / (ms * 1e-3) / 1e9
    return {"bytes": 2 * half, "ms": ms, "GBs": gbs, "frac": gbs / HBM_PEAK_GBS}


def _unstructured_legs(args):
    return {W_NAMES.get(int(c), c): unstructured_leg(log, _layouts(args.un_layouts), not args.un_spmv_only, int(c))
            for c in args.un_workloads.split(",")}


W_NAMES = {5: "hexahedra", 6: "tetrahedra"}


def _layouts(spec):
    out = []
    for item in spec.split(","):
        order, sigma = item.split(":")
        out.append((order, int(sigma)))
    return out


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
    ap.add_argument("--no-sweep", action="store_true", help="skip the 64-frequency sweep comparison")
    ap.add_argument("--sweep-method", default="tfqmr", choices=["bicgstabl", "bicgstab", "gmres", "tfqmr"],
                    help="Krylov method of both sides of the sweep comparison")
    ap.add_argument("--sweep-l", type=int, default=8, help="l of BiCGStab(l) in the sweep comparison")
    ap.add_argument("--schwarz", action="store_true", help="(default) run the 24-subdomain Schwarz leg")
    ap.add_argument("--adjoint", action="store_true", help="(default) run the 16-frequency adjoint leg")
    ap.add_argument("--no-schwarz", action="store_true", help="skip the 24-subdomain Schwarz leg")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the 16-frequency adjoint leg")
    ap.add_argument("--cpu-side", nargs=2, metavar=("KIND", "DIR"), help=argparse.SUPPRESS)
    ap.add_argument("--cpu-wait", type=float, default=150.0,
                    help="seconds to wait after the GPU legs for the CPU-side direct solve")
    ap.add_argument("--extras", default="",
                    help="comma list of the extra solves to run (default: all), e.g. gmres50,tfqmr")
    ap.add_argument("--spmm-only", action="store_true",
                    help="only time the sweep's multi-vector product (hardware-counter runs)")
    ap.add_argument("--unstructured", action="store_true",
                    help="also run the unstructured-mesh leg (product per row numbering, solves)")
    ap.add_argument("--un-layouts", default="given:0,rcm:0,rcm:256",
                    help="row numberings of the unstructured leg, order:sigma,...; solves run on the "
                         "first and the last")
    ap.add_argument("--un-spmv-only", action="store_true", help="unstructured leg without the solves")
    ap.add_argument("--un-workloads", default="5,6", help="unstructured workloads: 5 hexahedra, 6 tetrahedra")
    ap.add_argument("--legs-only", action="store_true",
                    help="skip the headline solve: run only the sweep (unless --no-sweep), Schwarz and adjoint "
                         "legs that are asked for and print them as one JSON line")
    args = ap.parse_args()
    if args.cpu_side:
        kind, outdir = args.cpu_side
        (cpu_side_direct if kind == "direct" else cpu_side_sweep_ref)(outdir)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU sharding "
              "of this solver is a design, not a built path", file=sys.stderr)
        sys.exit(2)

    do_schwarz = not args.no_schwarz
    do_adjoint = not args.no_adjoint
    side = None
    if not args.legs_only and not args.spmv_only:
        side = start_cpu_side(args.no_cpu)

    import torch
    import workloads as W
    from paper_2112_00087_amd import Helmholtz

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    if args.spmm_only:
        if args.calib_copy:
            _calib_copy()
        print(json.dumps(spmm_leg(log, reps=args.spmv_reps)), flush=True)
        return
    if args.legs_only:
        if args.calib_copy:
            _calib_copy()
        legs = {}
        if not args.no_sweep:
            legs["sweep"] = sweep_leg(log, method=args.sweep_method, ell=args.sweep_l)
        if args.schwarz:
            legs["schwarz"] = schwarz_leg(log)
        if args.adjoint:
            legs["adjoint"] = adjoint_leg(log)
        if "sweep" in legs:
            legs["sweep"].pop("_columns", None)
        if args.unstructured:
            legs["unstructured"] = _unstructured_legs(args)
        print(json.dumps(legs), flush=True)
        return
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
        _calib_copy()
    if args.spmv_only:
        args.steps = 0
    # the product timings below need an operator even when no solve is timed
    model.set_frequency(freq)
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
    # the product in the form the solver ran (stencil on a box, split on other
    # meshes, complex when an absorption field makes every entry complex),
    # then the complex128 form for reference
    form = solver_form(model)
    ms = model.time_spmv(args.spmv_reps, "fp64", form)
    byts = model.spmv_bytes("fp64", form)
    gbs = byts / (ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "traffic": MEASURED_TRAFFIC.get(form),
            "kernel": f"k_spmv<double, {FORM_ID[form]}> ({form} form sliced-ELL product)",
            "avg_kernel_ms": ms, "algorithmic_bytes": byts}
    log(f"spmv ({form}): {ms * 1e3:.1f} us, {gbs:.0f} GB/s ({100 * gbs / HBM_PEAK_GBS:.1f}% of HBM peak)")
    solve_roof = None
    if args.steps > 0:
        # whole-solve roofline: per BiCGStab iteration two products plus 16
        # complex128 vector passes (k_p 4, k_v 1 beyond its product, k_s 3,
        # k_t 1, k_xr 7), over the iterations the timed solve took
        it = infos[-1]["iters"]
        per_it = 2 * byts + 16 * 16 * n
        solve_roof = {"bytes_per_iteration": per_it, "iterations": it,
                      "achieved": per_it * it / dt / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": per_it * it / dt / 1e9 / HBM_PEAK_GBS}
        log(f"solve roofline: {per_it / 1e6:.0f} MB per iteration, {solve_roof['achieved']:.0f} GB/s "
            f"({100 * solve_roof['frac']:.1f}% of HBM peak)")

    extra = {"device_copy": _copy_rate(byts)}
    log(f"device copy of {extra['device_copy']['bytes'] / 1e6:.0f} MB: {extra['device_copy']['ms'] * 1e3:.1f} us, "
        f"{extra['device_copy']['GBs']:.0f} GB/s")
    if form != "complex":
        msc = model.time_spmv(args.spmv_reps, "fp64", "complex")
        bc = model.spmv_bytes("fp64", "complex")
        extra["spmv_complex128"] = {"ms": msc, "bytes": bc, "GBs": bc / (msc * 1e-3) / 1e9,
                                    "frac": bc / (msc * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                    "traffic": MEASURED_TRAFFIC.get("complex")}
        log(f"spmv (complex): {msc * 1e3:.1f} us, {extra['spmv_complex128']['GBs']:.0f} GB/s")
    if not args.no_extra and not args.spmv_only:
        ms32 = model.time_spmv(args.spmv_reps, "mixed", form)
        b32 = model.spmv_bytes("mixed", form)
        extra["spmv_fp32_GBs"] = b32 / (ms32 * 1e-3) / 1e9
        wanted = set(x for x in args.extras.split(",") if x)
        for label, o in (("gmres50", dict(method="gmres", restart=50)),
                         ("bicgstabl2", dict(method="bicgstabl", restart=2)),
                         ("bicgstabl4", dict(method="bicgstabl", restart=4)),
                         ("bicgstabl8", dict(method="bicgstabl", restart=8)),
                         ("tfqmr", dict(method="tfqmr")),
                         ("tfqmr_mixed", dict(method="tfqmr", precision="mixed", inner_tol=1e-2)),
                         ("bicgstabl4_mixed", dict(method="bicgstabl", restart=4, precision="mixed", inner_tol=1e-2)),
                         ("bicgstab_mixed", dict(method="bicgstab", precision="mixed")),
                         ("gmres50_mixed", dict(method="gmres", restart=50, precision="mixed"))):
            if wanted and label not in wanted:
                continue
            model.set_frequency(freq)
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, inf = model.solve(f, tol=1e-8, max_matvec=30000, **o)
            torch.cuda.synchronize()
            extra[label] = {"s": time.perf_counter() - t, "status": inf["status"], "iters": inf["iters"],
                            "matvecs": inf["matvecs"], "inner_matvecs": inf["inner_matvecs"],
                            "relres_true": inf["relres_true"]}
            if label.startswith("gmres") and "mixed" not in label and inf["iters"] > 0:
                # bytes of an Arnoldi step in the three-pass CGS2 form: the
                # product, then j + (j + 3) + (j + 3) complex128 vector passes
                # (dots against v_0..v_{j-1}; update + second dots with w read
                # and written; update into v_{j+1}), j averaged over the cycle
                m = o["restart"]
                per_step = byts + (3 * (m - 1) / 2 + 6) * 16 * n
                us = extra[label]["s"] / inf["iters"] * 1e6
                extra[label].update(us_per_step=us, cgs2_bytes_per_step=per_step,
                                    cgs2_GBs=per_step / (us * 1e-6) / 1e9,
                                    cgs2_frac=per_step / (us * 1e-6) / 1e9 / HBM_PEAK_GBS)
            log(f"{label}: {extra[label]}")

    sweep = None
    if not args.no_sweep and not args.spmv_only:
        sweep = sweep_leg(log, method=args.sweep_method, ell=args.sweep_l)
        sweep["product"] = spmm_leg(log)
    if do_schwarz and not args.spmv_only:
        extra["schwarz"] = schwarz_leg(log)
    if do_adjoint and not args.spmv_only:
        extra["adjoint"] = adjoint_leg(log)
    if args.unstructured and not args.spmv_only:
        extra["unstructured"] = _unstructured_legs(args)

    cpu = None
    side_res = collect_cpu_side(side, args.cpu_wait)
    if sweep is not None:
        sweep_errors(sweep, side_res)
    if not args.no_cpu and not args.spmv_only:
        cpu = cpu_baseline(wl, infos[-1]["iters"], args.cpu_iters, side_res)
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
        "best_solve": best_solve(dt, extra),
        "sweep_speedup": None if sweep is None else {
            k[len("batched_"):]: v["speedup"] for k, v in sweep.items() if k.startswith("batched_")},
        "sweep": sweep,
        "roofline": roof,
        "solve_roofline": solve_roof,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
