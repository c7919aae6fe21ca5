"""Benchmark of the SP2 hot path on one MI355X.

A step is one full FP64 SP2 purification (Gershgorin bounds, X0, then per
iteration the fused X^2 / trace / norm / 2X - X^2 kernel, the deterministic
reductions and the device-side decision) of a synthetic banded Hamiltonian:
N = 32768, half-bandwidth 64, H_ij = exp(-0.5|i-j|) U(-1,1), H_ii ~ N(0,1),
seed 0, N_occ = N/4, capacity M = 256, drop tolerance 1e-8, run until
||X^2 - X||_F < 1e-6.  The inputs are resident on the device before the timed
region starts.

value = algorithmic X^2 bytes of every step kernel in the timed steps divided
by the wall time of those steps (GB/s); the timed solves record no events.  The
roofline object gives the step kernel alone, from one more solve outside the
timed region (bytes per launch / mean launch time from hipEvents recorded by
the library around every launch on the solve's stream).  Algorithmic bytes of
one X^2: every stored entry of X read once and of the pruned X^2 written once
(8-byte value + 4-byte index; 4-byte values in FP32 steps) plus the two
row-width arrays.

Also reported: the mixed-precision solve (FP32 phase, then FP64 steps) to the
same target; single X^2 steps at tau = 1e-5 on X0, the midpoint and the final
iterate; the mixed solve at N = 131072 against the FP64 solve (differences of
X, Tr X and Tr(XH)); the batched workload (256 instances of uneven size in one
call, against solving them one by one); the dense-block variant at N = 8192
(BF16x3 against FP64 MFMA products); the paper's model Hamiltonians (one X^2
of H for metals, semiconductors and soft matter, SP2 on the two gapped
systems); and the oracle on the host cores as cpu_baseline (OpenMP rows on the
host share of cores, with the host's STREAM triad bandwidth beside it).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector and matrix peak
N, B, M_CAP = 32768, 64, 256
TAU, TARGET = 1e-8, 1e-6
# mixed: FP32 phase at 1e-7, FP64 tail at a tighter 1e-9 (the FP32 phase leaves
# rounding noise that the FP64 steps must not prune back in), switch at 1e-2
TAU_MIXED64, TAU_FP32, SWITCH_ETA = 1e-9, 1e-7, 1e-2
METRIC = "ELLPACK X² GB/s (%HBM peak) + SP2 solve ms to ‖X²−X‖_F<1e-6, FP64 vs mixed"


def host_cpu():
    """The host's processor as lscpu reports it (model, sockets, cores, NUMA
    nodes), and the CPUs this process may run on."""
    import subprocess
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return {"model": info.get("Model name"), "sockets": info.get("Socket(s)"),
            "cores_per_socket": info.get("Core(s) per socket"), "threads_per_core": info.get("Thread(s) per core"),
            "numa_nodes": info.get("NUMA node(s)"), "cpus_usable": len(os.sched_getaffinity(0))}


def cpu_threads():
    """Threads of the CPU baseline: the CPUs this process may use, capped by
    OMP_NUM_THREADS when that is set (the host share of one GPU)."""
    n = len(os.sched_getaffinity(0))
    try:
        n = min(n, int(os.environ.get("OMP_NUM_THREADS", n)))
    except ValueError:
        pass
    return max(1, n)


def cpu_baseline_child(seconds_budget):
    """The CPU-baseline measurement, run in a process of its own whose OpenMP
    threads are bound as the paper binds them (OMP_PROC_BIND=spread,
    OMP_PLACES=cores), with every output row first touched by the thread that
    fills it: a STREAM triad for the host's memory bandwidth, then the
    oracle's X^2 on the workload's X0 and following oracle SP2 iterates on all
    threads until the budget is used, and two of those products on one
    thread."""
    host = host_cpu()  # (before the OpenMP runtime binds this thread to one core)

    import oracle
    from paper_2102_08505_amd import synth

    threads = oracle.threads(cpu_threads())
    triad = oracle.stream_triad(1 << 27, 10)
    nnz, idx, val, M = synth.banded_hamiltonian(N, B)
    H = oracle.Ell(N, M, nnz, idx, val)
    rc, lo, hi = oracle.gershgorin(H)
    rc, X, w = oracle.x0(H, lo, hi, TAU, Mo=M + 1)
    # X0 copied into rows first touched in the row schedule
    nz, ix, vl = oracle.empty_rows(N, X.M, X.val.dtype)
    nz[:], ix[:], vl[:] = X.nnz, X.idx, X.val
    X = oracle.Ell(N, X.M, nz, ix, vl)
    X0 = X
    first, times, total_bytes, total_s, calls, passes = [], [], 0, 0.0, 0, 0
    t_start = time.perf_counter()
    while time.perf_counter() - t_start < seconds_budget:
        # one pass: the oracle's SP2 trajectory from X0 to ||X^2 - X||_F < TARGET (the
        # products the GPU solve computes), each X^2 timed
        X, passes = X0, passes + 1
        for n in range(100):
            if passes == 1 and n < 2:
                first.append(X)
            t0 = time.perf_counter()
            rc, Y, d1, d2, wy = oracle.x2(X, TAU, M2=512)
            dt = time.perf_counter() - t0
            if passes == 1:
                times.append(dt)
            calls += 1
            total_bytes += int(X.nnz.sum()) * 12 + 4 * N + int(Y.nnz.sum()) * 12 + 4 * N
            total_s += dt
            if oracle.norm2(X, Y)[0] < TARGET * TARGET:
                break
            up = abs(2 * oracle.pairwise(d1) - oracle.pairwise(d2) - N / 4) < abs(oracle.pairwise(d2) - N / 4)
            if up:
                rc, X, w = oracle.update(X, Y, TAU, Mo=512)
            else:
                X = Y
    oracle.threads(1)
    one_bytes, one_s = 0, 0.0
    for Xi in first:
        t0 = time.perf_counter()
        rc, Y, d1, d2, wy = oracle.x2(Xi, TAU, M2=512)
        one_s += time.perf_counter() - t0
        one_bytes += int(Xi.nnz.sum()) * 12 + int(Y.nnz.sum()) * 12 + 8 * N
    value = total_bytes / total_s / 1e9
    return {"value": value, "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle X^2 (OpenMP rows, {threads} threads, OMP_PROC_BIND=spread OMP_PLACES=cores, "
                      f"first-touch rows) over the oracle's SP2 trajectory of the same N={N} b={B} tau={TAU:g} "
                      f"workload to ||X^2-X||_F<{TARGET:g} ({len(times)} products), {passes} pass(es), "
                      f"{calls} calls, {total_s:.1f} s of X^2",
            "single_thread": {"value": one_bytes / one_s / 1e9, "unit": "GB/s",
                              "sample": f"the first {len(first)} of those products on one thread",
                              "speedup_of_threads": one_s / sum(times[:2])},
            "stream_triad_GBs": triad, "frac_of_triad": value / triad if triad > 0 else None,
            "host": host}


def cpu_baseline(seconds_budget=20.0):
    """Runs cpu_baseline_child in a child process (its OpenMP binding is set
    before the runtime starts and it never touches the GPU)."""
    import subprocess
    env = dict(os.environ, OMP_PROC_BIND="spread", OMP_PLACES="cores", OMP_NUM_THREADS=str(cpu_threads()))
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-only",
                        "--cpu-seconds", str(seconds_budget)], env=env, capture_output=True, text=True,
                       timeout=600)
    if r.returncode != 0:
        raise RuntimeError("CPU baseline failed:\n" + r.stderr[-2000:])
    return json.loads(r.stdout.strip().splitlines()[-1])


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "x2_sym_f64_n32768_traffic.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2102_08505_amd", "csrc", "ell_sym16.hip")


def code_sha256(path):
    """SHA-256 of a C++ source with its // comments, trailing blanks and empty
    lines removed: it changes with the code, not with its comments."""
    import hashlib
    import re
    with open(path, encoding="utf-8") as f:
        lines = [re.sub(r"\s*//.*$", "", ln).rstrip() for ln in f]
    return hashlib.sha256("\n".join(ln for ln in lines if ln).encode()).hexdigest()


def measured_traffic():
    """HBM bytes per launch of the step kernel from the committed rocprofv3
    runs (L2-to-memory requests split by size, checked against a plain copy);
    None when the kernel's code has changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        sha = code_sha256(KERNEL_SOURCE)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_code_sha256") != sha:
        return None
    return rec.get("hbm_bytes_per_launch")


def copy_calibration():
    """A plain device copy of known size (3 x 512 MiB), profiled with the same
    counters to scale FETCH_SIZE / WRITE_SIZE into bytes."""
    import torch
    n = 64 * 1024 * 1024
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": n * 8, "launches": 3}), flush=True)


def batched_leg(E, synth, torch, count=256):
    """The batched workload: 256 Hamiltonians, N uniform in 64..2048, half-bandwidth
    max(4, N/32), mixed precision (FP32 phase, then FP64) to ||X^2-X||_F < 1e-6;
    one batched call against the same instances solved one after another."""
    specs = synth.batched_instances(count, seed=0)
    Hs, Db, Ds, ps = [], [], [], []
    for q, (n, b) in enumerate(specs):
        nnz, idx, val, m = synth.banded_hamiltonian(n, b, seed=0, stream=q)
        Hs.append(E.DeviceEll.from_host(n, m, nnz, idx, val))
        Db.append(E.DeviceEll(n, 4 * b))
        Ds.append(E.DeviceEll(n, 4 * b))
        ps.append(E.sp2_params(n // 4, TAU_MIXED64, TARGET, max_iter=200, precision=E.SP2_MIXED,
                               tau_fp32=TAU_FP32, switch_eta=SWITCH_ETA, poll_every=0))
    hh, hb = [h.h for h in Hs], [d.h for d in Db]
    E.sp2_solve_batched(hh, hb, ps, history=False)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc_b, reps_b = E.sp2_solve_batched(hh, hb, ps, history=False)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    t0 = time.perf_counter()
    singles = [E.sp2_solve(Hs[q].h, Ds[q].h, ps[q], history=False) for q in range(count)]
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    rows = sum(n for n, _ in specs)
    return {"workload": f"{count} banded Hamiltonians, N uniform in 64..2048 (sum {rows} rows), "
                        f"half-bandwidth max(4, N/32), mixed tau {TAU_FP32:g}/{TAU_MIXED64:g}, "
                        f"to ||X^2-X||_F<{TARGET:g}",
            "status": int(rc_b), "ok": sum(1 for r in reps_b if r["status"] == 0),
            "tuned": {"iterations_per_graph": reps_b[0]["batch_k"],
                      "step_kernel": "register-tiled VALU" if reps_b[0]["batch_kernel"] else "matrix cores"},
            "batched_ms": tb * 1e3, "sequential_ms": ts * 1e3, "speedup_vs_sequential": ts / tb,
            "max_iterations": max(r["iterations"] for r in reps_b),
            "max_eta": max(r["eta"] for r in reps_b),
            "same_as_single": all(reps_b[q]["iterations"] == singles[q][1]["iterations"]
                                  and reps_b[q]["eta"] == singles[q][1]["eta"] for q in range(count))}


def x2_single_leg(E, H, tau=1e-5):
    """One FP64 X^2 step timed on X0, on the midpoint iterate and on the final
    iterate of an SP2 solve of the benchmark H at drop tolerance tau (run to
    its eta floor), from the library's per-launch events and algorithmic bytes."""
    p = E.sp2_params(N / 4, tau, TARGET, max_iter=200, profile=1)
    D = E.DeviceEll(N, M_CAP)
    E.sp2_solve(H.h, D.h, p)  # warm-up
    rc, rep = E.sp2_solve(H.h, D.h, p)
    secs, byts = rep["x2_seconds_each"], rep["x2_bytes_each"]
    k = min(len(secs), len(byts))
    out = {"tau": tau, "status": int(rc), "iterations": rep["iterations"], "eta_floor": rep["eta"]}
    for name, q in (("x0", 0), ("mid", k // 2), ("final", k - 1)):
        if k == 0:
            break
        gbs = byts[q] / secs[q] / 1e9
        out[name] = {"iteration": int(q), "us": float(secs[q] * 1e6), "bytes": int(byts[q]), "GBs": float(gbs),
                     "hbm_frac": float(gbs / HBM_PEAK_GBS)}
    return out


def accuracy_leg(E, synth, torch, n=131072, b=64):
    """Mixed precision at N = 131072 (FP32 values and products, FP64 traces,
    branch, convergence test and final steps) against the FP64 solve of the same
    H, which equals the FP64 oracle bit for bit (the parity tests): Frobenius
    difference of the density matrices and the differences of Tr X and Tr(XH)."""
    import numpy as np
    import scipy.sparse as sp
    nnz, idx, val, m = synth.banded_hamiltonian(n, b, seed=0)
    H = E.DeviceEll.from_host(n, m, nnz, idx, val)
    # tau = 1e-8 leaves the FP64 solve above eta = 1e-6 at this size (its floor grows with N), so
    # both solves end with the mixed run's FP64 tolerance
    out = {"workload": f"banded H N={n} half-bandwidth {b}, N_occ={n // 4}, to ||X^2-X||_F<{TARGET:g}; "
                       f"FP64 tau {TAU_MIXED64:g}; mixed tau {TAU_FP32:g}/{TAU_MIXED64:g}"}

    def csr(D):
        N, M, dn, di, dv = D.download()
        rows = np.repeat(np.arange(N), dn)
        keep = (np.arange(M)[None, :] < dn[:, None]).reshape(-1)
        return sp.csr_matrix((dv[keep], (rows, di[keep])), shape=(N, N))

    mats, energy = {}, {}
    for name, prec, tau in (("f64", E.SP2_F64, TAU_MIXED64), ("mixed", E.SP2_MIXED, TAU_MIXED64)):
        D = E.DeviceEll(n, M_CAP)
        p = E.sp2_params(n / 4, tau, TARGET, max_iter=200, precision=prec, tau_fp32=TAU_FP32,
                         switch_eta=SWITCH_ETA)
        E.sp2_solve(H.h, D.h, p, history=False)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, rep = E.sp2_solve(H.h, D.h, p, history=False)
        torch.cuda.synchronize()
        out[name] = {"status": int(rc), "solve_ms": (time.perf_counter() - t0) * 1e3,
                     "iterations": rep["iterations"], "fp32_iterations": rep["fp32_iterations"], "eta": rep["eta"]}
        # the step kernel's own rate at a size whose three span buffers exceed the
        # 256 MB last-level cache: one more solve with events around every launch
        p.profile = 1
        _, prof = E.sp2_solve(H.h, D.h, p, history=False)
        gbs = prof["x2_bytes"] / prof["x2_seconds"] / 1e9
        out[name]["x2_us_per_launch"] = prof["x2_seconds"] / prof["x2_launches"] * 1e6
        out[name]["x2_GBs"] = gbs
        out[name]["x2_hbm_frac"] = gbs / HBM_PEAK_GBS
        mats[name] = csr(D)
        rc_e, energy[name] = E.ellpack_trace_product(D.h, H.h)  # Tr(XH) on the device
        if rc_e != E.ELL_OK:
            raise RuntimeError(E.ellpack_strerror(rc_e))
    X64, X32 = mats["f64"], mats["mixed"]
    dX = X32 - X64
    tr64, tr32 = X64.diagonal().sum(), X32.diagonal().sum()
    txh64, txh32 = energy["f64"], energy["mixed"]
    out["err_vs_f64"] = {"fro_dX": float(np.sqrt(dX.multiply(dX).sum())),
                         "fro_dX_rel": float(np.sqrt(dX.multiply(dX).sum() / X64.multiply(X64).sum())),
                         "max_abs_dX": float(abs(dX).max()) if dX.nnz else 0.0,
                         "abs_dTrX": float(abs(tr32 - tr64)), "abs_dTrXH": float(abs(txh32 - txh64)),
                         "TrX_f64": float(tr64), "TrXH_f64": float(txh64)}
    out["speedup_mixed_vs_f64"] = out["f64"]["solve_ms"] / out["mixed"]["solve_ms"]
    return out


def last_product_alu(D, prof):
    """Arithmetic roofline of the last product of a profiled solve: D is the
    iterate whose X^2 it computed; its multiply-adds F = sum_i sum_{k in row i}
    nnz(row k), counted on the host."""
    import numpy as np
    _, dM, dn, di, _ = D.download()
    di = di.reshape(-1, dM)
    keep = np.arange(dM)[None, :] < dn[:, None]
    F = int(dn.astype(np.int64)[di[keep]].sum())
    t_last = float(prof["x2_seconds_each"][-1])
    b_last = int(prof["x2_bytes_each"][-1])
    return {"flops_last_launch": 2 * F, "seconds_last_launch": t_last, "achieved_tflops": 2 * F / t_last / 1e12,
            "peak_tflops": FP64_PEAK_TFLOPS, "frac": 2 * F / t_last / 1e12 / FP64_PEAK_TFLOPS,
            "intensity_flop_per_byte": 2 * F / b_last, "ridge_flop_per_byte": FP64_PEAK_TFLOPS * 1e3 / HBM_PEAK_GBS}


def fp64_target_leg(E, H, torch, tau=1e-10, target=1e-8, reps=3):
    """FP64 SP2 of the benchmark H to the FP64 idempotency target 1e-8, at the
    drop tolerance that reaches it at this size (the floor of ||X^2 - X||_F
    grows with tau): solve time, iterations, final width, the step kernel's
    per-launch rate against the HBM roofline and, for the last product, against
    the FP64 roofline (the rows are wider here: the intensity passes the ridge)."""
    import numpy as np
    D = E.DeviceEll(N, M_CAP)
    p = E.sp2_params(N / 4, tau, target, max_iter=200)
    E.sp2_solve(H.h, D.h, p, history=False)  # warm-up (and capacity growth)
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, rep = E.sp2_solve(H.h, D.h, p, history=False)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    p.profile = 1
    _, prof = E.sp2_solve(H.h, D.h, p, history=True)
    launches = prof["x2_launches"]
    gbs = prof["x2_bytes"] / prof["x2_seconds"] / 1e9
    return {"workload": f"FP64 SP2 of the benchmark H (N={N}, half-bandwidth {B}), tau={tau:g}, "
                        f"to ||X^2-X||_F<{target:g}",
            "status": int(rc), "solve_ms": float(np.median(times)) * 1e3, "iterations": rep["iterations"],
            "final_M": rep["final_M"], "eta": rep["eta"],
            "x2_us_per_launch": prof["x2_seconds"] / launches * 1e6, "x2_GBs": gbs, "x2_hbm_frac": gbs / HBM_PEAK_GBS,
            "alu_last_product": last_product_alu(D, prof)}


def prune_mode_leg(E, synth, torch, H, reps=5, n_small=4096):
    """One pruning per iteration against two (sp2_params.prune_once), FP64, to
    ||X^2 - X||_F < 1e-6 on the benchmark H: two prunings at tau = 1e-8 (the
    headline solve), one pruning at tau = 1e-8 and at 1e-9 (its norm includes
    the pruned tail of X^2, so at 1e-8 it stalls above the target and the stall
    rule stops it) -- time, iterations, eta, the step kernel's per-launch time,
    and how far each density matrix and energy Tr(DH) ends from the headline
    solve's; then, at N = 4096 with the same recipe, each configuration's
    distance to the exact projector onto the N/4 lowest eigenvectors of H
    (FP64 eigendecomposition on the GPU)."""
    import numpy as np
    import scipy.sparse as sp

    def csr(D):
        N_, M_, dn, di, dv = D.download()
        rows = np.repeat(np.arange(N_), dn)
        keep = (np.arange(M_)[None, :] < dn[:, None]).reshape(-1)
        return sp.csr_matrix((dv[keep], (rows, di[keep])), shape=(N_, N_))

    configs = (("two_prunings_tau1e-8", 0, 1e-8), ("one_pruning_tau1e-8", 1, 1e-8),
               ("one_pruning_tau1e-9", 1, 1e-9))
    out = {"workload": f"FP64 SP2 of the benchmark H (N={N}, half-bandwidth {B}) to ||X^2-X||_F<{TARGET:g} "
                       f"with two prunings per iteration and with one; distance to the exact projector at "
                       f"N={n_small}"}
    mats, energy = {}, {}
    for name, once, tau in configs:
        D = E.DeviceEll(N, M_CAP)
        p = E.sp2_params(N / 4, tau, TARGET, max_iter=200, prune_once=once)
        E.sp2_solve(H.h, D.h, p, history=False)  # warm-up
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, rep = E.sp2_solve(H.h, D.h, p, history=False)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        p.profile = 1
        _, prof = E.sp2_solve(H.h, D.h, p, history=False)
        out[name] = {"status": int(rc), "solve_ms": float(np.median(times)) * 1e3,
                     "solve_ms_device": rep["seconds"] * 1e3, "iterations": rep["iterations"], "eta": rep["eta"],
                     "x2_us_per_launch": prof["x2_seconds"] / prof["x2_launches"] * 1e6}
        mats[name] = csr(D)
        rc_e, energy[name] = E.ellpack_trace_product(D.h, H.h)
        if rc_e != E.ELL_OK:
            raise RuntimeError(E.ellpack_strerror(rc_e))
    ref = configs[0][0]
    for name, _, _ in configs[1:]:
        dX = mats[name] - mats[ref]
        out[name]["fro_dD_vs_two_prunings"] = float(np.sqrt(dX.multiply(dX).sum()))
        out[name]["abs_dTrDH_vs_two_prunings"] = float(abs(energy[name] - energy[ref]))
    # the exact projector at a size an eigendecomposition takes in a moment
    nnz, idx, val, m = synth.banded_hamiltonian(n_small, B, seed=0)
    Hs = E.DeviceEll.from_host(n_small, m, nnz, idx, val)
    Hd = np.zeros((n_small, n_small))
    for i in range(n_small):
        Hd[i, idx[i * m:i * m + nnz[i]]] = val[i * m:i * m + nnz[i]]
    w, V = torch.linalg.eigh(torch.from_numpy(Hd).cuda())
    Vo = V[:, :n_small // 4]
    P = (Vo @ Vo.T).cpu().numpy()
    small = {"N": n_small, "gap_at_fermi": float(w[n_small // 4] - w[n_small // 4 - 1])}
    for name, once, tau in configs:
        D = E.DeviceEll(n_small, M_CAP)
        rc, rep = E.sp2_solve(Hs.h, D.h, E.sp2_params(n_small / 4, tau, TARGET, max_iter=200, prune_once=once),
                              history=False)
        small[name] = {"status": int(rc), "iterations": rep["iterations"], "eta": rep["eta"],
                       "fro_D_minus_P": float(np.linalg.norm(csr(D).toarray() - P))}
    out["vs_projector"] = small
    return out


def nonbanded_leg(E, synth, torch, reps=10):
    """Products whose rows are not intervals: one FP64 step (X^2, 2X - X^2,
    traces, norm) of the nearest-neighbour Hamiltonian of a 32^3 cubic lattice
    (N = 32768, 7 entries per row spread over 2049 columns; the products of a
    row fit the hashed row accumulator), and of a random symmetric matrix with
    about 100 entries per row spread over all of N = 20000 columns (rows of
    about 9000 products: the window kernel)."""
    import numpy as np
    out = {"workload": "one FP64 step (tau 1e-5) of the 32^3 lattice Hamiltonian (hashed accumulator) and of a "
                       "random symmetric N=20000 matrix with ~100 scattered entries per row (window kernel)"}
    rng = np.random.default_rng(5)

    def scattered(n, per_row):
        i = np.repeat(np.arange(n), per_row)
        j = rng.integers(0, n, size=n * per_row)
        keep = i != j
        lo, hi = np.minimum(i[keep], j[keep]), np.maximum(i[keep], j[keep])
        key = np.unique(lo.astype(np.int64) * n + hi)
        lo, hi = key // n, key % n
        v = rng.uniform(-1, 1, size=lo.size) * 0.1
        rows = np.concatenate([lo, hi, np.arange(n)])
        cols = np.concatenate([hi, lo, np.arange(n)])
        vals = np.concatenate([v, v, rng.uniform(-1, 1, size=n)])
        order = np.lexsort((cols, rows))
        rows, cols, vals = rows[order], cols[order], vals[order]
        nnz = np.bincount(rows, minlength=n).astype(np.int32)
        m = int(nnz.max())
        start = np.concatenate([[0], np.cumsum(nnz)[:-1]])
        slot = np.arange(rows.size) - start[rows]
        idx = np.full(n * m, -1, np.int32)
        val = np.zeros(n * m)
        idx[rows * m + slot] = cols
        val[rows * m + slot] = vals
        return nnz, idx, val, m

    cases = (("lattice_32", 32768, synth.grid3d_hamiltonian(32), 64),
             ("scattered_20000", 20000, scattered(20000, 50), 12288))
    for name, n, (nnz, idx, val, m), cap in cases:
        X = E.DeviceEll.from_host(n, m, nnz, idx, val)
        Y = E.DeviceEll(n, cap)
        U = E.DeviceEll(n, cap)
        rc, res, widths = E.ellpack_x2_step(X.h, Y.h, U.h, 1e-5)  # warm-up
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, res, widths = E.ellpack_x2_step(X.h, Y.h, U.h, 1e-5)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        ms = float(np.median(times)) * 1e3
        ny = int(Y.download()[2].sum())
        fma = int(sum(int(nnz[idx[i * m:i * m + nnz[i]]].sum()) for i in range(n)))
        byt = int(nnz.sum()) * 12 + ny * 12 + 8 * n
        out[name] = {"status": int(rc), "N": n, "width_X": int(nnz.max()), "width_X2": int(widths[0]), "ms": ms,
                     "fma": fma, "GBs": byt / ms / 1e6, "gfma_per_s": fma / ms / 1e6}
    return out


def model_leg(E, synth, torch, reps=5):
    """The paper's model Hamiltonians (metals, semiconductors, soft matter,
    section "On the Generation of Model Hamiltonian System Matrices"): one FP64
    X^2 of H itself at tau = 1e-5 on each system at 32000 orbitals; then SP2,
    FP64 and mixed, on the two gapped systems at 4096 orbitals and at the
    32000 orbitals of the paper's ExaSP2 runs, N_occ = the eigenvalues below
    the 0 eV Fermi level (dense spectrum at 4096; at 32000 Sylvester's inertia
    of block Schur complements, counted for the semiconductor at 0.05, inside
    its gap (0, 0.93), since its highest occupied states round to within
    1e-9 of 0)."""
    import numpy as np
    out = {"workload": "model Hamiltonians (A/B two-level chains, drop threshold 1e-5): X^2 of H at tau 1e-5; "
                       f"SP2 at N=4096 and 32000, FP64 tau {TAU_MIXED64:g} at 4096 and {0.1 * TAU_MIXED64:g} at 32000 "
                       f"(also the mixed solves' FP64 steps), mixed FP32 tau {TAU_FP32:g}, to "
                       f"||X^2-X||_F<{TARGET:g}"}
    x2 = {}
    for kind, n in (("metal", 32000), ("semiconductor", 32000), ("soft_matter", 32000)):
        nnz, idx, val, m = synth.model_hamiltonian(kind, n)
        X = E.DeviceEll.from_host(n, m, nnz, idx, val)
        Y = E.DeviceEll(n, min(4096, n))
        rc, tr, w = E.ellpack_x2_threshold(X.h, Y.h, 1e-5)  # warm-up; the product's width
        if rc != E.ELL_OK:
            x2[kind] = {"N": n, "status": int(rc), "width": int(w)}
            continue
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            E.ellpack_x2_threshold(X.h, Y.h, 1e-5)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / reps
        ynnz = Y.download()[2]
        byts = (int(nnz.sum()) * 12 + 4 * n) + (int(ynnz.sum()) * 12 + 4 * n)
        x2[kind] = {"N": n, "status": int(rc), "H_width": int(m), "H_sparsity": 1.0 - float(nnz.sum()) / n / n,
                    "x2_width": int(w), "ms": sec * 1e3, "bytes": byts, "GBs": byts / sec / 1e9,
                    "fma": int(nnz.astype(np.int64)[idx.reshape(n, m)[np.arange(m)[None, :] < nnz[:, None]]].sum())}
        x2[kind]["tflops"] = 2 * x2[kind]["fma"] / sec / 1e12
        del X, Y
    out["x2"] = x2
    sp2 = {}
    for n, kind in ((4096, "semiconductor"), (4096, "soft_matter"), (32000, "semiconductor"),
                    (32000, "soft_matter")):
        nnz, idx, val, m = synth.model_hamiltonian(kind, n)
        if n <= 4096:
            n_occ, w = synth.fermi_occupation(nnz, idx, val, m)
            res = {"N": n, "n_occ": n_occ, "gap_at_fermi": float(w[n_occ] - w[n_occ - 1]),
                   "spectrum": [float(w[0]), float(w[-1])]}
        else:
            mu = 0.05 if kind == "semiconductor" else 0.0
            n_occ, margin = synth.fermi_occupation_banded(nnz, idx, val, m, mu=mu)
            res = {"N": n, "n_occ": n_occ, "n_occ_below": mu, "inertia_margin": margin}
        H = E.DeviceEll.from_host(n, m, nnz, idx, val)
        # tau = 1e-8 leaves FP64 above eta = 1e-6 on these spectra: both solves use the mixed run's FP64
        # tau; at 32000 orbitals 1e-9 leaves the semiconductor's mixed solve stalled at eta = 3.1e-6
        # (rows of 3500 entries pruned at 1e-9), so both solves there prune at 1e-10
        tau = TAU_MIXED64 if n <= 4096 else 0.1 * TAU_MIXED64
        res["tau_fp64"] = tau
        for name, prec in (("f64", E.SP2_F64), ("mixed", E.SP2_MIXED)):
            D = E.DeviceEll(n, 256)
            p = E.sp2_params(n_occ, tau, TARGET, max_iter=200, precision=prec, tau_fp32=TAU_FP32,
                             switch_eta=SWITCH_ETA)
            E.sp2_solve(H.h, D.h, p, history=False)  # warm-up (and capacity growth)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, rep = E.sp2_solve(H.h, D.h, p, history=False)
            torch.cuda.synchronize()
            res[name] = {"status": int(rc), "solve_ms": (time.perf_counter() - t0) * 1e3,
                         "iterations": rep["iterations"], "fp32_iterations": rep["fp32_iterations"],
                         "eta": rep["eta"], "trace": rep["trace_x"], "final_M": rep["final_M"]}
            del D
        sp2[f"{kind}_{n}"] = res
        del H
    out["sp2"] = sp2
    return out


def dense_leg(E, synth, torch, n=8192, b=512):
    """Dense-block variant: N = 8192 dense H (half-bandwidth 512), SP2 to
    ||X^2-X||_F < 1e-6 with BF16x3 products (then FP64 steps) and in plain FP64."""
    Hh = synth.dense_hamiltonian(n, b, seed=0)
    dH = torch.from_numpy(Hh).cuda()
    dD = torch.empty_like(dH)
    out = {"workload": f"dense banded H N={n} half-bandwidth {b}, N_occ={n // 4}, to ||X^2-X||_F<{TARGET:g}"}
    for mode, name in ((E.DENSE_BF16X3, "bf16x3"), (E.DENSE_F64, "f64")):
        p = E.sp2_params(n / 4, 0.0, TARGET, max_iter=100, poll_every=8, profile=1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, rep = E.dense_sp2_solve(dH.data_ptr(), n, dD.data_ptr(), mode, p, torch.cuda.current_stream(),
                                    history=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        # per product of the mode's own precision (a BF16x3 solve ends with a few FP64 products)
        secs, prec = rep["x2_seconds_each"], rep["prec"][:len(rep["x2_seconds_each"])]
        own = secs[prec == (1 if mode == E.DENSE_BF16X3 else 0)]
        per = float(own.mean()) if len(own) else rep["x2_seconds"] / max(rep["x2_launches"], 1)
        flops = 2.0 * n ** 3
        # H is symmetric: the products compute the tiles on and above the diagonal
        # (128 x 128), nt (nt + 1) / 2 of nt^2
        nt = (n + 127) // 128
        executed = flops * (nt * (nt + 1) / 2) / (nt * nt)
        out[name] = {"status": int(rc), "solve_ms": wall * 1e3, "iterations": rep["iterations"],
                     "fp32_iterations": rep["fp32_iterations"], "eta": rep["eta"],
                     "x2_ms_per_product": per * 1e3,
                     "x2_tflops": flops / per / 1e12 if per > 0 else None,
                     "x2_tflops_executed": executed / per / 1e12 if per > 0 else None}
    bf, f64 = out["bf16x3"], out["f64"]
    out["speedup_bf16x3_vs_f64"] = f64["solve_ms"] / bf["solve_ms"]
    out["note"] = ("x2_tflops counts 2 N^3 per product (the whole X^2); the symmetric product executes the upper "
                   "triangle of tiles only (x2_tflops_executed), against which mfma_frac is taken")
    # MFMA rooflines: BF16x3 executes three bf16 products per X^2 (2.5 PFLOP/s dense
    # bf16 peak); FP64 runs at the 78.6 TFLOP/s FP64 matrix peak
    if bf["x2_tflops_executed"]:
        bf["mfma_frac"] = 3 * bf["x2_tflops_executed"] / 2500.0
    if f64["x2_tflops_executed"]:
        f64["mfma_frac"] = f64["x2_tflops_executed"] / 78.6
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing on the host")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the N = 131072 mixed-vs-FP64 comparison")
    ap.add_argument("--no-x2-single", action="store_true", help="skip the tau = 1e-5 single X^2 timings")
    ap.add_argument("--no-model", action="store_true", help="skip the paper's model Hamiltonians")
    ap.add_argument("--no-fp64-target", action="store_true",
                    help="skip the FP64 solve to ||X^2-X||_F < 1e-8 (tau = 1e-10)")
    ap.add_argument("--no-nonbanded", action="store_true", help="skip the non-banded products")
    ap.add_argument("--no-prune-mode", action="store_true",
                    help="skip the comparison of one and two prunings per iteration")
    ap.add_argument("--main-only", action="store_true",
                    help="only the FP64 solves of the headline line (for profiling the step kernel)")
    ap.add_argument("--profile-size", type=int, default=0,
                    help="with --main-only: run the FP64 solves at this N instead (tau 1e-9 above N = 32768), "
                         "for profiling the step kernel at a size beyond the last-level cache")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain copy of known size (for scaling the HBM counters)")
    ap.add_argument("--cpu-baseline-only", action="store_true",
                    help="only the CPU baseline (host cores, no GPU): one JSON object")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="time budget of the CPU baseline's X^2 calls")
    args = ap.parse_args()
    if args.cpu_baseline_only:
        print(json.dumps(cpu_baseline_child(args.cpu_seconds)))
        return
    if args.profile_size and not args.main_only:
        print("--profile-size goes with --main-only", file=sys.stderr)
        sys.exit(2)
    if args.main_only:
        args.no_cpu = args.no_mixed = args.no_batched = args.no_dense = True
        args.no_accuracy = args.no_x2_single = args.no_model = args.no_fp64_target = True
        args.no_prune_mode = args.no_nonbanded = True
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU row-block split "
              f"is a design, not a build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2102_08505_amd import ellsp2 as E
    from paper_2102_08505_amd import synth

    E.load()
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    global N, TAU
    if args.profile_size:
        N = args.profile_size
        if N > 32768:
            TAU = TAU_MIXED64  # (tau 1e-8 leaves the FP64 solve above the target at larger N)
    nnz, idx, val, M = synth.banded_hamiltonian(N, B)
    H = E.DeviceEll.from_host(N, M, nnz, idx, val, stream=stream)
    D = E.DeviceEll(N, M_CAP, stream=stream)

    def solve(precision, profile=0, history=False):
        tau = TAU if precision == E.SP2_F64 else TAU_MIXED64
        p = E.sp2_params(N / 4, tau, TARGET, max_iter=200, precision=precision, tau_fp32=TAU_FP32,
                         switch_eta=SWITCH_ETA, profile=profile)
        rc, rep = E.sp2_solve(H.h, D.h, p, history=history)
        return rc, rep

    for _ in range(args.warmup):
        solve(E.SP2_F64)
    torch.cuda.synchronize()
    reps = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rc, rep = solve(E.SP2_F64)
        reps.append((rc, rep))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rcs = {rc for rc, _ in reps}
    x2_bytes = sum(r["x2_bytes"] for _, r in reps)
    last = reps[-1][1]
    ms_per_step = wall / args.steps * 1e3
    value = x2_bytes / wall / 1e9
    # the step kernel's own rate: one more solve, outside the timed region, with
    # hipEvents around every X^2 launch on the solve's stream
    _, prof = solve(E.SP2_F64, profile=1, history=True)
    launches = prof["x2_launches"]
    x2_sec = prof["x2_seconds"]
    achieved = (prof["x2_bytes"] / launches) / (x2_sec / launches) / 1e9
    alu = last_product_alu(D, prof)

    mixed = None
    if not args.no_mixed:
        for _ in range(args.warmup):
            solve(E.SP2_MIXED)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        mreps = [solve(E.SP2_MIXED) for _ in range(args.steps)]
        torch.cuda.synchronize()
        mwall = time.perf_counter() - t1
        mr = mreps[-1][1]
        mixed = {"status": int(mreps[-1][0]), "ms_per_solve": mwall / args.steps * 1e3,
                 "iterations": mr["iterations"], "fp32_iterations": mr["fp32_iterations"],
                 "eta": mr["eta"], "tau_fp32": TAU_FP32, "tau_fp64": TAU_MIXED64, "switch_eta": SWITCH_ETA,
                 "speedup_vs_fp64": ms_per_step / (mwall / args.steps * 1e3)}

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"FP64 SP2 solve of a banded Hamiltonian N={N} half-bandwidth {B} "
                               f"(exp(-0.5|i-j|)U(-1,1) couplings, N(0,1) diagonal, seed 0), N_occ={N // 4}, "
                               f"M={M_CAP}, tau={TAU:g}, to ||X^2-X||_F<{TARGET:g}",
                   "N": N, "bandwidth": B, "M": M_CAP, "tau": TAU, "idem_target": TARGET, "n_occ": N // 4},
        "sp2": {"status": sorted(rcs), "iterations": last["iterations"], "eta": last["eta"],
                "final_M": last["final_M"], "solve_ms_device": last["seconds"] * 1e3,
                "x2_launches_per_solve": launches,
                "x2_ms_per_launch": x2_sec / launches * 1e3},
        "mixed": mixed,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel": "k_x2_sym_step (X^2 of the bitwise symmetric span form on the FP64 matrix "
                               "cores, pruning, traces, norm, the iterate of the branch fixed beforehand; "
                               "the last workgroup reduces the partial sums and takes the SP2 decision)",
                     "bytes_per_launch": prof["x2_bytes"] / launches,
                     "alu": alu},
    }
    legs = (("fp64_to_1e-8", args.no_fp64_target, lambda: fp64_target_leg(E, H, torch)),
            ("prune_modes", args.no_prune_mode, lambda: prune_mode_leg(E, synth, torch, H)),
            ("nonbanded", args.no_nonbanded, lambda: nonbanded_leg(E, synth, torch)),
            ("x2_single_tau1e-5", args.no_x2_single, lambda: x2_single_leg(E, H)),
            ("batched", args.no_batched, lambda: batched_leg(E, synth, torch)),
            ("dense", args.no_dense, lambda: dense_leg(E, synth, torch)),
            ("mixed_accuracy", args.no_accuracy, lambda: accuracy_leg(E, synth, torch)),
            ("model_hamiltonians", args.no_model, lambda: model_leg(E, synth, torch)),
            ("cpu_baseline", args.no_cpu, lambda: cpu_baseline(args.cpu_seconds)))
    for name, skip, leg in legs:
        if skip:
            continue
        t0 = time.perf_counter()
        line[name] = leg()
        # progress on stderr (stdout carries the one JSON line)
        print(f"bench: {name} done in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
