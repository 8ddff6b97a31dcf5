#!/usr/bin/env python3
"""Benchmark: self-energy moment sets per second on one MI355X.

A step is one self-energy moment set {Sigma^{(n,<)}, Sigma^{(n,>)} : n <= nmom_max}
for one molecule, produced from device-resident eps and L through the C ABI
(particle-hole gather, density-response moments, W-moment cores and the
self-energy contraction).  The block-Lanczos poles and the upfolded
eigensolve are timed once afterwards and reported beside the metric.

Workload (default): nocc=100, nvir=400, naux=1500, nmom_max=11, TDA screening,
seeded synthetic inputs (occupied eps ~ U[-1.5,-0.3] Ha, virtual eps ~ U[0.1,3.0] Ha,
L symmetric Gaussian with std 0.3/sqrt(naux) and exp(-|p-q|/8) decay), mixed
precision, with the FP64 form timed beside it.  The same JSON line also
carries the RPA form at that size (mixed and FP64, a few sets) and the
64-molecule batch (a few graph replays beside sequential calls);
--no-extra leaves them out.

Prints ONE JSON line (see the keys below).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MI355X_PEAK = {"f64": 78.6e12, "bf16": 2.5e15, "i8": 5.0e15, "f32": 157.3e12}


def set_flops(o, v, A, N):
    """Algorithmic flops of one TDA moment set: recursion (4N+2) A^2 ov,
    W-core contraction (N+1) A^2 M(M+1) and self-energy contraction
    (N+1) A M^2 (M+1): R_t L is symmetric in its orbital pair and Sigma^(n)
    in (p, q), so each symmetric pair is counted once."""
    M = o + v
    return (4 * N + 2) * A * A * o * v + (N + 1) * A * A * M * (M + 1.0) + (N + 1) * A * M * M * (M + 1.0)


def host_facts():
    """Cores, CPU model and BLAS of the host the oracle runs on."""
    import numpy as np
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    blas, threads = None, None
    try:
        from threadpoolctl import threadpool_info
        info = [d for d in threadpool_info() if d.get("user_api") == "blas"]
        if info:
            blas = f"{info[0].get('internal_api')} {info[0].get('version')}"
            threads = max(int(d.get("num_threads", 1)) for d in info)
    except Exception:
        pass
    return {"cpu_count": os.cpu_count(), "cpu_model": model, "blas": blas or np.__config__.__name__,
            "blas_threads": threads or os.cpu_count()}


def cpu_baseline(o, v, A, N, seed):
    """Time the oracle as it stands on a bounded sample of the same workload:
    the full TDA recursion (eta~ and R_t), plus the self-energy contraction
    restricted to t = 0 (one of the nmom_max+1 identical-cost t passes of the
    oracle's loop); each part best of 3.  The set time is extrapolated as the
    recursion time + (N+1) x the t = 0 time (the full oracle set takes minutes)."""
    import gwsynth
    from oracle import gw as ogw
    facts = host_facts()
    eps, L = gwsynth.system(o, v, A, seed)
    V, D = ogw.particle_hole(eps, L, o)
    t_rec, t_sig = [], []
    for _ in range(3):
        t0 = time.perf_counter()
        eta = ogw.tda_eta(V, D, N)
        R = ogw.w_core(eta, V)
        t1 = time.perf_counter()
        ogw.sigma_moments(eps, L, o, R[:1])
        t2 = time.perf_counter()
        t_rec.append(t1 - t0)
        t_sig.append(t2 - t1)
        del eta
    tr, ts = min(t_rec), min(t_sig)
    t_set = tr + (N + 1) * ts
    return {"value": 1.0 / t_set, "unit": "sets/s", "cores": int(facts["blas_threads"]), "kind": "oracle",
            "sample": (f"extrapolated: full TDA recursion ({tr:.2f} s) + self-energy contraction for t=0 "
                       f"({ts:.2f} s) x {N + 1} t-passes, each best of 3; same inputs, FP64 NumPy"),
            "host": facts}


def fold_kernel_source():
    """The text the stage-1 kernel is built from: its job struct, the LDS
    swizzle and the kernel itself (hashed to tie recorded counters to it)."""
    csrc = os.path.join(ROOT, "paper_2504_17439_amd", "csrc")
    jobs = open(os.path.join(csrc, "mixed_jobs.h")).read()
    src = open(os.path.join(csrc, "sigma_mixed.hip")).read()
    a = jobs.index("struct FoldJob {")
    part1 = jobs[a:jobs.index("};", a) + 2]
    b = src.index("__device__ __forceinline__ int swz(")
    part2 = src[b:src.index("\n", b)]
    c = src.index("template <int NT>\nstruct FoldSlab {")
    part3 = src[c:src.index("// Grouped, persistent, XCD-aware: the tiles of every job")]
    return part1 + part2 + part3


def recorded_traffic(o, v, A, N):
    """HBM bytes per stage-1 launch from the committed rocprofv3 counter runs
    (FETCH_SIZE and WRITE_SIZE scaled by a plain-copy calibration), used only
    for the workload they were taken on and while the kernel source is the one
    they were taken with; otherwise None."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "fold_mixed_traffic.json")))
        h = hashlib.sha256(fold_kernel_source().encode()).hexdigest()
    except (OSError, ValueError, KeyError):
        return None
    if h != rec.get("kernel_source_sha256") or (o, v, A, N) != (100, 400, 1500, 11):
        return None
    return rec["traffic_bytes_per_launch"]


def measure_batched(nsys, seed, steps, warmup, branches=4):
    """64-molecule batch (nmo uniform over multiples of 5 in [60, 400], nocc =
    nmo/5, naux = 3.5 nmo, TDA, nmom_max = 7, mixed): sets/s of the captured
    batch replay, beside sequential single-molecule calls in mixed precision
    and in FP64 (inputs drawn on the device)."""
    import torch
    import gwsynth
    from paper_2504_17439_amd import gwmom

    N = 7
    shapes = gwsynth.batch_shapes(nsys, seed=seed)
    print(f"[bench] generating {len(shapes)} molecules on the device", file=sys.stderr, flush=True)
    sys_t = []
    for k, (o, v, A) in enumerate(shapes):
        e, l = gwsynth.system_device(o, v, A, seed=seed * 1000 + k)
        sys_t.append((e, l, o))
    torch.cuda.synchronize()
    h = gwmom.Handle(0)
    seq = {}
    for prec in ("mixed", "fp64"):
        print(f"[bench] sequential single-molecule calls, {prec}", file=sys.stderr, flush=True)
        for e, l, o in sys_t[:2]:
            h.sigma_moments(e, l, o, N, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for e, l, o in sys_t:
            h.sigma_moments(e, l, o, N, precision=prec)
        torch.cuda.synchronize()
        seq[prec] = time.perf_counter() - t0
    print("[bench] planning the batch", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    b = h.batch(sys_t, N, precision="mixed", bopts={"autotune": 1, "branches": branches})
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    info = b.info()
    print(f"[bench] plan {plan_s:.1f} s {info}; warmup", file=sys.stderr, flush=True)
    for _ in range(warmup):
        b.run()
    torch.cuda.synchronize()
    print(f"[bench] timed region ({steps} batch replays)", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        b.run()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    b.close()
    h.close()
    del sys_t
    torch.cuda.empty_cache()
    nsets = len(shapes) * steps
    flops = sum(set_flops(o, v, A, N) for o, v, A in shapes)
    return {"sets_per_s": nsets / el, "ms_per_replay": 1e3 * el / steps, "replays": steps, "nsys": len(shapes),
            "sequential_sets_per_s": len(shapes) / seq["mixed"],
            "speedup_vs_sequential": (nsets / el) / (len(shapes) / seq["mixed"]),
            "sequential_fp64_sets_per_s": len(shapes) / seq["fp64"],
            "speedup_vs_sequential_fp64": (nsets / el) / (len(shapes) / seq["fp64"]),
            "plan_seconds": plan_s, "plan": info, "useful_tflops": flops * steps / el / 1e12,
            "workload": f"batch of {len(shapes)} molecules, TDA mixed, nmom_max={N}, nmo uniform over multiples "
                        "of 5 in [60, 400], nocc=nmo/5, naux=3.5 nmo, seed " + str(seed)}


def bench_batched(args):
    """The batch as its own JSON line (one step = one batch replay)."""
    r = measure_batched(args.nsys, args.seed, args.steps, args.warmup, args.branches)
    out = {
        "metric": "sigma_moment_sets_per_s", "value": r["sets_per_s"], "unit": "sets/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_replay"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "i8-digits/i32-acc/f64", "data": "synthetic",
        "config": {"workload": r["workload"] + "; one step = one batch", "nsys": r["nsys"], "nmom_max": 7,
                   "seed": args.seed},
    }
    out.update({k: r[k] for k in ("sequential_sets_per_s", "speedup_vs_sequential", "sequential_fp64_sets_per_s",
                                  "speedup_vs_sequential_fp64", "plan_seconds", "plan", "useful_tflops")})
    print(json.dumps(out), flush=True)


def bench_evgw(args):
    """evGW at the c3 size: wall time and iterations of the device loop in
    FP64 and in mixed precision (one JSON line; not the headline metric)."""
    import torch
    import gwsynth
    from paper_2504_17439_amd import gwmom

    o, v, A, N = args.nocc, args.nvir, args.naux, args.nmom
    print(f"[bench] evgw inputs o={o} v={v} A={A} N={N}", file=sys.stderr, flush=True)
    eps, L = gwsynth.system(o, v, A, args.seed)
    h = gwmom.Handle(0)
    e = torch.from_numpy(eps).to("cuda:0")
    l = torch.from_numpy(L).to("cuda:0")
    del L
    out = {"metric": "evgw_seconds", "unit": "s", "higher_is_better": False, "n_gpus": 1,
           "config": {"workload": f"evGW, TDA, nocc={o} nvir={v} naux={A} nmom_max={N}", "tol_ha": 1e-6}}
    for prec in ("fp64", "mixed"):
        opts = {"moment_eps": 1e-9} if prec == "mixed" else None
        h.sigma_moments(e, l, o, N, "tda", prec)       # warm-up (workspace, code objects)
        torch.cuda.synchronize()
        print(f"[bench] evgw {prec}", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        r = h.evgw(e, l, o, N, "tda", prec, tol=1e-6, max_iter=20, opts=opts, allow_noconv=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        q = r["qp"].cpu().numpy()
        out[prec] = {"seconds": el, "iterations": r["iterations"], "converged": r["converged"],
                     "seconds_per_iteration": el / max(r["iterations"], 1), "last_change": r["last_change"],
                     "homo_lumo_qp": [float(q[o - 1]), float(q[o])]}
    out["frontier_qp_diff_mixed_vs_fp64"] = max(abs(out["mixed"]["homo_lumo_qp"][i] - out["fp64"]["homo_lumo_qp"][i])
                                               for i in range(2))
    print(json.dumps(out), flush=True)


def bench_qsgw(args):
    """qsGW (SRG) at the c3 size: wall time and iterations of the device loop
    with FP64 and with mixed self-energy moments (one JSON line; not the
    headline metric)."""
    import torch
    import gwsynth
    from paper_2504_17439_amd import gwmom

    o, v, A, N = args.nocc, args.nvir, args.naux, args.nmom
    print(f"[bench] qsgw inputs o={o} v={v} A={A} N={N}", file=sys.stderr, flush=True)
    eps, L = gwsynth.system(o, v, A, args.seed)
    h = gwmom.Handle(0)
    e = torch.from_numpy(eps).to("cuda:0")
    l = torch.from_numpy(L).to("cuda:0")
    del L
    out = {"metric": "qsgw_seconds", "unit": "s", "higher_is_better": False, "n_gpus": 1,
           "config": {"workload": f"qsGW (SRG s=500), TDA, nocc={o} nvir={v} naux={A} nmom_max={N}",
                      "tol_ha": 1e-6}}
    for prec in ("fp64", "mixed"):
        opts = {"moment_eps": 1e-9} if prec == "mixed" else None
        h.sigma_moments(e, l, o, N, "tda", prec)       # warm-up (workspace, code objects)
        torch.cuda.synchronize()
        print(f"[bench] qsgw {prec}", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        r = h.qsgw(e, l, o, N, "tda", prec, tol=1e-6, max_iter=20, opts=opts, allow_noconv=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        q = r["qp"].cpu().numpy()
        out[prec] = {"seconds": el, "iterations": r["iterations"], "converged": r["converged"],
                     "scf_steps": r["scf_steps"], "seconds_per_iteration": el / max(r["iterations"], 1),
                     "last_change": r["last_change"], "homo_lumo": [float(q[o - 1]), float(q[o])]}
    out["frontier_diff_mixed_vs_fp64"] = max(abs(out["mixed"]["homo_lumo"][i] - out["fp64"]["homo_lumo"][i])
                                             for i in range(2))
    print(json.dumps(out), flush=True)


def bench_spectral(args):
    """Green's-function post-processing at the c3 size (one JSON line; not the
    headline metric): mixed self-energy moments and FP64 poles, then the
    spectral function over nomega frequencies (per orbital and total), the
    Aufbau filling and the electron-number shift of the auxiliary energies.
    gw_spectral (Lorentzian matrix + FP64 GEMM) is timed with HIP events on
    the handle's stream and set against the FP64 matrix peak (2 flops per
    orbital, state and frequency)."""
    import numpy as np
    import torch
    import gwsynth
    from paper_2504_17439_amd import gwmom

    o, v, A, N = args.nocc, args.nvir, args.naux, args.nmom
    M = o + v
    nw = args.nomega
    print(f"[bench] spectral inputs o={o} v={v} A={A} N={N} nomega={nw}", file=sys.stderr, flush=True)
    eps, L = gwsynth.system(o, v, A, args.seed)
    h = gwmom.Handle(0)
    e = torch.from_numpy(eps).to("cuda:0")
    l = torch.from_numpy(L).to("cuda:0")
    del L
    so, sv = h.sigma_moments(e, l, o, N, "tda", "mixed")
    fock = torch.diag(e).contiguous()
    p = h.poles(so, sv, fock, opts={"moment_eps": 1e-9})
    E, chi = p["E"], p["chi"]
    dim = E.shape[0]
    omega = torch.linspace(float(eps.min()) - 0.5, float(eps.max()) + 0.5, nw, dtype=torch.float64, device="cuda:0")
    delta = 0.01
    print(f"[bench] spectral dim={dim}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        h.spectral(E, chi, omega, delta, per_orbital=True)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        Atot, Ap = h.spectral(E, chi, omega, delta, per_orbital=True)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    flops = 2.0 * M * dim * nw                       # A_p(w) for every orbital, state and frequency
    peak = 78.6e12
    t0 = time.perf_counter()
    st = h.aufbau(E, chi, 2.0 * o)
    torch.cuda.synchronize()
    t_auf = time.perf_counter() - t0
    t0 = time.perf_counter()
    z = h.zeta_shift(p, fock, 2.0 * o)
    torch.cuda.synchronize()
    t_zeta = time.perf_counter() - t0
    q0, qz = p["qp"].cpu().numpy(), z["qp"].cpu().numpy()
    out = {"metric": "spectral_function_ms", "value": ms, "unit": "ms", "higher_is_better": False, "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"spectral function, TDA mixed moments, nocc={o} nvir={v} naux={A} "
                                  f"nmom_max={N}, nomega={nw}, delta={delta}", "dim": dim},
           "roofline": {"bound": "mfma", "achieved": flops / (ms * 1e-3) / 1e12, "peak": peak / 1e12,
                        "unit": "TFLOP/s", "frac": flops / (ms * 1e-3) / peak, "traffic": None},
           "aufbau": {"seconds": t_auf, "nfill": st["nfill"], "nelec": st["nelec"], "mu": st["mu"]},
           "zeta_shift": {"seconds": t_zeta, "zeta": z["zeta"], "nelec": z["nelec"], "eig_calls": z["eig_calls"],
                          "max_qp_shift": float(np.abs(qz - q0).max()),
                          "frontier_qp_shift": float(max(abs(qz[o - 1] - q0[o - 1]), abs(qz[o] - q0[o])))},
           "sum_rule_check": float(Atot.sum().item() * float(omega[1] - omega[0]) / M)}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="single", choices=["single", "batched", "evgw", "qsgw", "spectral"])
    ap.add_argument("--nomega", type=int, default=2048, help="spectral: frequencies")
    ap.add_argument("--nsys", type=int, default=64)
    ap.add_argument("--branches", type=int, default=4, help="batched: concurrent per-molecule streams")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--nocc", type=int, default=100)
    ap.add_argument("--nvir", type=int, default=400)
    ap.add_argument("--naux", type=int, default=1500)
    ap.add_argument("--nmom", type=int, default=11)
    ap.add_argument("--screening", default="tda", choices=["tda", "rpa"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", default="both", choices=["both", "mixed", "fp64"],
                    help="both: time the mixed form (the reported value) and the FP64 form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="leave out the RPA and batched figures")
    ap.add_argument("--extra-steps", type=int, default=3, help="RPA sets / batch replays timed")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design, not implemented)",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "batched":
        bench_batched(args)
        return
    if args.workload == "evgw":
        bench_evgw(args)
        return
    if args.workload == "qsgw":
        bench_qsgw(args)
        return
    if args.workload == "spectral":
        bench_spectral(args)
        return

    import numpy as np
    import torch
    import gwsynth
    from paper_2504_17439_amd import gwmom

    o, v, A, N = args.nocc, args.nvir, args.naux, args.nmom
    M = o + v
    print(f"[bench] generating inputs o={o} v={v} A={A} N={N}", file=sys.stderr, flush=True)
    eps, L = gwsynth.system(o, v, A, args.seed)
    h = gwmom.Handle(0)
    e = torch.from_numpy(eps).to("cuda:0")
    l = torch.from_numpy(L).to("cuda:0")
    del L
    so = torch.empty(N + 1, M, M, dtype=torch.float64, device="cuda:0")
    sv = torch.empty_like(so)
    fams_all = ("sigma_fold", "sigma_contract", "recur_xvt", "recur_rv", "recur_rr", "recur_digits", "rpa_quad",
                "mixed_prep", "mixed_zdig")

    def run(screening, prec, steps, warmup):
        out = (torch.empty_like(so), torch.empty_like(sv))

        def step():
            h.sigma_moments(e, l, o, N, screening, prec, out=out)

        print(f"[bench] {screening} {prec}: warmup", file=sys.stderr, flush=True)
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        h.timing(True)
        h.timing_reset()
        print(f"[bench] {screening} {prec}: timed region ({steps} sets)", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        fams = {f: h.timing_read(f) for f in fams_all}
        h.timing(False)
        return out, (t1 - t0), fams

    def pole_error(pm, T_occ, T_vir):
        """Per-pole error of poles pm against FP64 moments T (P10 of the
        oracle's pins): the largest relative deviation, over n <= N and both
        sectors, of the moments sum_l v_pl v_ql e_l^n the poles reproduce."""
        errs = []
        for e_, v_, T in ((pm["e_occ"], pm["v_occ"], T_occ), (pm["e_vir"], pm["v_vir"], T_vir)):
            ee = e_.cpu().numpy()
            vv = v_.cpu().numpy()
            Tn = T.cpu().numpy()
            w = np.ones_like(ee)
            for n in range(N + 1):
                rec = (vv * w) @ vv.T
                errs.append(float(np.abs(rec - Tn[n]).max() / np.abs(Tn[n]).max()))
                w = w * ee
        return errs

    precs = ["mixed", "fp64"] if args.precision == "both" else [args.precision]
    results = {}
    for prec in precs:
        results[prec] = run(args.screening, prec, args.steps, args.warmup)
    head = precs[0]
    (so_h, sv_h), elapsed, fams = results[head]
    sets_per_s = args.steps / elapsed

    # dominant kernel: stage 1 of the self-energy contraction (the fold GEMM);
    # its algorithmic flops per set are (N+1) naux^2 nmo (nmo + 1): the
    # products R_t L over the symmetric orbital pairs x <= q
    fold_ms, fold_n = fams["sigma_fold"]
    launches_per_set = max(fold_n, 1) / args.steps
    avg_flops = (N + 1) * A * A * M * (M + 1.0) / launches_per_set
    avg_ms = fold_ms / max(fold_n, 1)
    achieved = avg_flops / (avg_ms * 1e-3)
    # the mixed fold runs on the int8 MFMA: its own dtype's dense peak (5.0 POP/s)
    peak = MI355X_PEAK["f64" if head == "fp64" else "i8"]
    roofline = {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12,
                "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None,
                "kernel": "sigma_fold_kernel" if head == "fp64" else "fold_mixed_kernel",
                "launch_ms": avg_ms, "launch_flops": avg_flops}
    # work the kernel issues: the symmetric (x, q) pairs are formed once, in
    # 8 x 8 blocks of the upper block triangle (diagonal blocks whole)
    nb = (M + 7) // 8
    cols = nb * (nb + 1) // 2 * 64
    if head == "mixed":
        # ten int8 digit products per multiply-add over the padded aux range
        Ap = (A + 63) // 64 * 64
        issued = 2.0 * 10 * (N + 1) * Ap * Ap * cols / launches_per_set
        roofline["issued_tflops"] = issued / (avg_ms * 1e-3) / 1e12
        roofline["issued_frac"] = issued / (avg_ms * 1e-3) / peak
        roofline["traffic"] = recorded_traffic(o, v, A, N)
    else:
        issued = 2.0 * (N + 1) * A * A * cols / launches_per_set
        roofline["issued_tflops"] = issued / (avg_ms * 1e-3) / 1e12
        roofline["issued_frac"] = issued / (avg_ms * 1e-3) / peak

    out = {
        "metric": "sigma_moment_sets_per_s",
        "value": sets_per_s,
        "unit": "sets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head == "fp64" else "i8-digits/i32-acc/f64",
        "data": "synthetic",
        "config": {"workload": f"single molecule {args.screening.upper()} self-energy moment set, nocc={o} "
                               f"nvir={v} naux={A} nmom_max={N} (the mixed-vs-FP64 configuration)",
                   "nocc": o, "nvir": v, "naux": A, "nmom_max": N, "screening": args.screening,
                   "precision": head, "seed": args.seed},
        "roofline": roofline,
        "useful_tflops": set_flops(o, v, A, N) * sets_per_s / 1e12,
        "kernel_ms_per_set": {k: ms / args.steps for k, (ms, n) in fams.items() if n},
    }
    fock = torch.diag(e).contiguous()
    if "fp64" in results:
        (so64, sv64), el64, f64 = results["fp64"]
        out["fp64_sets_per_s"] = args.steps / el64
        out["fp64_kernel_ms_per_set"] = {k: ms / args.steps for k, (ms, n) in f64.items() if n}
        torch.cuda.synchronize()
        try:
            # the first call also sizes the workspaces and starts the
            # companion stream; the second is the steady-state cost
            for key in ("poles_first_ms", "poles_ms"):
                tp0 = time.perf_counter()
                ref = h.poles(so64, sv64, fock)
                torch.cuda.synchronize()
                out[key] = 1e3 * (time.perf_counter() - tp0)
        except gwmom.GWError as ex:
            ref = None
            out["poles_error"] = str(ex)
        if head == "mixed":
            out["speedup_vs_fp64"] = sets_per_s / out["fp64_sets_per_s"]
            a, b = so_h.cpu().numpy(), so64.cpu().numpy()
            c, d = sv_h.cpu().numpy(), sv64.cpu().numpy()
            out["moment_rel_err"] = [float(max(np.abs(a[n] - b[n]).max() / np.abs(b[n]).max(),
                                               np.abs(c[n] - d[n]).max() / np.abs(d[n]).max()))
                                     for n in range(N + 1)]
            try:
                mres = h.poles(so_h, sv_h, fock, opts={"moment_eps": 1e-9})
                perr = pole_error(mres, so64, sv64)
                out["pole_moment_err"] = perr
                out["pole_moment_err_max"] = max(perr)
                if ref is not None:
                    # the FP64 poles' own reconstruction of the FP64 moments, for reference
                    out["pole_moment_err_fp64_max"] = max(pole_error(ref, so64, sv64))
                if ref is not None:
                    q64 = ref["qp"].cpu().numpy()
                    w64 = ref["qp_weight"].cpu().numpy()
                    qm = mres["qp"].cpu().numpy()
                    front = [p for p in range(max(0, o - 5), min(M, o + 5)) if w64[p] >= 0.9]
                    out["qp_err_frontier_ha"] = float(np.abs(qm[front] - q64[front]).max())
                    out["qp_frontier_orbitals"] = front
                    out["homo_lumo_qp"] = [float(q64[o - 1]), float(q64[o])]
            except gwmom.GWError as ex:
                out["mixed_poles_error"] = str(ex)
        elif ref is not None:
            out["homo_lumo_qp"] = [float(ref["qp"][o - 1]), float(ref["qp"][o])]
    if not args.no_extra and args.screening == "tda":
        # RPA screening at the same size: the FP64 quadrature of the zeroth
        # moment in both forms, the recursion and contractions mixed or FP64
        rpa = {}
        for prec in ("mixed", "fp64"):
            _, el_r, fr = run("rpa", prec, args.extra_steps, 1)
            rpa[prec] = {"sets_per_s": args.extra_steps / el_r,
                         "kernel_ms_per_set": {k: ms / args.extra_steps for k, (ms, n) in fr.items() if n}}
        out["rpa_sets_per_s"] = rpa["mixed"]["sets_per_s"]
        out["rpa_fp64_sets_per_s"] = rpa["fp64"]["sets_per_s"]
        out["rpa_speedup_vs_fp64"] = rpa["mixed"]["sets_per_s"] / rpa["fp64"]["sets_per_s"]
        out["rpa_kernel_ms_per_set"] = rpa["mixed"]["kernel_ms_per_set"]
        out["rpa_fp64_kernel_ms_per_set"] = rpa["fp64"]["kernel_ms_per_set"]
        out["rpa_steps"] = args.extra_steps
    h.close()
    del e, l, so, sv, results, so_h, sv_h
    torch.cuda.empty_cache()
    if not args.no_extra and args.screening == "tda":
        r = measure_batched(args.nsys, args.seed, args.extra_steps, 1, args.branches)
        out["batched_sets_per_s"] = r["sets_per_s"]
        out["batched"] = {k: r[k] for k in ("ms_per_replay", "replays", "nsys", "sequential_sets_per_s",
                                            "speedup_vs_sequential", "sequential_fp64_sets_per_s",
                                            "speedup_vs_sequential_fp64", "plan_seconds", "useful_tflops",
                                            "workload")}
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(o, v, A, N, args.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
