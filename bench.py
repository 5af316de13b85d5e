#!/usr/bin/env python3
"""Throughput of the CTMRG step (Sec. 3, Algorithm 3) for the q=20 dodecahedron model on one MI355X.

A step is one full pass of the method on the GPU: extension products and W-mix
(the extended corner C', (q m) x (q m)), the FP64 diagonalization (the m leading
eigenpairs and the normalization n_C over the whole spectrum), the
multiplet-preserving cut, the half-row products, W-mix and projection, and the
normalizations.  Every step works on the full padded size N = q m.  Inputs are
the dodecahedron spin vectors and K = 1/T; the state is whatever the iteration
produces from the fixed boundary (synthetic, deterministic).

Four paths are timed one after the other from the same initial state: FP32 or
FP64 contractions (the mixed path keeps the eigensolver, the state and every
normalization in FP64), each with the two-stage eigensolver (all eigenvalues
every step) and with the warm-started one (the leading m + p eigenpairs from the
previous step's, n_C from ||C'^2||_F where the bounded tail could matter).  The
headline `value` is the mixed path with the warm-started eigensolver;
`mixed_over_fp64` divides it by the plain FP64 path (two-stage), and
`mixed_vs_fp64_after_run` gives how far their observables are apart after the
same steps.  `paths` holds all four, `roofline` the dominant kernel of the
headline path (the products C' V, timed by HIP events around each launch),
`two_stage_roofline` the dominant kernel of the two-stage path (the wavefront
bulge chasing), `contraction_roofline` the largest contraction kernel,
`kept_subspace_mixed_vs_fp64` the largest principal angle between the kept eigenvectors of
one mixed and one FP64 step from the same state against the eigen-gap at the cut,
`time_to_fixed_point` whole runs at m = 64 against the oracle's fixed point, and
`cpu_baseline` the oracle's step time on the host.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 (vector and matrix)
PEAK_FP32_TFLOPS = 157.3  # MI355X dense FP32 matrix
PEAK_BF16_TFLOPS = 2500.0  # MI355X dense bf16 matrix
PEAK_HBM_GBS = 8000.0


def stage_flops(q: int, m: int):
    """Algorithmic flop counts of the single-launch contraction kernels of one step."""
    N = q * m
    return {
        "extension": 2.0 * N * N * m,            # X = A^T (Omega A)
        "wmix_C": 2.0 * q ** 4 * m * m,          # C' = W-mix(X)
        "halfrow": 2.0 * N * N * m,              # Y = A^T U~
        "wmix_Z": 2.0 * q ** 4 * m * m,          # Z = W-mix(Y)
        "projection": 2.0 * m * N * N,           # P~ = U^T Z
    }


def bulge_chasing_bytes(N: int, b: int):
    """Launches of the wavefront bulge-chasing kernel and their algorithmic HBM bytes.

    Sweep j (j = 0 .. N-3) has ns(j) = 1 + (N-3-j) // b steps.  Step (j, t) reads and
    writes its three blocks of the band, in doubles: the left block (len x ncl, whose
    first column is annihilated), the lower triangle of the diagonal block
    (len (len+1) / 2) and the block below (nbl x len); it also writes its reflector
    (b doubles) and tau.  One launch runs all steps with 3 j + t = tau; there are
    3 (N-3) + ns(N-3) launches.
    """
    import numpy as np
    j = np.arange(N - 2, dtype=np.int64)
    ns = 1 + (N - 3 - j) // b
    total = 0.0
    for t in range(int(ns.max())):
        jj = j[ns > t]
        if t == 0:
            r0, ncl = jj + 1, 1
        else:
            r0, ncl = jj + 1 + t * b, b
        ln = np.minimum(r0 + b, N) - r0
        n0 = r0 + ln
        nbl = np.minimum(n0 + b, N) - n0
        doubles = 2 * (ln * ncl + ln * (ln + 1) // 2 + nbl * ln) + b + 1
        total += 8.0 * float(doubles.sum())
    launches = 3 * (N - 3) + int(ns[-1])
    return launches, total


def host_cpu():
    """The host's CPU model, physical cores and the CPUs this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        import psutil
        phys = psutil.cpu_count(logical=False)
    except Exception:
        phys = None
    try:
        usable = len(os.sched_getaffinity(0))
    except Exception:
        usable = os.cpu_count()
    return {"model": model, "physical_cores": phys, "usable_cpus": usable}


def cpu_baseline(q_vectors, K, m_sample, m_target):
    """One oracle step (its own Jacobi eigensolver, FP64) measured on the host at m_sample, from the
    state the fixed-boundary iteration reaches once the kept dimension is full (three steps:
    1 -> 20 -> 400 -> m_sample states).  The measured figure is `value`; an O(m^3) scaling to
    m_target is reported separately and labelled as such."""
    from oracle import ctmrg_oracle as O
    o = O.OracleCTMRG(q_vectors, K, m_sample)
    while o.P.shape[1] < m_sample:
        o.step()
    warm = o.k
    t0 = time.perf_counter()
    o.step()
    dt = time.perf_counter() - t0
    cpu = host_cpu()
    scale = (m_target / m_sample) ** 3
    return {
        "value": 1.0 / dt,
        "unit": "steps/s",
        "cores": O.num_threads(),
        "kind": "oracle",
        "sample": (f"one oracle step (Jacobi eigensolver, FP64) at q=20, m={m_sample} (C' {20 * m_sample}^2), "
                   f"T={1.0 / K:.4f}, from the state after {warm} steps, measured: {dt:.2f} s"),
        "m": m_sample,
        "seconds_per_step": dt,
        "cpu_model": cpu["model"],
        "physical_cores": cpu["physical_cores"],
        "usable_cpus": cpu["usable_cpus"],
        "threads": O.num_threads(),
        "extrapolated_to_m": {"m": m_target, "steps_per_s": 1.0 / (dt * scale),
                              "basis": f"the measured step times (m/{m_sample})^3 = {scale:.0f} (not measured)"},
    }


def run_path(V, K, m, band, precision, gap_tol, warmup, steps, eig="two_stage", warm_tol=0.0):
    """Warm up, then time `steps` CTMRG steps of one context; per-stage HIP-event times, and for
    the warm-started eigensolver its counters over the timed steps and the HIP-event times of
    its products C' V."""
    import torch
    from paper_2004_08669_amd import ctmrg
    g = ctmrg.CTMRG(V, K, m, band=band, precision=precision, gap_tol=gap_tol, eig=eig, warm_tol=warm_tol)
    tag = f"{precision}/{eig}"
    for i in range(warmup):
        g.step(1)
        print(f"# {tag} warmup step {i + 1}/{warmup}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    g.set_profiling(True)
    before = g.eig_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        g.step(1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print(f"# {tag}: {steps} steps in {t1 - t0:.3f} s", file=sys.stderr, flush=True)
    stages, nsteps = g.stage_times()
    after = g.eig_stats()
    obs = g.observables()
    g.close()
    dt = t1 - t0
    out = {
        "steps_per_s": steps / dt,
        "ms_per_step": 1000.0 * dt / steps,
        "stage_ms": {k: v / max(1, nsteps) for k, v in stages.items()},
        "obs": obs,
    }
    if eig == "warm":
        ws = after["warm_steps"] - before["warm_steps"]
        fb = after["fallback_steps"] - before["fallback_steps"]
        out["warm"] = {
            "timed_steps": steps,
            "warm_steps": ws,
            "fallback_steps": fb,
            "fallback_rate": fb / max(1, ws + fb),
            "passes_per_step": (after["passes"] - before["passes"]) / steps,
            "products_per_step": (after["products"] - before["products"]) / steps,
            "exact_tail_steps": after["exact_tails"] - before["exact_tails"],
            "tail_bound_last": after["tail_bound_last"],
            "last_residual": after["last_residual"],
            "product_ms": after["product_ms"],
            "product_flops": after["product_flops"],
            "product_launches": after["product_launches"],
        }
    return out


def time_to_fixed_point(V, T, m, tol, max_steps, band):
    """Wall time of whole runs to the fixed point (spectral change below tol) at q=20, m=64,
    from the fixed boundary, on three routes: FP64 with the two-stage eigensolver, FP64 with
    the warm-started one, and the mixed path (warm-started) to its FP32 noise floor followed
    by FP64 polishing steps (counted).  f, E, M and S_E are compared with the oracle's fixed
    point stored in tests/golden (same m, T and tolerance)."""
    import numpy as np
    import torch
    from paper_2004_08669_amd import ctmrg
    K = 1.0 / T
    path = os.path.join(ROOT, "tests", "golden", f"fixedpoint_q20_m{m}_T{T:.2f}.npz")
    ref = None
    if os.path.exists(path):
        with np.load(path, allow_pickle=False) as z:
            ref = {k: z[k] for k in z.files}

    def errs(ob):
        if ref is None:
            return None
        return {"f_rel": abs(ob["f"] - float(ref["f"])) / abs(float(ref["f"])),
                "E_abs": abs(ob["E"] - float(ref["E"])), "M_abs": abs(ob["M"] - float(ref["M"])),
                "S_E_abs": abs(ob["S_E"] - float(ref["S_E"])), "m_eff": [ob["m_eff"], int(ref["m_eff"])]}

    out = {"m": m, "T": T, "tol": tol, "max_steps": max_steps,
           "reference": (f"oracle fixed point (FP64, Jacobi / LAPACK eigensolver), {int(ref['steps'])} steps"
                         if ref is not None else None)}
    for name, prec, eig in (("fp64_two_stage", "fp64", "two_stage"), ("fp64_warm", "fp64", "warm")):
        g = ctmrg.CTMRG(V, K, m, band=band, precision=prec, eig=eig)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ks, d, conv = g.run_to_fixed_point(tol, max_steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ob = g.observables()
        st = g.eig_stats()
        g.close()
        out[name] = {"seconds": dt, "steps": ks, "delta": d, "converged": bool(conv), "vs_oracle": errs(ob)}
        if eig == "warm":
            out[name]["fallback_steps"] = st["fallback_steps"]
        print(f"# time to fixed point {name}: {ks} steps, {dt:.2f} s", file=sys.stderr, flush=True)
    # mixed to its noise floor (gap tolerance 1e-6, change below 1e-6), then FP64 polishing
    g = ctmrg.CTMRG(V, K, m, band=band, precision="fp32", gap_tol=1e-6, eig="warm")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    k1, d1, c1 = g.run_to_fixed_point(1e-6, max_steps)
    st = g.export_state()
    g.close()
    h = ctmrg.CTMRG(V, K, m, band=band, precision="fp64", eig="warm")
    h.import_state(st)
    k2, d2, c2 = h.run_to_fixed_point(tol, max_steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ob = h.observables()
    h.close()
    out["mixed_then_fp64_warm"] = {"seconds": dt, "steps": k1 + k2, "mixed_steps": k1, "fp64_steps": k2,
                                   "delta": d2, "converged": bool(c1 and c2), "vs_oracle": errs(ob)}
    print(f"# time to fixed point mixed+polish: {k1}+{k2} steps, {dt:.2f} s", file=sys.stderr, flush=True)
    return out


def subspace_angle(V, K, m, band, gap_tol, warmup, precision="fp32"):
    """The kept subspace of a mixed path against the FP64 path's, from the same FP64 state
    (after `warmup` FP64 steps): one step of each, the largest principal angle between the
    kept eigenvectors U (sin theta from the singular values of U_mixed^T U_fp64), the eigen-gap
    at the cut |lambda_m_eff| - |lambda_m_eff+1| of C', and the Davis-Kahan bound
    ||C'_mixed - C'_fp64||_2 / gap (the spectral norm bounded by the Frobenius norm)."""
    import numpy as np
    from paper_2004_08669_amd import ctmrg
    a = ctmrg.CTMRG(V, K, m, band=band, gap_tol=gap_tol)
    a.step(warmup)
    st = a.export_state()
    a.extend()
    Ca = a.get("cext")
    a.import_state(st)
    a.step(1)
    Ua, lam = a.get("U"), a.get("spectrum")
    me_a = int(np.count_nonzero(a.get("omega")))
    a.close()
    b = ctmrg.CTMRG(V, K, m, band=band, precision=precision, gap_tol=gap_tol)
    b.import_state(st)
    b.extend()
    Cb = b.get("cext")
    b.import_state(st)
    b.step(1)
    Ub = b.get("U")
    me_b = int(np.count_nonzero(b.get("omega")))
    b.close()
    me = min(me_a, me_b)
    s = np.linalg.svd(Ua[:, :me].T @ Ub[:, :me], compute_uv=False)
    sin_max = float(np.sqrt(max(0.0, 1.0 - float(s.min()) ** 2)))
    mags = np.sort(np.abs(lam))[::-1]
    l1 = float(mags[0])
    gap = float(mags[me - 1] - mags[me])
    dC = float(np.linalg.norm(Ca - Cb))
    return {"precision": precision, "gap_tol": gap_tol, "after_fp64_steps": warmup, "m_eff": [me_a, me_b],
            "sin_theta_max": sin_max,
            "eigen_gap_rel": gap / l1, "dC_fro_rel": dC / l1, "davis_kahan_bound": dC / gap if gap > 0 else None}


EIGEN_STAGES = ["dense_to_band", "band_to_tridiag", "bisection", "select_cut_entropy", "inverse_iteration",
                "orthonormalize", "backtransform_band", "backtransform_dense"]


def eigh_comparison(V, K, m, band, warmup):
    """Timed comparison only: the vendor dense symmetric eigensolver (torch.linalg on ROCm, hipSOLVER /
    rocSOLVER syevd) on an extended corner C' of the same workload.  Not part of the CTMRG path."""
    import torch
    from paper_2004_08669_amd import ctmrg as ct

    g = ct.CTMRG(V, K, m, band=band, precision="fp64")
    g.step(warmup)
    g.extend()
    C = torch.from_numpy(g.get("cext")).cuda()
    g.close()
    try:
        torch.backends.cuda.preferred_linalg_library("cusolver")
    except Exception:
        pass
    lib = str(torch.backends.cuda.preferred_linalg_library())
    out = {"n": int(C.shape[0]), "torch_linalg_library": lib}
    for name, fn in (("values", torch.linalg.eigvalsh), ("values_and_vectors", torch.linalg.eigh)):
        fn(C)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn(C)
        e1.record()
        torch.cuda.synchronize()
        out[f"syevd_{name}_ms"] = e0.elapsed_time(e1)
        print(f"# vendor eigensolver, {name}: {out[f'syevd_{name}_ms']:.1f} ms", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=16,
                    help="untimed steps; the kept dimension settles at m after about 12 steps from the boundary")
    ap.add_argument("--m", type=int, default=512)
    ap.add_argument("--T", type=float, default=0.4398)
    ap.add_argument("--band", type=int, default=16)
    ap.add_argument("--precision", choices=["both", "fp32", "fp64"], default="both",
                    help="both: time the mixed path (the headline value) and the FP64 path")
    ap.add_argument("--gap-tol", type=float, default=1e-6,
                    help="multiplet gap of the cut, the same on both paths")
    ap.add_argument("--eig", choices=["both", "two_stage", "warm"], default="both",
                    help="both: the two-stage and the warm-started eigensolver (the headline is the warm one)")
    ap.add_argument("--no-fixed-point", action="store_true", help="skip the time-to-fixed-point runs (m=64)")
    ap.add_argument("--no-subspace", action="store_true", help="skip the kept-subspace angle of mixed vs FP64")
    ap.add_argument("--warm-tol", type=float, default=0.0,
                    help="residual tolerance of the warm-started solver on the mixed paths (0: the library default)")
    ap.add_argument("--no-bf16x3", action="store_true",
                    help="skip the split-bf16 path (contractions as three bf16 products, warm-started eigensolver)")
    ap.add_argument("--gap-tol-bf16x3", type=float, default=1e-6,
                    help="multiplet gap of the cut on the split-bf16 path (default: the same cut rule as the other "
                         "paths; at m=512 the gaps at the cut, ~2e-6 |lambda_1|, are below its rounding, and a wider "
                         "gap merges the tail and cuts far below m)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-m", type=int, default=128)
    ap.add_argument("--compare-eigh", action="store_true",
                    help="also time the vendor syevd (torch.linalg.eigh on ROCm) on a C' of the same workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the CTMRG step of one (T, m) problem runs on a single MI355X "
              f"(independent temperatures would shard with no communication); --gpus {args.gpus} is not run.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import ctmrg_inputs as I

    torch.cuda.set_device(0)
    V = I.dodecahedron()
    q, m, K = len(V), args.m, 1.0 / args.T
    print(f"# bench: q={q} m={m} T={args.T} warmup={args.warmup} steps={args.steps}", file=sys.stderr, flush=True)
    order = ["fp32", "fp64"] if args.precision == "both" else [args.precision]
    ts, wm = {}, {}
    if args.eig != "warm":
        for prec in order:
            ts[prec] = run_path(V, K, m, args.band, prec, args.gap_tol, args.warmup, args.steps)
    if args.eig != "two_stage":
        for prec in order:
            wm[prec] = run_path(V, K, m, args.band, prec, args.gap_tol, args.warmup, args.steps, eig="warm",
                                warm_tol=args.warm_tol if prec != "fp64" else 0.0)
    x3 = None
    if not args.no_bf16x3 and args.eig != "two_stage" and "fp32" in order:
        x3 = run_path(V, K, m, args.band, "bf16x3", args.gap_tol_bf16x3, args.warmup, args.steps, eig="warm",
                      warm_tol=args.warm_tol)
    # the headline: the mixed path (the first precision) with the warm-started eigensolver when it ran
    head_eig = "warm" if wm else "two_stage"
    head_prec = order[0]
    head = (wm if wm else ts)[head_prec]
    stage_ms = head["stage_ms"]
    obs = head["obs"]

    flops = stage_flops(q, m)

    def product_roofline(w):
        """The warm solver's products C' V (split-K gemm_mfma_kernel<128, 128> and its partial
        sum), each bracketed by HIP events on the stream that runs it."""
        if w["product_launches"] <= 0:
            return None
        avg_s = w["product_ms"] * 1e-3 / w["product_launches"]
        fl = w["product_flops"] / w["product_launches"]
        ach = fl / avg_s / 1e12
        return {"kernel": "gemm_mfma_kernel<128, 128, 16, 4, 2, A_RM<double>, B_RM<double>, EpiPartial> + partial sum "
                          "(products C' V of the warm solver)",
                "bound": "mfma", "achieved": ach, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / PEAK_FP64_TFLOPS, "traffic": None, "algorithmic_flops_per_launch": fl,
                "avg_launch_ms": avg_s * 1e3, "launches": w["product_launches"]}

    def bulge_roofline(st):
        """The wavefront bulge-chasing kernel (band -> tridiagonal) of the two-stage solver: its
        stage's HIP-event time (the launches plus one band extraction of a few microseconds) over
        its launches."""
        N = q * m
        launches, bulge_bytes = bulge_chasing_bytes(N, args.band)
        avg_launch_s = st["band_to_tridiag"] * 1e-3 / launches
        per_launch = bulge_bytes / launches
        achieved = per_launch / avg_launch_s / 1e9
        return {"kernel": f"bulge_front_kernel<{args.band}>", "bound": "hbm", "achieved": achieved,
                "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                "algorithmic_bytes_per_launch": per_launch, "launches_per_step": launches,
                "avg_launch_us": avg_launch_s * 1e6}

    roofline = product_roofline(head["warm"]) if head_eig == "warm" else bulge_roofline(stage_ms)
    # The largest contraction kernel, against the matrix-core peak of its precision.
    kernel_stages = ["extension", "wmix_C", "halfrow", "wmix_Z", "projection"]
    dom = max(kernel_stages, key=lambda k: stage_ms[k])
    c_ach = flops[dom] / (stage_ms[dom] * 1e-3) / 1e12
    c_peak = PEAK_FP32_TFLOPS if head_prec == "fp32" else PEAK_FP64_TFLOPS
    contraction_roofline = {
        "kernel": dom,
        "bound": "mfma",
        "achieved": c_ach,
        "peak": c_peak,
        "unit": "TFLOP/s",
        "frac": c_ach / c_peak,
        "algorithmic_flops_per_launch": flops[dom],
        "avg_launch_ms": stage_ms[dom],
        "all": {k: round(flops[k] / (stage_ms[k] * 1e-3) / 1e12 / c_peak, 4) for k in kernel_stages
                if stage_ms[k] > 0},
    }
    desc = {"fp32": "mixed (FP32 contractions, FP64 eigensolver and state)", "fp64": "FP64"}
    edesc = {"two_stage": "two-stage eigensolver (all eigenvalues every step)",
             "warm": "warm-started top-m eigensolver (two-stage solver in the first steps and as fallback)"}
    out = {
        "metric": "CTMRG steps/s at q=20 m=512 (mixed vs FP64, same error); % MFMA peak",
        "value": head["steps_per_s"],
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32+f64" if head_prec == "fp32" else "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"CTMRG step, q=20 dodecahedron, m={m} (C' {q * m}x{q * m}), T={args.T}, fixed boundary, "
                         f"{desc[head_prec]}, {edesc[head_eig]}"),
            "q": q, "m": m, "T": args.T, "precision": head_prec, "band": args.band, "gap_tol": args.gap_tol,
            "warm_tol": args.warm_tol if args.warm_tol > 0 else "default",
            "eigensolver": head_eig,
        },
        "roofline": roofline,
        "contraction_roofline": contraction_roofline,
        "stages_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "state": {"m_eff": obs["m_eff"], "S_E": obs["S_E"], "xi_e": obs["xi_e"], "delta": obs["delta"]},
    }

    def after_run(a, b):
        return {"f_rel": abs(a["f"] - b["f"]) / abs(b["f"]), "E_abs": abs(a["E"] - b["E"]),
                "M_abs": abs(a["M"] - b["M"]), "S_E_abs": abs(a["S_E"] - b["S_E"]), "m_eff": [a["m_eff"], b["m_eff"]]}

    paths = {}
    for solver, rr in (("two_stage", ts), ("warm", wm)):
        for prec, r in rr.items():
            ent = {"steps_per_s": r["steps_per_s"], "ms_per_step": r["ms_per_step"],
                   "stages_ms": {k: round(v, 4) for k, v in r["stage_ms"].items() if v > 0}}
            if "warm" in r:
                ent.update({k: r["warm"][k] for k in ("fallback_steps", "warm_steps", "fallback_rate",
                                                      "passes_per_step", "products_per_step", "exact_tail_steps",
                                                      "tail_bound_last", "last_residual")})
                if prec in ts:
                    ent["speedup_vs_two_stage"] = r["steps_per_s"] / ts[prec]["steps_per_s"]
                    ent["vs_two_stage_after_run"] = after_run(r["obs"], ts[prec]["obs"])
            paths[f"{prec}_{solver}"] = ent
    if x3 is not None:
        ent = {"steps_per_s": x3["steps_per_s"], "ms_per_step": x3["ms_per_step"], "gap_tol": args.gap_tol_bf16x3,
               "stages_ms": {k: round(v, 4) for k, v in x3["stage_ms"].items() if v > 0}}
        ent.update({k: x3["warm"][k] for k in ("fallback_steps", "warm_steps", "fallback_rate", "passes_per_step",
                                               "products_per_step", "exact_tail_steps", "last_residual")})
        if "fp32" in wm:
            ent["speedup_vs_fp32_warm"] = x3["steps_per_s"] / wm["fp32"]["steps_per_s"]
        if "fp64" in ts:
            ent["vs_fp64_two_stage_after_run"] = after_run(x3["obs"], ts["fp64"]["obs"])
        # the split-bf16 contractions against the bf16 matrix-core peak (three bf16 products per
        # algorithmic multiply-add) and as FP32-equivalent rates against the FP32 peak
        xs = x3["stage_ms"]
        ent["contraction_roofline"] = {
            "peak_bf16_tflops": PEAK_BF16_TFLOPS,
            "bf16_mfma_frac": {k: round(3.0 * flops[k] / (xs[k] * 1e-3) / 1e12 / PEAK_BF16_TFLOPS, 4)
                               for k in kernel_stages if xs.get(k, 0) > 0},
            "fp32_equivalent_tflops": {k: round(flops[k] / (xs[k] * 1e-3) / 1e12, 2)
                                       for k in kernel_stages if xs.get(k, 0) > 0},
            "fp32_path_tflops": {k: round(flops[k] / (stage_ms[k] * 1e-3) / 1e12, 2)
                                 for k in kernel_stages if stage_ms.get(k, 0) > 0} if head_prec == "fp32" else None,
        }
        paths["bf16x3_warm"] = ent
    out["paths"] = paths
    if "fp64" in ts and head_prec != "fp64":
        # the plain FP64 path: FP64 contractions and the two-stage eigensolver; all paths ran the same
        # steps from the same initial state
        out["mixed_over_fp64"] = head["steps_per_s"] / ts["fp64"]["steps_per_s"]
        out["mixed_over_fp64_basis"] = (f"the headline path ({desc[head_prec]}, {head_eig}) over the plain FP64 "
                                        f"path (two-stage eigensolver)")
        out["mixed_vs_fp64_after_run"] = after_run(obs, ts["fp64"]["obs"])
        ratios = {}
        for solver, rr in (("two_stage", ts), ("warm", wm)):
            if "fp32" in rr and "fp64" in rr:
                ratios[f"mixed_over_fp64_both_{solver}"] = rr["fp32"]["steps_per_s"] / rr["fp64"]["steps_per_s"]
        out["ratios"] = ratios
    if ts:
        out["two_stage_roofline"] = bulge_roofline(ts[order[0]]["stage_ms"])
    if "fp32" in order and "fp64" in order and not args.no_subspace:
        out["kept_subspace_mixed_vs_fp64"] = subspace_angle(V, K, m, args.band, args.gap_tol, args.warmup)
        if x3 is not None:
            out["kept_subspace_bf16x3_vs_fp64"] = subspace_angle(V, K, m, args.band, args.gap_tol_bf16x3,
                                                                 args.warmup, precision="bf16x3")
    if not args.no_fixed_point:
        out["time_to_fixed_point"] = time_to_fixed_point(V, 0.40, 64, 1e-12, 3000, args.band)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(V, K, args.cpu_sample_m, m)
    if args.compare_eigh:
        r64 = ts.get("fp64", head)
        cmp = eigh_comparison(V, K, m, args.band, args.warmup)
        cmp["own_eigensolver_ms"] = sum(r64["stage_ms"][k] for k in EIGEN_STAGES)
        cmp["own_eigensolver_computes"] = "all eigenvalues and the m leading eigenvectors"
        out["eigh_comparison"] = cmp
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
