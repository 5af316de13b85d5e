"""Temperature sweeps of the CTMRG fixed point with its K-derivatives (the scans of Sec. IV).

One context per cutoff m; each temperature starts from the previous one's fixed point
(ctmrg_sweep with warm start), and at every converged point the fixed-point derivative gives
dF/dK (the energy u per site), d2F/dK2 = dE/dK (the specific heat per site is
c = du/dT = -K^2 d2F/dK2) and dM/dK
along the fixed point.  Optional checks at every k-th temperature: dF/dK against the central
difference [F(K + dK) - F(K - dK)] / 2 dK over fixed points at K +- dK (started from the fixed
point at K, in a second context), and at every point against the impurity energy E.

A (T, m) grid is one context per cutoff, the cutoffs in order: `--m 120,240,500` or one of the two
cutoff sets of the paper's scaling analysis (Sec. IV: set A = {120, 240, 500, 800}, set B = {500,
600, 700, 800}, over 0.35 <= T <= 0.56 unless --T0/--T1 say otherwise).  The observables of every
point are M, S_E and xi_e (with f and E); the derivatives are optional there (--no-derivative).

Usage (from the repository root, on a gfx950 GPU):

  python -m paper_2004_08669_amd.sweep --m 128 --T0 0.40 --T1 0.48 --n 41 --fd-every 10 \\
      --out sweep_m128.json
  python -m paper_2004_08669_amd.sweep --set A --n 22 --no-derivative --fd-every 0 --out grid_a.json

All work runs in the library (ctmrg_sweep, ctmrg_fixed_point_derivative); this module only
marshals arguments and writes the JSON summary.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import ctmrg


def vertex_set(name: str) -> np.ndarray:
    import ctmrg_inputs as I
    return {"dodecahedron": I.dodecahedron, "icosahedron": I.icosahedron, "cube": I.cube,
            "tetrahedron": I.tetrahedron, "ising": I.ising}[name]()


# the two cutoff sets of the paper's finite-m scaling analysis (Sec. IV), and its temperature range
CUTOFF_SETS = {"A": (120, 240, 500, 800), "B": (500, 600, 700, 800)}
PAPER_T_RANGE = (0.35, 0.56)


def run(V, m: int, Ts, tol: float, max_steps: int, fd_every: int, dK: float, log=sys.stderr,
        precision: str = "fp64", eig: str = "two_stage", gap_tol=None, out_path=None, derivative: bool = True,
        on_point=None) -> dict:
    """The sweep on one context of the given contraction precision and eigensolver (the derivative
    itself always runs in FP64).  With out_path the summary is rewritten after every temperature;
    on_point(summary), when given, is called instead after every temperature."""
    Ts = [float(t) for t in Ts]
    g = ctmrg.CTMRG(V, 1.0 / Ts[0], m, precision=precision, eig=eig, gap_tol=gap_tol)
    points, checks = [], []
    t0 = time.perf_counter()
    for i, T in enumerate(Ts):
        # one temperature per call, so that progress is reported; with warm_start each call
        # continues from the fixed point the context holds (the boundary for the first)
        t1 = time.perf_counter()
        p = g.sweep([T], tol, max_steps, warm_start=True, derivative=derivative)[0]
        p["seconds"] = time.perf_counter() - t1
        points.append(p)
        line = (f"# m={m} T={T:.5f}: {p['steps']} steps (Delta {p['delta']:.2e}), f {p['f']:.12f} "
                f"E {p['E']:.10f} M {p['M']:.10f} S_E {p['S_E']:.8f} xi_e {p['xi_e']:.6f}")
        d = p.get("derivative")
        if d is not None:
            line += (f"; dF/dK {d['dF_dK']:.10f} d2F/dK2 {d['d2F_dK2']:.8f} dM/dK {d['dM_dK']:.8f} "
                     f"({d['iterations']} products J t, status {d['status']})")
        print(line + f", {p['seconds']:.1f} s", file=log, flush=True)
        if (d is not None and fd_every > 0 and i % fd_every == 0 and p["converged"] and d["status"] == 0
                and d["iterations"] > 0):
            # F at K +- dK over fixed points started from this one (a second context)
            K = 1.0 / T
            h = ctmrg.CTMRG(V, K, m, precision=precision, eig=eig, gap_tol=gap_tol)
            h.import_state(g.export_state())
            pair = h.sweep([1.0 / (K + dK), 1.0 / (K - dK)], tol, max_steps, warm_start=True)
            h.close()
            fd = ((K + dK) * pair[0]["f"] - (K - dK) * pair[1]["f"]) / (2 * dK)
            checks.append({"T": T, "dK": dK, "central_difference_dF_dK": fd, "dF_dK": d["dF_dK"],
                           "abs_diff": abs(d["dF_dK"] - fd), "converged": all(x["converged"] for x in pair)})
            print(f"# check T={T:.5f}: dF/dK {d['dF_dK']:.10f}, central difference {fd:.10f}", file=log, flush=True)
        if on_point is not None:
            on_point(_summary(V, m, tol, precision, eig, time.perf_counter() - t0, points, checks))
        elif out_path:
            _write(out_path, _summary(V, m, tol, precision, eig, time.perf_counter() - t0, points, checks))
    total = time.perf_counter() - t0
    g.close()
    res = _summary(V, m, tol, precision, eig, total, points, checks)
    if out_path:
        _write(out_path, res)
    return res


def _summary(V, m, tol, precision, eig, total, points, checks) -> dict:
    rows = []
    for p in points:
        d = p.get("derivative") or {"status": None, "iterations": 0, "aligned_steps": 0}
        ok = p["converged"] and d["status"] == 0 and d["iterations"] > 0
        rows.append({"T": p["T"], "K": 1.0 / p["T"], "steps": p["steps"], "converged": p["converged"],
                     "delta": p["delta"], "m_eff": p["m_eff"], "f": p["f"], "E": p["E"], "M": p["M"], "S_E": p["S_E"],
                     "xi_e": p["xi_e"], "derivative": ok, "derivative_status": d["status"],
                     "dF_dK": d["dF_dK"] if ok else None, "d2F_dK2": d["d2F_dK2"] if ok else None,
                     "dM_dK": d["dM_dK"] if ok else None,
                     "specific_heat": -(p["T"] ** -2) * d["d2F_dK2"] if ok else None,
                     "dF_dK_minus_E": d["dF_dK"] - p["E"] if ok else None, "tangent_products": d["iterations"],
                     "aligned_steps": d["aligned_steps"], "seconds": p.get("seconds")})
    diffs = [abs(r["dF_dK_minus_E"]) for r in rows if r["derivative"]]
    return {"m": m, "q": int(np.asarray(V).shape[0]), "tol": tol, "precision": precision, "eigensolver": eig,
            "seconds": total, "points": rows, "central_difference_checks": checks,
            "max_abs_dF_dK_minus_E": max(diffs) if diffs else None}


def run_grid(V, ms, Ts, tol: float, max_steps: int, fd_every: int, dK: float, log=sys.stderr,
             precision: str = "fp64", eig: str = "two_stage", gap_tol=None, out_path=None,
             derivative: bool = True) -> dict:
    """The (T, m) grid: one sweep over Ts per cutoff, the cutoffs in the given order.  With out_path
    the grid so far (finished cutoffs and the current one) is rewritten after every temperature."""
    done = []

    def write(current):
        if out_path:
            _write(out_path, {"grid": done + [current]})

    for m in ms:
        done.append(run(V, int(m), Ts, tol, max_steps, fd_every, dK, log=log, precision=precision, eig=eig,
                        gap_tol=gap_tol, derivative=derivative, on_point=write))
        if out_path:
            _write(out_path, {"grid": done})
    return {"grid": done}


def _write(path: str, res: dict):
    with open(path, "w") as fh:
        fh.write(json.dumps(res) + "\n")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--vertices", default="dodecahedron",
                    choices=["dodecahedron", "icosahedron", "cube", "tetrahedron", "ising"])
    ap.add_argument("--m", default="128", help="cutoff, or a comma-separated list of cutoffs (a (T, m) grid)")
    ap.add_argument("--set", choices=sorted(CUTOFF_SETS), default=None,
                    help="one of the cutoff sets of the paper's scaling analysis (overrides --m)")
    ap.add_argument("--T0", type=float, default=None, help="default 0.40, or 0.35 with --set")
    ap.add_argument("--T1", type=float, default=None, help="default 0.48, or 0.56 with --set")
    ap.add_argument("--n", type=int, default=41)
    ap.add_argument("--tol", type=float, default=1e-12)
    ap.add_argument("--max-steps", type=int, default=3000)
    ap.add_argument("--fd-every", type=int, default=10, help="central-difference check every k-th temperature (0: none)")
    ap.add_argument("--dK", type=float, default=1e-5)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16x3"],
                    help="contractions of the sweep's steps (the derivative runs in FP64)")
    ap.add_argument("--eig", default="two_stage", choices=["two_stage", "warm"])
    ap.add_argument("--gap-tol", type=float, default=None)
    ap.add_argument("--no-derivative", action="store_true", help="observables only (no fixed-point derivative)")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    if args.set:
        ms = list(CUTOFF_SETS[args.set])
        t0, t1 = PAPER_T_RANGE
    else:
        ms = [int(x) for x in str(args.m).split(",") if x.strip()]
        t0, t1 = 0.40, 0.48
    if not ms or any(m < 1 for m in ms):
        ap.error("--m needs positive cutoffs")
    Ts = np.linspace(args.T0 if args.T0 is not None else t0, args.T1 if args.T1 is not None else t1, args.n)
    kw = dict(precision=args.precision, eig=args.eig, gap_tol=args.gap_tol, out_path=args.out,
              derivative=not args.no_derivative)
    V = vertex_set(args.vertices)
    if len(ms) == 1:
        res = run(V, ms[0], Ts, args.tol, args.max_steps, args.fd_every, args.dK, **kw)
    else:
        res = run_grid(V, ms, Ts, args.tol, args.max_steps, args.fd_every, args.dK, **kw)
    res["vertices"] = args.vertices
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
