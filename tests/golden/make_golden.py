#!/usr/bin/env python3
"""Writes the stored expected values under tests/golden/ by calling the CPU oracle only.

Nothing here runs the GPU library: every number comes from oracle/ctmrg_oracle.py on the
seeded inputs of ctmrg_inputs.py.  Usage (from the repository root):

  python tests/golden/make_golden.py onestep --m 128 --seed 0 --steps 2
      Jacobi-oracle steps of the q = 20 dodecahedron model at T = 0.4398 from the seeded
      random state random_state(seed, 20, m) (Sec. III, Algorithm 3).  Stores, after every
      step, the full spectrum of C', m_eff, n_C, S_E (Eq. 6), the kept omega, n_P, and
      gauge-invariant functions of the new state: the q x q matrix Tr(P_s Om P_sg Om), the
      environment sums of the observables and M (Eq. 5).  --eig lapack takes numpy's LAPACK driver as the
      diagonalization step (the two-step m = 256 file, seed 2).

  python tests/golden/make_golden.py fixedpoint --m 64 --T 0.40
      The fixed-boundary run from the initial state of Algorithm 3 until the kept spectrum
      changes by less than 1e-12 (or 3000 steps), with numpy's LAPACK eigensolver as the
      diagonalization step.  Stores f, E, M, S_E, m_eff, the kept spectrum, the number of
      steps, and the effective correlation length xi_e with |lambda_2 / lambda_1| of the
      row-to-row transfer matrix (Sec. II).  --eig jacobi uses the oracle's own solver (small m).

  python tests/golden/make_golden.py derivative --m 12 --T 0.40
      References of the fixed-point derivative: F = beta f, the impurity energy E and the
      observables at K = 1/T and at K +- 1e-4 (each fixed point converged to 1e-13, the
      shifted ones started from the converged state at K), Jacobi oracle.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import ctmrg_inputs as I  # noqa: E402
from oracle import ctmrg_oracle as O  # noqa: E402


def invariants(o: O.OracleCTMRG) -> dict:
    """Gauge-invariant functions of the current state (P, omega) and the last step."""
    P, om = o.P, o.omega
    POm = P * om[None, None, :]
    # G[s, sg] = Tr(P_s Om P_sg Om) = sum_ab (P_s Om)[a,b] (P_sg Om)[b,a]
    G = np.einsum("sab,tba->st", POm, POm)
    Zb, Zh, Zd, Zd_h = o.environment_sums()
    return {"G": G, "Zb": Zb, "Zh": Zh, "Zd": Zd, "Zd_h": Zd_h, "E": 0.5 * Zd_h / Zd,
            "M": o.magnetization()}


def onestep(args):
    V = I.dodecahedron()
    K = 1.0 / args.T
    P, om = I.random_state(args.seed, 20, args.m)
    o = O.OracleCTMRG(V, K, args.m, eig=args.eig)
    o.import_state(P, om, k=0)
    out = {"q": 20, "m": args.m, "T": args.T, "seed": args.seed, "steps": args.steps, "eig": args.eig}
    for k in range(1, args.steps + 1):
        t0 = time.perf_counter()
        r = o.step()
        print(f"step {k}: {time.perf_counter() - t0:.1f} s, m_eff {r.m_eff}", flush=True)
        inv = invariants(o)
        pre = f"s{k}_"
        out[pre + "lam"] = r.lam
        out[pre + "m_eff"] = r.m_eff
        out[pre + "n_C"] = r.n_C
        out[pre + "S_E"] = r.S_E
        out[pre + "omega"] = r.omega
        out[pre + "n_P"] = r.n_P
        for key, val in inv.items():
            out[pre + key] = val
    if args.steps >= 2:
        out["ln_kappa_W"] = o.ln_kappa_W()
        out["f"] = -0.5 * args.T * out["ln_kappa_W"]
    name = f"onestep_q20_m{args.m}_T{args.T}_seed{args.seed}.npz"
    np.savez(os.path.join(HERE, name), **{k: np.asarray(v) for k, v in out.items()})
    print("wrote", name)


def fixedpoint(args):
    V = I.dodecahedron()
    K = 1.0 / args.T
    o = O.OracleCTMRG(V, K, args.m, eig=args.eig, tau=args.tau)
    t0 = time.perf_counter()
    converged = False
    while o.k < args.max_steps:
        o.step()
        if o.k % 100 == 0:
            print(f"T={args.T} step {o.k} delta {o.delta:.3e} {time.perf_counter() - t0:.0f} s", flush=True)
        if o.k >= 2 and o.delta < args.tol:
            converged = True
            break
    obs = o.observables()
    # effective correlation length of the fixed point (gauge invariant: the spectrum of T)
    lam_t, xi = O.correlation_length(o.P, "dense" if o.P.shape[1] <= 40 else "arpack")
    out = {"q": 20, "m": args.m, "T": args.T, "tol": args.tol, "tau": args.tau, "converged": converged, "steps": o.k,
           "delta": o.delta, "f": obs["f"], "E": obs["E"], "M": obs["M"], "S_E": obs["S_E"],
           "m_eff": obs["m_eff"], "ln_kappa_ratio": obs["ln_kappa_ratio"], "omega": o.omega,
           "lam": o.last.lam, "xi_e": xi, "tm_ratio": abs(lam_t[1] / lam_t[0])}
    tag = "" if args.tau == 1e-10 else f"_tau{args.tau:.0e}"
    name = f"fixedpoint_q20_m{args.m}_T{args.T:.2f}{tag}.npz"
    np.savez(os.path.join(HERE, name), **{k: np.asarray(v) for k, v in out.items()})
    print("wrote", name, "converged", converged, "steps", o.k, flush=True)


def derivative(args):
    V = I.dodecahedron()
    K = 1.0 / args.T
    h = args.h

    def converge(Kx, start=None):
        o = O.OracleCTMRG(V, Kx, args.m, eig=args.eig)
        if start is not None:
            o.import_state(start.P, start.omega, k=1)
        while o.k < 5000:
            o.step()
            if o.k >= 3 and o.delta < 1e-13:
                return o
        raise RuntimeError("no convergence")

    o0 = converge(K)
    op = converge(K + h, o0)
    om = converge(K - h, o0)
    out = {"q": 20, "m": args.m, "T": args.T, "K": K, "h": h}
    for tag, o in (("0", o0), ("p", op), ("m", om)):
        obs = o.observables()
        out["F_" + tag] = -obs["minus_beta_f"]
        out["E_" + tag] = obs["E"]
        out["M_" + tag] = obs["M"]
        out["m_eff_" + tag] = obs["m_eff"]
    name = f"derivative_q20_m{args.m}_T{args.T:.2f}.npz"
    np.savez(os.path.join(HERE, name), **{k: np.asarray(v) for k, v in out.items()})
    print("wrote", name, flush=True)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("onestep")
    a.add_argument("--m", type=int, required=True)
    a.add_argument("--seed", type=int, default=0)
    a.add_argument("--T", type=float, default=0.4398)
    a.add_argument("--steps", type=int, default=1)
    a.add_argument("--eig", default="jacobi")
    b = sub.add_parser("fixedpoint")
    b.add_argument("--m", type=int, default=64)
    b.add_argument("--T", type=float, required=True)
    b.add_argument("--tol", type=float, default=1e-12)
    b.add_argument("--max-steps", type=int, default=3000)
    b.add_argument("--eig", default="lapack")
    b.add_argument("--tau", type=float, default=1e-10, help="multiplet gap of the cut, relative to |lambda_1|")
    c = sub.add_parser("derivative")
    c.add_argument("--m", type=int, default=12)
    c.add_argument("--T", type=float, default=0.40)
    c.add_argument("--h", type=float, default=1e-4)
    c.add_argument("--eig", default="jacobi")
    args = ap.parse_args()
    {"onestep": onestep, "fixedpoint": fixedpoint, "derivative": derivative}[args.cmd](args)


if __name__ == "__main__":
    main()
