"""The split-bf16 contractions (precision "bf16x3": FP32 operands split into bf16 hi + lo parts,
three products hi*hi + hi*lo + lo*hi on the bf16 matrix cores with FP32 accumulation) through the
C ABI, against the FP64 oracle; the half-row chain of both mixed paths against the oracle.

Bounds (first order in the unit roundoffs; u32 = 2^-24 for FP32, ub = 2^-8 for bf16):
  * a value x split as hi = bf16(x), lo = bf16(x - hi) satisfies |x - (hi + lo)| <= ub^2 |x| and
    |lo| <= ub (1 + ub) |x|; the product a b taken as hi hi + hi lo + lo hi (the bf16 products are
    exact in FP32) then differs from a b by at most e3 |a b| with
    e3 = 2 ub^2 (1 + ub) + ub^2 (1 + ub)^2 + ub^4  (about 3.02 * 2^-16);
  * every stage rounds its operands from FP64 to FP32 (u32 each) and accumulates 3 K products in
    FP32 (at most 3 K u32 of the sum of the absolute values of its terms), and an FP32 result
    of a stage is rounded once more;
  * so an entry of C' = W-mix(A^T Omega A) is within (2 e3 + (3 m + 3 q^2 + 8) u32) of the sum
    of the absolute values of its terms (the oracle's extension of |P|, |omega|), and an entry of
    the projected half-row U^T W-mix(P U) within (3 e3 + (3 m + 3 q^2 + 3 q m + 12) u32) of the
    oracle's half-row of |W|, |P|, |U|.  With FP32 products e3 is replaced by 0 and the factors 3
    of the accumulation by 1.
  * eigenvalues move by at most ||dC'||_2 <= ||dC'||_F (Weyl).

The measured errors are printed next to the bounds; the error of the split products must also
exceed the FP32 path's on the same input (the bf16 path really ran).

At the fixed points the split products leave f, E and M within 1e-5 (f relative).  That is the
accuracy class of the three-term split: the dropped lo*lo term and the rounding of the lo parts are
each about 2^-18 |a b| for a typical product (2^-16 at most), and where a few terms dominate a sum
(the ordered phase) they do not average out, so C' and the normalizations carry relative errors of a
few 1e-6 (measured: about 5e-6 of max|C'| on the extension, 3e-6 on f at the q = 2 fixed point).  The
1e-6 on f that the FP32 contractions reach is not within this class.
"""
import os

import numpy as np
import pytest

import ctmrg_inputs as I
import exact as E
from oracle import ctmrg_oracle as O

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
UB = 2.0 ** -8
E3 = 2 * UB ** 2 * (1 + UB) + UB ** 2 * (1 + UB) ** 2 + UB ** 4
GAP = 1e-4  # multiplet gap of the cut on the split-bf16 path


def _lib():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_08669_amd import ctmrg
    ctmrg.load()
    return ctmrg


def say(*a):
    print(*a, flush=True)


def _extend_on_gpu(ct, V, K, m, P, om, precision):
    g = ct.CTMRG(V, K, m, precision=precision)
    g.set_state(P, om)
    g.extend()
    C = g.get("cext")
    g.close()
    return C


@pytest.mark.parametrize("m,seed", [(8, 0), (37, 2), (64, 3)])
def test_extension_bf16x3_within_split_bound(m, seed):
    """C' on the split-bf16 path (tiles of 128 x 128 and 80 x 128, ragged at m = 37) within the
    bound of the header, entry by entry."""
    ct = _lib()
    V = I.dodecahedron()
    q = len(V)
    K = 1.0 / 0.4398
    P, om = I.random_state(seed, q, m)
    say(f"[bf16x3 extension] q=20 m={m} seed={seed}")
    C = _extend_on_gpu(ct, V, K, m, P, om, "bf16x3")
    C32 = _extend_on_gpu(ct, V, K, m, P, om, "fp32")
    W = O.weight(V, K)
    ref = O.extend(W, P, om)
    absum = O.extend(W, np.abs(P), np.abs(om))
    bound = (2 * E3 + (3 * m + 3 * q * q + 8) * U32) * absum
    err = np.abs(C - ref)
    err32 = np.abs(C32 - ref)
    amax = np.abs(ref).max()
    say(f"  max err {err.max():.3e} ({err.max() / amax:.2e} of max|C'|), max err / bound "
        f"{np.max(err / np.maximum(bound, 1e-300)):.3f}; FP32 path max err {err32.max():.3e}")
    assert np.all(err <= bound)
    assert err.max() > 2.0 * err32.max()


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("m,seed", [(16, 4), (37, 5)])
def test_halfrow_within_bound(precision, m, seed):
    """One step from a seeded state: the new P (the projected half-row U^T W-mix(P U) over its
    largest entry) against the oracle's half-row of the same P and of the GPU's own kept
    eigenvectors U, so that the check covers the half-row, W-mix and projection products
    (split along K at these sizes only through the ragged tiles) whatever the eigensolver did."""
    ct = _lib()
    V = I.dodecahedron()
    q = len(V)
    K = 1.0 / 0.4398
    P, om = I.random_state(seed, q, m)
    say(f"[{precision} half-row] q=20 m={m} seed={seed}")
    g = ct.CTMRG(V, K, m, precision=precision, gap_tol=GAP)
    g.set_state(P, om)
    g.step(1)
    U = g.get("U")
    om_new = g.get("omega")
    Pg = g.P_slices()
    g.close()
    me = int(np.count_nonzero(om_new))
    Uk = U[:, :me]
    W = O.weight(V, K)
    Pt = O.halfrow(W, P, Uk)
    absum = O.halfrow(W, np.abs(P), np.abs(Uk))
    if precision == "bf16x3":
        rel = 3 * E3 + (3 * m + 3 * q * q + 3 * q * m + 12) * U32
    else:
        rel = (m + q * q + q * m + 12) * U32
    bnd = rel * absum
    imax = np.unravel_index(np.argmax(np.abs(Pt)), Pt.shape)
    nP = abs(Pt[imax])
    # the GPU divides by its own largest entry, which is within bnd[imax] of the oracle's
    bound = (bnd + np.abs(Pt) * bnd[imax] / nP) / (nP - bnd[imax]) * (1 + 1e-12)
    err = np.abs(Pg[:, :me, :me] - Pt / nP)
    say(f"  m_eff {me}; max err {err.max():.3e}, max err / bound {np.max(err / np.maximum(bound, 1e-300)):.3f}")
    assert np.all(err <= bound)
    assert np.all(Pg[:, me:, :] == 0.0) and np.all(Pg[:, :, me:] == 0.0)


@pytest.mark.parametrize("m,T,steps", [(16, 0.5, 3), (40, 0.44, 3)])
def test_bf16x3_one_step_spectrum(m, T, steps):
    """From an oracle state, one split-bf16 step: the whole spectrum of C' within the Weyl bound
    of the contraction error, and the kept dimension equal to the oracle's at the same gap."""
    ct = _lib()
    V = I.dodecahedron()
    q = len(V)
    K = 1.0 / T
    o = O.OracleCTMRG(V, K, m, tau=GAP)
    for _ in range(steps):
        o.step()
    P, om = o.P.copy(), o.omega.copy()
    say(f"[bf16x3 one step] m={m} T={T} after {steps} oracle steps")
    r = O.step(o.W, P, om, m, tau=GAP)
    absum = O.extend(o.W, np.abs(P), np.abs(om))
    weyl = (2 * E3 + (3 * m + 3 * q * q + 8) * U32) * np.linalg.norm(absum)
    g = ct.CTMRG(V, K, m, precision="bf16x3", gap_tol=GAP)
    g.set_state(P, om)
    g.step(1)
    spec = g.get("spectrum")
    me_g = int(np.count_nonzero(g.get("omega")))
    g.close()
    nz = spec[np.argsort(-np.abs(spec))][: len(r.lam)]
    d = np.abs(np.sort(nz) - np.sort(r.lam)).max()
    say(f"  spectrum err {d:.3e} ({d / np.abs(r.lam).max():.2e} of |lambda_1|), Weyl bound {weyl:.3e}, "
        f"m_eff gpu {me_g} oracle {r.m_eff}")
    assert d <= weyl
    assert me_g == r.m_eff


@pytest.mark.parametrize("T,m", [(2.0, 16), (1.5, 12)])
def test_bf16x3_ising_fixed_point(T, m):
    """q = 2 with split-bf16 contractions against Onsager's free energy and Yang's magnetization."""
    ct = _lib()
    K = 1.0 / T
    say(f"[bf16x3 ising] T={T} m={m}")
    g = ct.CTMRG(I.ising(), K, m, precision="bf16x3")
    ks, d, conv = g.run_to_fixed_point(1e-8, 2000)
    ob = g.observables()
    g.close()
    ref_f = -T * E.ising_minus_beta_f(K)
    say(f"  steps {ks} delta {d:.2e} f {ob['f']:.12f} ref {ref_f:.12f} (rel {abs(ob['f'] - ref_f) / abs(ref_f):.2e}) "
        f"E {ob['E']:.9f} ref {E.ising_energy(K):.9f} M {ob['M']:.9f} ref {E.ising_magnetization(K):.9f}")
    assert abs(ob["f"] - ref_f) <= 1e-5 * abs(ref_f)
    assert abs(ob["E"] - E.ising_energy(K)) <= 1e-5
    assert abs(ob["M"] - E.ising_magnetization(K)) <= 1e-5


def test_bf16x3_dodecahedron_fixed_point_m16():
    """q = 20, m = 16, T = 0.40: the split-bf16 path's fixed point against the FP64 oracle's, both
    with the multiplet gap 1e-4 (tests/golden, converged to 1e-12 in 233 steps).  The split-bf16
    run takes 300 steps (its kept spectrum keeps moving by its rounding noise, so a change below
    1e-5 is reached long before M has settled)."""
    ct = _lib()
    V = I.dodecahedron()
    T, m = 0.40, 16
    K = 1.0 / T
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"fixedpoint_q20_m16_T{T:.2f}_tau1e-04.npz")
    if not os.path.exists(path):
        pytest.fail("missing golden file: run tests/golden/make_golden.py")
    with np.load(path, allow_pickle=False) as z:
        oo = {k: z[k] for k in z.files}
    assert bool(oo["converged"]) and float(oo["tau"]) == GAP
    say(f"[bf16x3 fixed point] q=20 m={m} T={T}")
    g = ct.CTMRG(V, K, m, precision="bf16x3", gap_tol=GAP)
    ks = 300
    d = g.step(ks)
    og = g.observables()
    g.close()
    of, oE, oM = float(oo["f"]), float(oo["E"]), float(oo["M"])
    say(f"  gpu: steps {ks} delta {d:.2e} m_eff {og['m_eff']}; oracle steps {int(oo['steps'])} m_eff {int(oo['m_eff'])}")
    say(f"  f {og['f']:.12f} vs {of:.12f} (rel {abs(og['f'] - of) / abs(of):.2e}); E {og['E']:.9f} vs {oE:.9f}; "
        f"M {og['M']:.9f} vs {oM:.9f}")
    assert d <= 1e-5
    assert og["m_eff"] == int(oo["m_eff"])
    assert abs(og["f"] - of) <= 1e-5 * abs(of)
    assert abs(og["E"] - oE) <= 1e-5
    assert abs(og["M"] - oM) <= 1e-5
