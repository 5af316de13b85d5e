"""The warm-started eigensolver (CTMRG_EIG_WARM) through the C ABI.

* q = 20, m = 64, T = 0.40: the fixed point reached with the warm solver against the oracle's
  (tests/golden/, written by make_golden.py from the oracle alone): f to 1e-10 relative, E and M
  to 1e-8, the same m_eff.  S_E (Eq. 6) is checked within the bound the solver reports for the
  part of the spectrum beyond its Ritz block.
* q = 20, m = 512 (the bench's size): from one state, the same steps with the warm solver and
  with the two-stage solver give the same kept spectrum, normalization, observables and the
  same gauge-invariant matrix Tr(P_s Om P_sg Om) of the new state.
* the mixed path with the warm solver at its m = 16 fixed point against the FP64 oracle.
"""
import math
import os

import numpy as np
import pytest

import ctmrg_inputs as I

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _lib():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_08669_amd import ctmrg
    ctmrg.load()
    return ctmrg


def say(*a):
    print(*a, flush=True)


def _golden(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.fail(f"missing golden file {name}: run tests/golden/make_golden.py")
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def _entropy_bound(tail, n):
    """Largest change of -sum w^4 ln w^4 from a share `tail` of sum w^4 spread over n states."""
    if tail <= 0.0:
        return 1e-12
    return 2.0 * tail * (math.log(n / tail) + 1.0) + 1e-12


def test_warm_fixed_point_m64_matches_oracle():
    ct = _lib()
    ref = _golden("fixedpoint_q20_m64_T0.40.npz")
    T, m = float(ref["T"]), int(ref["m"])
    say(f"[warm fixed point] q=20 m={m} T={T}")
    g = ct.CTMRG(I.dodecahedron(), 1.0 / T, m, eig="warm")
    ks, delta, conv = g.run_to_fixed_point(float(ref["tol"]), 3000)
    obs = g.observables()
    st = g.eig_stats()
    g.close()
    say(f"  {ks} steps, delta {delta:.2e}; stats {st}")
    say(f"  f {obs['f']!r} ({float(ref['f'])!r}) E {obs['E']!r} ({float(ref['E'])!r}) M {obs['M']!r} ({float(ref['M'])!r}) "
        f"S_E {obs['S_E']!r} ({float(ref['S_E'])!r})")
    assert conv
    assert st["warm_steps"] > ks // 2
    assert obs["m_eff"] == int(ref["m_eff"])
    assert abs(obs["f"] - float(ref["f"])) <= 1e-10 * abs(float(ref["f"]))
    assert abs(obs["E"] - float(ref["E"])) <= 1e-8
    assert abs(obs["M"] - float(ref["M"])) <= 1e-8
    # S_E of the observables runs over all eigenvalues of the last C'
    assert abs(obs["S_E"] - float(ref["S_E"])) <= 1e-10


def test_warm_matches_two_stage_m512():
    ct = _lib()
    V, K, m = I.dodecahedron(), 1.0 / 0.4398, 512
    say("[warm vs two-stage] q=20 m=512: 8 two-stage steps, then the same 4 steps on both solvers")
    a = ct.CTMRG(V, K, m)
    a.step(8)
    st = a.export_state()
    b = ct.CTMRG(V, K, m, eig="warm")
    b.import_state(st)
    for k in range(4):
        a.step(1)
        b.step(1)
        oa, ob = a.get("omega"), b.get("omega")
        me = int(np.count_nonzero(oa))
        dw = float(np.abs(oa[:me] ** 4 - ob[:me] ** 4).max())
        say(f"  step {k + 1}: m_eff {me}/{int(np.count_nonzero(ob))} max|d w^4| {dw:.2e} stats {b.eig_stats()}")
        assert int(np.count_nonzero(ob)) == me
    s = b.eig_stats()
    assert s["warm_steps"] >= 1, s
    oa, ob = a.observables(), b.observables()
    tail = s["tail_bound_max"]
    me = oa["m_eff"]
    wa, wb = oa["kept_spectrum"][:me], ob["kept_spectrum"][:me]
    say(f"  f {oa['f']!r}/{ob['f']!r} E {oa['E']!r}/{ob['E']!r} M {oa['M']!r}/{ob['M']!r} S_E {oa['S_E']!r}/{ob['S_E']!r} "
        f"tail bound {tail:.2e}")
    # omega is normalized by n_C, whose part beyond the Ritz block is known within the bound
    assert np.abs(wa - wb).max() <= 1e-11 + tail
    assert abs(oa["f"] - ob["f"]) <= 1e-12 * abs(oa["f"])
    assert abs(oa["E"] - ob["E"]) <= 1e-12
    assert abs(oa["M"] - ob["M"]) <= 1e-12
    assert abs(oa["S_E"] - ob["S_E"]) <= 1e-11
    # the S_E the warm step itself gave (the tail beyond its block bounded) is within its bound
    assert abs(s["last_step_S_E"] - oa["S_E"]) <= _entropy_bound(s["tail_bound_last"], 20 * m)
    Pa, Pb = a.P_slices(), b.P_slices()
    Ga = np.einsum("sab,tba->st", Pa * a.get("omega")[None, None, :], Pa * a.get("omega")[None, None, :])
    Gb = np.einsum("sab,tba->st", Pb * b.get("omega")[None, None, :], Pb * b.get("omega")[None, None, :])
    say(f"  max |G_a - G_b| / max |G_a| = {np.abs(Ga - Gb).max() / np.abs(Ga).max():.2e}")
    assert np.abs(Ga - Gb).max() <= 1e-10 * np.abs(Ga).max()
    a.close()
    b.close()


def test_warm_mixed_fixed_point_m16():
    ct = _lib()
    ref = _golden("fixedpoint_q20_m16_T0.40_tau1e-06.npz")
    T, m = float(ref["T"]), int(ref["m"])
    say(f"[warm mixed fixed point] q=20 m={m} T={T}")
    g = ct.CTMRG(I.dodecahedron(), 1.0 / T, m, precision="fp32", gap_tol=1e-6, eig="warm")
    ks, delta, conv = g.run_to_fixed_point(1e-6, 1500)
    obs = g.observables()
    st = g.eig_stats()
    g.close()
    say(f"  {ks} steps; stats {st}; f {obs['f']!r} ({float(ref['f'])!r}) M {obs['M']!r} ({float(ref['M'])!r})")
    assert conv
    assert st["warm_steps"] > 0
    assert obs["m_eff"] == int(ref["m_eff"])
    assert abs(obs["f"] - float(ref["f"])) <= 1e-6 * abs(float(ref["f"]))
    assert abs(obs["E"] - float(ref["E"])) <= 1e-5
    assert abs(obs["M"] - float(ref["M"])) <= 1e-5
