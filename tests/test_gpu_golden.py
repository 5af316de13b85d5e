"""The HIP path against stored oracle values (tests/golden/, written by make_golden.py, which
calls only the CPU oracle) at sizes where the oracle takes minutes per step.

* Two steps at q = 20, m = 128 (C' 2560 x 2560), one step (seed 1) and two steps (seed 2, the
  oracle's LAPACK diagonalization step) at m = 256 (5120 x 5120)
  from the seeded random states of ctmrg_inputs.random_state, T = 0.4398 (Sec. III,
  Algorithm 3): the full spectrum of C', the cut, the normalized kept spectrum, S_E (Eq. 6),
  and gauge-invariant functions of the new state -- the q x q matrix Tr(P_s Om P_sg Om) (it
  ties the slices together, so slices rotated by different orthogonal matrices fail it), the
  environment sums of the energy, and M (Eq. 5); f after two steps.  FP64, and the mixed paths
  (FP32 and split-bf16 contractions) to their own tolerances.
* Fixed points of the fixed-boundary run at m = 64, T in {0.40, 0.42, 0.44, 0.46, 0.48},
  each side converged on its own (kept spectrum changing by < 1e-12): f, E, M, S_E and m_eff.
"""
import glob
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


def _load(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.fail(f"missing golden file {name}: run tests/golden/make_golden.py")
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def _invariants(g, q, m):
    """Tr(P_s Om P_sg Om) on the GPU state (host arithmetic on exported buffers)."""
    P = g.P_slices()
    om = g.get("omega")
    POm = P * om[None, None, :]
    return np.einsum("sab,tba->st", POm, POm)


def _check_step(g, ref, pre, m, tol):
    q = 20
    N = q * m
    lam = np.sort(g.get("spectrum"))
    lam_o = np.sort(ref[pre + "lam"])
    l1 = np.abs(lam_o).max()
    om = g.get("omega")
    me = int(ref[pre + "m_eff"])
    obs = g.observables()
    # with a wider multiplet gap (the mixed paths) the cut may sit one multiplet lower: the kept
    # spectra are compared over the states both kept
    mc = me if tol["m_eff"] else min(me, int(obs["m_eff"]))
    G = _invariants(g, q, m)
    Go = ref[pre + "G"]
    d = {
        "spectrum": float(np.abs(lam - lam_o).max() / l1),
        "omega": float(np.abs(om[:mc] - ref[pre + "omega"][:mc]).max()),
        "S_E": abs(obs["S_E"] - float(ref[pre + "S_E"])),
        "G": float(np.abs(G - Go).max() / np.abs(Go).max()),
        "E": abs(obs["E"] - float(ref[pre + "E"])),
        "M": abs(obs["M"] - float(ref[pre + "M"])),
    }
    say(f"  {pre} m_eff gpu {obs['m_eff']} oracle {me}; differences {d}")
    if tol["m_eff"]:
        assert obs["m_eff"] == me
    for key, val in d.items():
        assert val <= tol[key], (key, val, tol[key])
    return obs


TOL64 = {"m_eff": True, "spectrum": 1e-13, "omega": 1e-12, "S_E": 1e-11, "G": 1e-10, "E": 1e-10, "M": 1e-10}


@pytest.mark.parametrize("name", sorted(os.path.basename(p) for p in glob.glob(os.path.join(GOLDEN, "onestep_*.npz"))))
def test_golden_steps_fp64(name):
    ct = _lib()
    ref = _load(name)
    m, seed, steps, T = int(ref["m"]), int(ref["seed"]), int(ref["steps"]), float(ref["T"])
    say(f"[golden fp64] {name}: q=20 m={m} seed={seed} steps={steps}")
    P, om = I.random_state(seed, 20, m)
    g = ct.CTMRG(I.dodecahedron(), 1.0 / T, m)
    g.set_state(P, om)
    for k in range(1, steps + 1):
        g.step(1)
        obs = _check_step(g, ref, f"s{k}_", m, TOL64)
    if steps >= 2:
        say(f"  f gpu {obs['f']!r} oracle {float(ref['f'])!r}")
        assert abs(obs["f"] - float(ref["f"])) <= 1e-10 * abs(float(ref["f"]))
    g.close()


# Differences from the FP64 oracle allowed to the mixed paths after one step: the FP32 contractions
# are accurate to about 1e-7 of max|C'|, the split-bf16 ones to about 1e-6 (tests/test_gpu_bf16x3.py
# bounds them entry by entry); the spectrum and the observables move by that much, and the cut may
# move by a multiplet.
TOL_MIXED = {
    "fp32": {"m_eff": False, "spectrum": 2e-6, "omega": 1e-5, "S_E": 1e-5, "G": 1e-4, "E": 1e-5, "M": 1e-5},
    "bf16x3": {"m_eff": False, "spectrum": 2e-5, "omega": 1e-4, "S_E": 1e-4, "G": 1e-3, "E": 1e-4, "M": 1e-4},
}


TOL_F_MIXED = {"fp32": 1e-6, "bf16x3": 1e-5}


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("name", sorted(os.path.basename(p) for p in glob.glob(os.path.join(GOLDEN, "onestep_*.npz"))))
def test_golden_steps_mixed(name, precision):
    """The mixed paths (FP32 contractions, or split-bf16 products with FP32 accumulation) against
    the FP64 oracle, every stored step (m = 256 is the precision configuration: T = 0.4398, C'
    5120 x 5120; the two-step file also gives f)."""
    ct = _lib()
    ref = _load(name)
    m, seed, T = int(ref["m"]), int(ref["seed"]), float(ref["T"])
    say(f"[golden {precision}] {name}: q=20 m={m} seed={seed}")
    P, om = I.random_state(seed, 20, m)
    g = ct.CTMRG(I.dodecahedron(), 1.0 / T, m, precision=precision)
    g.set_state(P, om)
    steps = int(ref["steps"])
    for k in range(1, steps + 1):
        g.step(1)
        tol = dict(TOL_MIXED[precision])
        if k >= 2:
            # the second step's C' is built from the first step's P~, whose error is the contraction
            # error carried through the kept eigenvectors (divided by the eigen-gaps at the cut): the
            # spectrum error grows by about 60 (FP32) and 30 (split-bf16) from the first step to the second
            # at m = 128; a factor of 100 is allowed
            tol["spectrum"] *= 100.0
        obs = _check_step(g, ref, f"s{k}_", m, tol)
    if steps >= 2:
        # f from the normalizations of the two steps (R-f), to the accuracy class of the path
        fo = float(ref["f"])
        say(f"  f gpu {obs['f']!r} oracle {fo!r} (relative {abs(obs['f'] - fo) / abs(fo):.2e})")
        assert abs(obs["f"] - fo) <= TOL_F_MIXED[precision] * abs(fo)
    g.close()


FIXED = sorted(os.path.basename(p) for p in glob.glob(os.path.join(GOLDEN, "fixedpoint_q20_m64_*.npz")))


@pytest.mark.parametrize("name", FIXED)
def test_golden_fixed_point_m64(name):
    """The run of each temperature stops when the kept spectrum changes by less than 1e-12 or
    after 3000 steps; where the oracle stopped at the step limit, the GPU takes exactly as many
    steps and the two states after them are compared."""
    ct = _lib()
    ref = _load(name)
    T, m = float(ref["T"]), int(ref["m"])
    converged = bool(ref["converged"])
    say(f"[golden fixed point] q=20 m={m} T={T}: oracle {'converged in' if converged else 'stopped after'} "
        f"{int(ref['steps'])} steps")
    g = ct.CTMRG(I.dodecahedron(), 1.0 / T, m)
    if converged:
        ks, delta, conv = g.run_to_fixed_point(float(ref["tol"]), 3000)
    else:
        ks = int(ref["steps"])
        delta = g.step(ks)
        conv = True
    obs = g.observables()
    g.close()
    say(f"  gpu: {ks} steps, delta {delta:.2e}; f {obs['f']!r} (oracle {float(ref['f'])!r}) "
        f"E {obs['E']!r} ({float(ref['E'])!r}) M {obs['M']!r} ({float(ref['M'])!r}) m_eff {obs['m_eff']} ({int(ref['m_eff'])})")
    assert conv
    assert obs["m_eff"] == int(ref["m_eff"])
    assert abs(obs["f"] - float(ref["f"])) <= 1e-10 * abs(float(ref["f"]))
    assert abs(obs["E"] - float(ref["E"])) <= 1e-8
    assert abs(obs["M"] - float(ref["M"])) <= 1e-8
    assert abs(obs["S_E"] - float(ref["S_E"])) <= 1e-8
    me = obs["m_eff"]
    assert np.abs(obs["kept_spectrum"][:me] - ref["omega"][:me]).max() <= 1e-9
    if "xi_e" in ref:
        # xi_e (Sec. II): the spectrum of the row-to-row transfer matrix does not depend on the gauge
        r = abs(obs["tm_lambda2"] / obs["tm_lambda1"])
        say(f"  xi_e {obs['xi_e']!r} (oracle {float(ref['xi_e'])!r}), |l2/l1| {r!r} ({float(ref['tm_ratio'])!r})")
        assert obs["tm_converged"] == 1
        assert abs(r - float(ref["tm_ratio"])) <= 1e-9
        assert abs(obs["xi_e"] - float(ref["xi_e"])) <= 1e-8 * float(ref["xi_e"])
