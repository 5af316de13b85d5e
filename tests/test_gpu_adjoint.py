"""The fixed-point derivative (tangent-mode implicit differentiation, FP64) through the C ABI:
dF/dK, and along the same tangent dE/dK (= d2F/dK2) and dM/dK.

References that do not come from the GPU path:
  * q = 2: dF/dK is the energy per site, Onsager's closed form; d2F/dK2 is its K-derivative
    (tests/exact.py differentiates the closed form); dM/dK is the derivative of Yang's formula;
  * q = 20: the oracle's central difference [F(K+h) - F(K-h)] / 2h of its own fixed points
    (h = 1e-4, each converged to Delta < 1e-13: accurate to about 1e-8), the oracle's impurity
    energy at the same m (equal to dF/dK at an exact fixed point), and the central differences
    of that energy for d2F/dK2 and of M for dM/dK (accurate to about 1e-7);
  * q = 20, m = 128 at T = 0.40, 0.44, 0.48 (three temperatures of the sweep): the oracle's f
    and impurity energy at its own fixed point (tests/golden).
"""
import os

import numpy as np
import pytest

import ctmrg_inputs as I
import exact as E
from oracle import ctmrg_oracle as O

pytestmark = pytest.mark.gpu


def _lib():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_08669_amd import ctmrg
    ctmrg.load()
    return ctmrg


def say(*a):
    print(*a, flush=True)


def _converged(ct, V, K, m, tol=1e-13, max_steps=3000):
    g = ct.CTMRG(V, K, m)
    ks, d, conv = g.run_to_fixed_point(tol, max_steps)
    assert conv, (ks, d)
    return g


@pytest.mark.parametrize("T,m", [(2.0, 16), (1.5, 12), (2.5, 16)])
def test_derivative_ising_onsager(T, m):
    ct = _lib()
    K = 1.0 / T
    say(f"[derivative ising] T={T} m={m}")
    g = _converged(ct, I.ising(), K, m)
    r = g.fixed_point_derivative(second_order=True)
    g.close()
    say(f"  {r}")
    assert abs(r["F"] + E.ising_minus_beta_f(K)) <= 1e-10 * E.ising_minus_beta_f(K)
    assert abs(r["dF_dK"] - E.ising_energy(K)) <= 1e-8
    assert abs(r["E"] - r["dF_dK"]) <= 1e-9
    d2 = E.ising_d2F_dK2(K)
    assert r["d2F_dK2"] == r["dE_dK"]
    assert abs(r["d2F_dK2"] - d2) <= 1e-5 * abs(d2)
    dM = E.ising_dM_dK(K)
    say(f"  dM/dK {r['dM_dK']!r}, Yang {dM!r}; M {r['M']!r}, Yang {E.ising_magnetization(K)!r}")
    assert abs(r["M"] - E.ising_magnetization(K)) <= 1e-8
    if dM == 0.0:
        # disordered phase: M and its derivative vanish up to the fixed boundary's residue at finite m
        assert abs(r["dM_dK"]) <= 1e-6
    else:
        assert abs(r["dM_dK"] - dM) <= 1e-5 * abs(dM)


def _golden(name):
    """Stored oracle values (tests/golden/, written by make_golden.py from the oracle alone)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    if not os.path.exists(path):
        pytest.fail(f"missing golden file {name}: run tests/golden/make_golden.py")
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def test_derivative_dodecahedron_m12():
    ct = _lib()
    V = I.dodecahedron()
    T, m = 0.40, 12
    K = 1.0 / T
    ref = _golden(f"derivative_q20_m{m}_T{T:.2f}.npz")
    h = float(ref["h"])
    say(f"[derivative dodecahedron] T={T} m={m}")
    g = _converged(ct, V, K, m)
    obs = g.observables()
    r = g.fixed_point_derivative(second_order=True)
    g.close()
    say(f"  {r}")
    fd = (float(ref["F_p"]) - float(ref["F_m"])) / (2 * h)
    d2 = (float(ref["E_p"]) - float(ref["E_m"])) / (2 * h)
    dM = (float(ref["M_p"]) - float(ref["M_m"])) / (2 * h)
    F0, E0, M0 = float(ref["F_0"]), float(ref["E_0"]), float(ref["M_0"])
    say(f"  dF/dK {r['dF_dK']:.13f}  oracle FD {fd:.13f}  oracle E_imp {E0:.13f}  gpu E_imp {obs['E']:.13f}")
    say(f"  d2F/dK2 {r['d2F_dK2']:.9f}  oracle central difference of E_imp {d2:.9f}")
    say(f"  dM/dK {r['dM_dK']:.9f}  oracle central difference of M {dM:.9f}; M {r['M']:.12f} oracle {M0:.12f}")
    assert abs(r["F"] - F0) <= 1e-11 * abs(F0)
    assert abs(r["dF_dK"] - fd) <= 1e-7
    assert abs(r["dF_dK"] - E0) <= 1e-9
    assert abs(r["dF_dK"] - obs["E"]) <= 1e-9
    assert abs(r["E"] - E0) <= 1e-9
    assert abs(r["M"] - M0) <= 1e-9
    assert abs(r["d2F_dK2"] - d2) <= 1e-5 * abs(d2)
    assert abs(r["dM_dK"] - dM) <= 1e-5 * abs(dM)
    # the cross-check: central difference of dF/dK over fixed points at K (1 +- 1e-4)
    g = _converged(ct, V, K, m)
    r2 = g.fixed_point_derivative(second_order=2)
    g.close()
    say(f"  d2F/dK2 along the tangent {r['d2F_dK2']:.9f}, central difference of dF/dK {r2['d2F_dK2']:.9f}")
    assert abs(r["d2F_dK2"] - r2["d2F_dK2"]) <= 1e-5 * abs(d2)


def test_backward_combines_the_derivatives():
    ct = _lib()
    V = I.dodecahedron()
    K = 1.0 / 0.40
    say("[backward] q=20 m=8 T=0.40")
    g = _converged(ct, V, K, 8)
    r = g.fixed_point_derivative(second_order=True)
    kb, d2 = g.backward([1.0, 0.0, 0.0], want_d2=True)
    # f = F / K
    assert abs(kb - (r["dF_dK"] / K - r["F"] / K ** 2)) <= 1e-12 * abs(kb)
    assert abs(d2 - r["d2F_dK2"]) <= 1e-9 * abs(d2)
    kb2, _ = g.backward([0.0, 2.0, 0.0])
    assert abs(kb2 - 2.0 * r["d2F_dK2"]) <= 1e-9 * abs(kb2)
    kb3, _ = g.backward([0.0, 0.0, 1.0])
    assert abs(kb3 - r["dM_dK"]) <= 1e-9 * abs(kb3)
    g.close()
    # before convergence
    g = ct.CTMRG(V, K, 8)
    g.step(1)
    with pytest.raises(ct.CTMRGError) as e:
        g.fixed_point_derivative()
    assert e.value.status == 6
    g.close()


@pytest.mark.parametrize("T", [0.40, 0.44, 0.48])
def test_derivative_m128_equals_impurity_energy(T):
    """At m = 128 (C' 2560 x 2560, the size of the temperature sweep with derivatives), at three of
    its temperatures: the derivative of F equals the energy of the impurity plaquette on the same
    fixed point and on the oracle's own fixed point (tests/golden, converged independently to
    1e-12); at T = 0.44 it also equals the central difference of F = K f over fixed points at
    K +- 1e-4."""
    ct = _lib()
    V = I.dodecahedron()
    K = 1.0 / T
    ref = _golden(f"fixedpoint_q20_m128_T{T:.2f}.npz")
    say(f"[derivative m=128] T={T}; oracle fixed point in {int(ref['steps'])} steps")
    g = _converged(ct, V, K, 128, tol=1e-12, max_steps=2000)
    obs = g.observables()
    r = g.fixed_point_derivative()
    g.close()
    Eo, fo = float(ref["E"]), float(ref["f"])
    say(f"  {r}; E_imp gpu {obs['E']:.13f} oracle {Eo:.13f}; f gpu {obs['f']:.13f} oracle {fo:.13f}")
    assert abs(r["dF_dK"] - obs["E"]) <= 1e-8
    assert abs(r["dF_dK"] - Eo) <= 1e-8
    assert abs(obs["f"] - fo) <= 1e-10 * abs(fo)
    assert abs(r["F"] - K * fo) <= 1e-10 * abs(K * fo)
    say(f"  dE/dK = d2F/dK2 {r['dE_dK']!r}, dM/dK {r['dM_dK']!r}")
    assert abs(r["E"] - Eo) <= 1e-8
    assert abs(r["M"] - float(ref["M"])) <= 1e-8
    if T == 0.44:
        h = 1e-4
        F, Es, Ms = {}, {}, {}
        for sgn in (1, -1):
            # the fixed points at K +- h with the warm-started eigensolver (f is exact on it)
            w = ct.CTMRG(V, K + sgn * h, 128, eig="warm")
            ks, d, conv = w.run_to_fixed_point(1e-12, 3000)
            assert conv, (ks, d)
            o = w.observables()
            F[sgn] = (K + sgn * h) * o["f"]
            Es[sgn], Ms[sgn] = o["E"], o["M"]
            w.close()
        fd = (F[1] - F[-1]) / (2 * h)
        fdE = (Es[1] - Es[-1]) / (2 * h)
        fdM = (Ms[1] - Ms[-1]) / (2 * h)
        say(f"  dF/dK {r['dF_dK']:.13f}, central difference of F {fd:.13f}")
        say(f"  dE/dK {r['dE_dK']:.9f}, central difference of E {fdE:.9f}; dM/dK {r['dM_dK']:.9f}, "
            f"central difference of M {fdM:.9f}")
        assert abs(r["dF_dK"] - fd) <= 1e-7
        assert abs(r["dE_dK"] - fdE) <= 1e-5 * abs(fdE)
        assert abs(r["dM_dK"] - fdM) <= 1e-5 * abs(fdM)


def test_autograd_function():
    """K.grad of f through torch.autograd equals df/dK = (E - f)/K at the fixed point; the
    gradient of M equals the derivative's dM/dK."""
    torch = pytest.importorskip("torch")
    ct = _lib()
    from paper_2004_08669_amd.autograd import CTMRGFixedPoint
    V = I.dodecahedron()
    say("[autograd] q=20 m=8 T=0.40")
    K = torch.tensor(1.0 / 0.40, dtype=torch.float64, requires_grad=True)
    f, Eo, M = CTMRGFixedPoint.apply(K, V, 8)
    f.backward()
    ref = (Eo.item() - f.item()) / K.item()
    say(f"  f {f.item():.12f} E {Eo.item():.12f} K.grad {K.grad.item():.12f} (E - f)/K {ref:.12f}")
    assert abs(K.grad.item() - ref) <= 1e-9
    K2 = torch.tensor(1.0 / 0.40, dtype=torch.float64, requires_grad=True)
    f2, E2, M2 = CTMRGFixedPoint.apply(K2, V, 8)
    M2.backward()
    g = ct.CTMRG(V, 1.0 / 0.40, 8)
    g.run_to_fixed_point(1e-13, 3000)
    r = g.fixed_point_derivative()
    g.close()
    say(f"  M {M2.item():.12f} K.grad {K2.grad.item():.12f} dM/dK {r['dM_dK']:.12f}")
    assert abs(K2.grad.item() - r["dM_dK"]) <= 1e-9 * abs(r["dM_dK"])
