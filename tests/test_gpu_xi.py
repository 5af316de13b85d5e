"""The effective correlation length xi_e (Sec. II, last paragraph) through the C ABI.

ctmrg_observables takes the two eigenvalues of largest modulus of the row-to-row transfer
matrix T = sum_s P_s (x) P_s by Lanczos on the GPU.  Checked against the oracle on the
same P (the GPU's state, read back):
  * m <= 40: all eigenvalues of T by LAPACK (oracle.correlation_length, "dense"):
    lambda_1 and lambda_2 to 1e-12 relative, xi_e to 1e-10 relative;
  * m = 128: ARPACK on the operator X -> sum_s P_s X P_s (oracle, "arpack");
  * q = 2 (Ising): xi_e on the GPU's fixed point equals the oracle's on the same P, and
    lies just below the infinite-lattice value 1 / ln(1 / sinh^2 2K) (above T_c).

The fixed points of tests/golden (oracle-only) carry xi_e too: test_gpu_golden.py and
test_gpu_parity.py compare it with the GPU's own fixed point (the spectrum of T does not depend
on the gauge of P).
"""
import math

import numpy as np
import pytest

import ctmrg_inputs as I
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


@pytest.mark.parametrize("m,T,steps", [(1, 0.44, 1), (3, 0.44, 4), (8, 0.40, 20), (24, 0.48, 30), (40, 0.44, 25)])
def test_xi_matches_oracle_dense(m, T, steps):
    ct = _lib()
    say(f"[xi dense] q=20 m={m} T={T} steps={steps}")
    g = ct.CTMRG(I.dodecahedron(), 1.0 / T, m)
    g.step(steps)
    ob = g.observables()
    P = g.P_slices()
    g.close()
    lam, xi = O.correlation_length(P, "dense")
    say(f"  gpu l1 {ob['tm_lambda1']!r} l2 {ob['tm_lambda2']!r} xi {ob['xi_e']!r} res {ob['tm_residual']:.2e} "
        f"it {ob['tm_iterations']}; oracle {lam[0]!r} {lam[1]!r} xi {xi!r}")
    assert ob["tm_converged"] == 1
    assert ob["tm_residual"] <= 1e-10
    assert abs(ob["tm_lambda1"] - lam[0]) <= 1e-12 * abs(lam[0])
    assert abs(ob["tm_lambda2"] - lam[1]) <= 1e-12 * abs(lam[0])
    if m == 1:
        assert ob["xi_e"] == 0.0 and ob["tm_lambda2"] == 0.0
    else:
        assert abs(ob["xi_e"] - xi) <= 1e-10 * xi


def test_xi_matches_arpack_m128():
    ct = _lib()
    say("[xi arpack] q=20 m=128 T=0.4398, 12 steps")
    g = ct.CTMRG(I.dodecahedron(), 1.0 / 0.4398, 128)
    g.step(12)
    ob = g.observables()
    P = g.P_slices()
    g.close()
    lam, xi = O.correlation_length(P, "arpack")
    say(f"  gpu {ob['tm_lambda1']!r} {ob['tm_lambda2']!r} xi {ob['xi_e']!r} it {ob['tm_iterations']}; "
        f"arpack {lam[0]!r} {lam[1]!r} xi {xi!r}")
    assert ob["tm_converged"] == 1 and ob["tm_residual"] <= 1e-10
    assert abs(ob["tm_lambda1"] - lam[0]) <= 1e-11 * abs(lam[0])
    assert abs(ob["tm_lambda2"] - lam[1]) <= 1e-11 * abs(lam[0])
    assert abs(ob["xi_e"] - xi) <= 1e-9 * xi


@pytest.mark.parametrize("T", [3.0, 4.0])
def test_xi_ising_above_tc(T):
    ct = _lib()
    K = 1.0 / T
    say(f"[xi ising] T={T} m=32")
    g = ct.CTMRG(I.ising(), K, 32)
    g.run_to_fixed_point(1e-13, 4000)
    ob = g.observables()
    P = g.P_slices()
    g.close()
    lam, xi = O.correlation_length(P, "dense")
    exact = -1.0 / math.log(math.sinh(2 * K) ** 2)
    say(f"  gpu xi {ob['xi_e']!r} oracle {xi!r} exact (m -> inf) {exact!r}")
    assert abs(ob["xi_e"] - xi) <= 1e-10 * xi
    assert 0.97 * exact < ob["xi_e"] < exact
