"""Pins of the CPU oracle against what the physics and the mathematics fix (no GPU).

Each test checks the oracle against something other than itself: closed forms
(Onsager, Yang, the Ising-copy mappings of the cube and square models, the
four-state Potts duality of the tetrahedron model), brute-force partition
functions of small clusters, a library eigensolver on synthetic matrices, and
invariants stated in Sec. II of the paper (C real symmetric, rho PSD, the entropy
bound of Algorithm 3).  A plausible mistake -- a wrong leg order of W, a K/2
coupling, a dropped bond, a transposed operand, a wrong normalization -- fails
at least one of them (see test_planted_leg_order and test_planted_half_coupling).
"""
import math

import numpy as np
import pytest

import ctmrg_inputs as I
import exact as E
from oracle import ctmrg_oracle as O


# --------------------------------------------------------------------------- Jacobi

@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (7, 2), (60, 3), (151, 4)])
def test_jacobi_known_spectrum(n, seed):
    lam = I.graded_spectrum(seed, n)
    A = I.random_symmetric_with_spectrum(seed, lam)
    ev, vec = O.jacobi(A)
    scale = np.abs(lam).max()
    assert np.allclose(np.sort(ev), np.sort(lam), rtol=0, atol=1e-13 * scale * max(1, n) ** 0.5)
    assert np.abs(A @ vec - vec * ev).max() <= 1e-12 * scale
    assert np.abs(vec.T @ vec - np.eye(n)).max() <= 1e-12
    # the special case that reduces to a library routine
    assert np.allclose(np.sort(ev), np.linalg.eigvalsh(A), rtol=0, atol=1e-12 * scale)


def test_jacobi_degenerate_and_zero():
    A = np.zeros((5, 5))
    ev, vec = O.jacobi(A)
    assert np.all(ev == 0) and np.allclose(vec, np.eye(5))
    lam = np.array([2.0, 2.0, 2.0, -2.0, 0.0, 0.0, 1e-9])
    A = I.random_symmetric_with_spectrum(9, lam)
    ev, vec = O.jacobi(A)
    assert np.allclose(np.sort(ev), np.sort(lam), atol=1e-14)
    assert np.abs(vec.T @ vec - np.eye(7)).max() < 1e-13


def test_sort_and_cut():
    lam = np.array([0.5, -1.0, 1.0, 0.25, -0.25, 1e-20])
    order = O.sort_spectrum(lam)
    assert list(lam[order]) == [1.0, -1.0, 0.5, 0.25, -0.25, 1e-20]
    ls = lam[order]
    # |1| = |-1|: m=1 would split the pair, so nothing smaller than 2 is admissible
    assert O.cut_dimension(ls, 1, 1e-10, 1e-13) == 1  # fallback keeps the rank-limited count
    assert O.cut_dimension(ls, 2, 1e-10, 1e-13) == 2
    assert O.cut_dimension(ls, 4, 1e-10, 1e-13) == 3  # 0.25 / -0.25 pair would be split
    assert O.cut_dimension(ls, 6, 1e-10, 1e-13) == 5  # 1e-20 is below the rank threshold


# --------------------------------------------------------------------------- weight

def test_weight_values_and_symmetry():
    V = I.dodecahedron()
    q, K = 20, 1.0 / 0.4398
    W = O.weight(V, K)
    assert W.shape == (q, q, q, q)
    assert math.isclose(W[0, 0, 0, 0], math.exp(4 * K), rel_tol=1e-14)
    # dot products from one vertex: {1, sqrt5/3, 1/3, -1/3, -sqrt5/3, -1} with multiplicities {1,3,6,6,3,1}
    d = np.round(V @ V[0], 12)
    vals, counts = np.unique(d, return_counts=True)
    r5 = math.sqrt(5) / 3
    assert np.allclose(vals, [-1, -r5, -1 / 3, 1 / 3, r5, 1])
    assert list(counts) == [1, 3, 6, 6, 3, 1]
    # the plaquette's dihedral symmetry: cyclic order s -> sigma -> sigma' -> s'
    cyc = W.transpose(1, 3, 0, 2)      # (s,sigma,s',sigma') -> rotate the four corners
    assert np.allclose(W, cyc, rtol=1e-14)
    refl = W.transpose(1, 0, 3, 2)     # swap s<->sigma and s'<->sigma'
    assert np.allclose(W, refl, rtol=1e-14)
    Wm = O.weight_matrix(V, K)
    assert np.allclose(Wm, Wm.T)


# --------------------------------------------------------------------------- brute force

@pytest.mark.parametrize(
    "name,V,K,kmax,m",
    [
        ("ising", I.ising(), 0.4, 4, 64),
        ("three-vectors", I.tetrahedron()[:3], 0.7, 3, 27),
        ("tetrahedron", I.tetrahedron(), 0.9, 2, 16),
        ("dodecahedron", I.dodecahedron(), 1.0 / 0.44, 2, 20),
    ],
)
def test_bruteforce_clusters(name, V, K, kmax, m):
    """Untruncated CTMRG: ln Tr C'_k^4 = 4 ln b_k equals ln Z of the 2k x 2k cluster with fixed perimeter."""
    o = O.OracleCTMRG(V, K, m)
    for k in range(1, kmax + 1):
        o.step()
        assert np.all(np.abs(o.last.Pt - o.last.Pt.transpose(0, 2, 1)) <= 1e-12 * o.last.n_P)
        ref = E.cluster_lnZ_transfer(V, K, k)
        assert abs(4 * o.ln_b - ref) <= 1e-12 * abs(ref), (k, 4 * o.ln_b, ref)


def test_bruteforce_by_enumeration():
    V = I.ising()
    for k, K in [(1, 0.3), (1, 0.8)]:
        o = O.OracleCTMRG(V, K, 8)
        for _ in range(k):
            o.step()
        assert math.isclose(4 * o.ln_b, math.log(E.cluster_Z_enumerate(V, K, k)), rel_tol=1e-13)


def _literal_weight(V, K):
    """Algorithm 3's reshaping read literally: w_{(s,sigma),(s',sigma')} = W_{s sigma s' sigma'}
    with Eq. 1's cyclic order s, sigma, s', sigma' (so s' opposite s)."""
    G = V @ V.T
    return np.exp(K * (G[:, :, None, None] + G.T[None, :, :, None] + G[None, None, :, :]
                       + G.T[:, None, None, :]))


def test_planted_leg_order(monkeypatch):
    """The literal leg order builds a different network: it fails the brute-force pin at k=2."""
    V, K = I.tetrahedron()[:3], 0.7
    monkeypatch.setattr(O, "weight", _literal_weight)
    o = O.OracleCTMRG(V, K, 27)
    o.step()
    assert abs(4 * o.ln_b - E.cluster_lnZ_transfer(V, K, 1)) < 1e-12  # one vertex: same
    o.step()
    assert abs(4 * o.ln_b - E.cluster_lnZ_transfer(V, K, 2)) > 1e-3


def test_planted_half_coupling(monkeypatch):
    """A K/2 coupling (face weight on every plaquette) fails the Onsager pin."""
    real = O.weight
    monkeypatch.setattr(O, "weight", lambda V, K: real(V, 0.5 * K))
    o, obs = O.run_fixed_point(I.ising(), 0.5, 16, tol=1e-12)
    assert abs(obs["minus_beta_f"] - E.ising_minus_beta_f(0.5)) > 1e-2


# --------------------------------------------------------------------------- closed forms

@pytest.mark.parametrize("T,m", [(2.0, 16), (1.5, 12), (2.1, 24)])
def test_ising_onsager_yang(T, m):
    K = 1.0 / T
    o, obs = O.run_fixed_point(I.ising(), K, m, tol=1e-13)
    assert obs["converged"]
    assert abs(obs["minus_beta_f"] - E.ising_minus_beta_f(K)) <= 1e-10 * E.ising_minus_beta_f(K)
    assert abs(obs["E"] - E.ising_energy(K)) <= 1e-8
    assert abs(obs["M"] - E.ising_magnetization(K)) <= 1e-8
    assert abs(obs["ln_kappa_ratio"] - obs["ln_kappa_W"]) <= 1e-10


def test_ising_disordered():
    K = 1.0 / 2.5
    o, obs = O.run_fixed_point(I.ising(), K, 16, tol=1e-13)
    assert abs(obs["minus_beta_f"] - E.ising_minus_beta_f(K)) <= 1e-10 * E.ising_minus_beta_f(K)
    assert abs(obs["E"] - E.ising_energy(K)) <= 1e-8
    assert abs(obs["M"]) <= 1e-5


def test_ising_energy_is_dF_dK():
    """E per site = -d(-beta f)/dK: finite difference of the oracle's own free energy."""
    K, h = 0.5, 1e-4
    fp = O.run_fixed_point(I.ising(), K + h, 16, tol=1e-14)[1]["minus_beta_f"]
    fm = O.run_fixed_point(I.ising(), K - h, 16, tol=1e-14)[1]["minus_beta_f"]
    e = O.run_fixed_point(I.ising(), K, 16, tol=1e-14)[1]["E"]
    assert abs(-(fp - fm) / (2 * h) - e) < 1e-7


def test_ising_second_difference_of_F_is_the_closed_form():
    """d2(beta f)/dK2 by the second difference of the oracle's free energy (the reference the
    GPU derivative tests use at q = 20) against the K-derivative of Onsager's energy."""
    K, H = 0.5, 1e-3
    F = [-O.run_fixed_point(I.ising(), K + t * H, 16, tol=1e-14)[1]["minus_beta_f"] for t in (-1, 0, 1)]
    d2 = (F[0] - 2 * F[1] + F[2]) / (H * H)
    ref = E.ising_d2F_dK2(K)
    assert abs(d2 - ref) <= 1e-4 * abs(ref)


@pytest.mark.parametrize("T", [2.0, 1.5])
def test_ising_dM_dK_closed_form(T):
    """The derivative of Yang's magnetization in tests/exact.py (the reference of the GPU's dM/dK
    at q = 2) against the central difference of the oracle's M over fixed points at K +- h
    (h = 1e-5: M varies fast near T_c, so the difference's h^2 term is kept below 1e-7)."""
    K, h = 1.0 / T, 1e-5
    Mp = O.run_fixed_point(I.ising(), K + h, 16, tol=1e-14)[1]["M"]
    Mm = O.run_fixed_point(I.ising(), K - h, 16, tol=1e-14)[1]["M"]
    ref = E.ising_dM_dK(K)
    assert abs((Mp - Mm) / (2 * h) - ref) <= 1e-6 * abs(ref)


def test_cube_is_three_ising_copies():
    T = 0.6
    K = 1.0 / T
    o, obs = O.run_fixed_point(I.cube(), K, 27, tol=1e-12)
    assert abs(obs["minus_beta_f"] - 3 * E.ising_minus_beta_f(K / 3)) <= 1e-11
    assert abs(obs["E"] - E.ising_energy(K / 3)) <= 1e-9
    assert abs(obs["M"] - E.ising_magnetization(K / 3)) <= 1e-9


def test_square_is_two_ising_copies():
    K = 1.0
    o, obs = O.run_fixed_point(I.square(), K, 36, tol=1e-12)
    assert abs(obs["minus_beta_f"] - 2 * E.ising_minus_beta_f(K / 2)) <= 1e-12
    assert abs(obs["E"] - E.ising_energy(K / 2)) <= 1e-10
    assert abs(obs["M"] - E.ising_magnetization(K / 2)) <= 1e-10


def test_tetrahedron_potts_duality():
    """Off-critical pin of the q=4 tetrahedron model: f(K) - f(K*) from the Potts duality."""
    K = 1.0
    Ks = E.tetra_dual_K(K)
    assert 1.0 / Ks > E.TC_TETRA > 1.0 / K
    a = O.run_fixed_point(I.tetrahedron(), K, 32, tol=1e-12)[1]
    b = O.run_fixed_point(I.tetrahedron(), Ks, 32, tol=1e-12)[1]
    assert abs(a["minus_beta_f"] - b["minus_beta_f"] - E.tetra_duality_offset(K)) <= 1e-12


def test_tetrahedron_critical_point():
    """Ordered just below T_c = 4/(3 ln 3), disordered just above; E(T_c) = -4/3 (loose: critical)."""
    lo = O.run_fixed_point(I.tetrahedron(), 1.0 / (0.9 * E.TC_TETRA), 16, tol=1e-11)[1]
    hi = O.run_fixed_point(I.tetrahedron(), 1.0 / (1.1 * E.TC_TETRA), 16, tol=1e-11)[1]
    assert lo["M"] > 0.5 and abs(hi["M"]) < 1e-3
    # at criticality the finite-m error decays slowly (logarithmic corrections of the
    # four-state Potts class): only require it to shrink with m and stay within 3e-2
    c8 = O.run_fixed_point(I.tetrahedron(), 1.0 / E.TC_TETRA, 8, tol=1e-9, max_steps=4000)[1]
    c24 = O.run_fixed_point(I.tetrahedron(), 1.0 / E.TC_TETRA, 24, tol=1e-9, max_steps=4000)[1]
    assert abs(c24["E"] + 4.0 / 3.0) < abs(c8["E"] + 4.0 / 3.0) < 0.1
    assert abs(c24["E"] + 4.0 / 3.0) < 3e-2


# --------------------------------------------------------------------------- invariants

def test_invariants_dodecahedron():
    V = I.dodecahedron()
    o = O.OracleCTMRG(V, 1.0 / 0.5, 8)
    for _ in range(6):
        r = o.step(keep_cext=True)
        assert r.asym <= 1e-13
        assert math.isclose(np.sum(r.w ** 4), 1.0, rel_tol=1e-13)
        rank = int(np.sum(np.abs(r.lam) > 1e-13 * abs(r.lam[0])))
        assert -1e-15 <= r.S_E <= math.log(rank) + 1e-12
        assert np.abs(r.P - r.P.transpose(0, 2, 1)).max() <= 1e-12
        # rho = C'^4 is positive semi-definite
        assert np.all(r.lam ** 4 >= 0)
        assert np.abs(r.U.T @ r.U - np.eye(r.m_eff)).max() <= 1e-12


def _dodeca_obs(V, m=8, steps=40, s0=0):
    o = O.OracleCTMRG(V, 1.0 / 0.5, m, s0=s0)
    for _ in range(steps):
        o.step()
    return o.observables()


def test_relabelling_invariance():
    """Observables depend only on dot products: a vertex permutation (boundary spin kept) and a
    global rotation leave them unchanged; so does moving the boundary to any other vertex."""
    V = I.dodecahedron()
    ref = _dodeca_obs(V)
    perm = I.random_permutation(3, 20)
    a = _dodeca_obs(V[perm])
    b = _dodeca_obs(V @ I.random_rotation(5).T)
    c = _dodeca_obs(V, s0=13)
    for obs in (a, b, c):
        for key in ("f", "E", "M", "S_E", "ln_kappa_ratio"):
            assert abs(obs[key] - ref[key]) <= 1e-10 * max(1.0, abs(ref[key])), key


def test_free_and_fixed_boundary_agree_above_tc():
    K = 1.0 / 2.8
    a = O.run_fixed_point(I.ising(), K, 16, bc="fixed", tol=1e-13)[1]
    b = O.run_fixed_point(I.ising(), K, 16, bc="free", tol=1e-13)[1]
    assert abs(a["f"] - b["f"]) <= 1e-11 * abs(a["f"])
    assert abs(b["M"]) < 1e-8


# --------------------------------------------------------------------------- entanglement entropy (Eq. 6)

def _two_state_entropy(K):
    """First step of the fixed-boundary Ising run by hand: with P = [1] on the boundary spin,
    C'[(s'),(sigma')] = exp(K (1 + v_sigma' + v_sigma' v_s' + v_s')) = [[e^{4K}, 1], [1, 1]].
    Its eigenvalues solve l^2 - (a + 1) l + (a - 1) = 0, a = e^{4K}; rho = C'^4 / Tr C'^4
    has the two weights p = l_+^4 / (l_+^4 + l_-^4) and 1 - p."""
    a = math.exp(4.0 * K)
    r = math.sqrt((a - 1.0) ** 2 + 4.0)
    lp, lm = 0.5 * (a + 1.0 + r), 0.5 * (a + 1.0 - r)
    p = lp ** 4 / (lp ** 4 + lm ** 4)
    return -p * math.log(p) - (1.0 - p) * math.log(1.0 - p)


@pytest.mark.parametrize("K", [0.2, 0.45])
def test_entropy_first_step_closed_form(K):
    o = O.OracleCTMRG(I.ising(), K, 4)
    r = o.step()
    assert r.lam.shape == (2,)
    assert abs(r.S_E - _two_state_entropy(K)) <= 1e-14


@pytest.mark.parametrize("T", [2.0, 1.5])
def test_entropy_ising_fixed_point_free_fermions(T):
    """At the Ising fixed point rho = C^4/Tr C^4 is Baxter's free-fermion corner density
    matrix: levels -ln(rho_j/rho_1) are sums of distinct 2 j eps, and S_E = -Tr rho ln rho is
    the sum over modes of ln(1+e^{-e_j}) + e_j/(e^{e_j}+1) (closed form in tests/exact.py)."""
    K = 1.0 / T
    o, obs = O.run_fixed_point(I.ising(), K, 32, tol=1e-14)
    assert abs(obs["S_E"] - E.ising_ctm_entropy(K)) <= 1e-12
    w4 = np.sort(o.last.w ** 4)[::-1]
    levels = -np.log(w4[:6] / w4[0])
    assert np.abs(levels - E.ising_ctm_levels(K, 6)).max() <= 1e-7


@pytest.mark.parametrize("V,K,m,steps", [(I.tetrahedron(), 0.5, 16, 2), (I.dodecahedron(), 2.0, 8, 1),
                                         (I.cube(), 1.0, 8, 2)])
def test_entropy_is_von_neumann_of_rho(V, K, m, steps):
    """Eq. 6 by a different route: rho = C'^4 / Tr C'^4 formed as a matrix and
    S = -Tr(rho logm(rho)) with the matrix logarithm, on the step's own extended corner."""
    from scipy import linalg
    import warnings
    o = O.OracleCTMRG(V, K, m)
    for _ in range(steps):
        r = o.step(keep_cext=True)
    C = 0.5 * (r.cext + r.cext.T)
    C4 = np.linalg.matrix_power(C, 4)
    rho = C4 / np.trace(C4)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        S = -float(np.trace(rho @ linalg.logm(rho)).real)
    assert abs(r.S_E - S) <= 1e-13


def test_entropy_maximal_for_equal_weights():
    """The bound of Algorithm 3 is attained by a flat spectrum: n equal |omega| give ln n."""
    for n in (1, 2, 7, 160):
        w = np.full(n, n ** -0.25)
        w[::3] *= -1.0
        assert abs(O.entropy(w) - math.log(n)) <= 1e-13 * max(1.0, math.log(n))


@pytest.mark.parametrize("planted", ["ln_w", "w_squared"])
def test_planted_entropy_mistakes(monkeypatch, planted):
    """-sum w^4 ln w (a factor 4 off) and -sum w^2 ln w^4 fail the closed forms above."""
    def ln_w(w):
        w4 = w ** 4
        nz = w4 > 0
        return float(-np.sum(w4[nz] * np.log(np.abs(w[nz]))))

    def w_squared(w):
        w2 = w ** 2
        nz = w2 > 0
        return float(-np.sum(w2[nz] * np.log(w2[nz] ** 2)))

    monkeypatch.setattr(O, "entropy", {"ln_w": ln_w, "w_squared": w_squared}[planted])
    o = O.OracleCTMRG(I.ising(), 0.45, 4)
    r = o.step()
    assert abs(r.S_E - _two_state_entropy(0.45)) > 1e-3
    o, obs = O.run_fixed_point(I.ising(), 0.5, 32, tol=1e-14)
    assert abs(obs["S_E"] - E.ising_ctm_entropy(0.5)) > 1e-4


def test_fix_signs_hand_values():
    """The gauge convention: each column is negated when its entry of largest magnitude (the
    first one among equals) is negative; columns are otherwise unchanged."""
    U = np.array([[0.6, -0.8, 0.5], [-0.8, 0.6, -0.5], [0.0, 0.0, 0.0]])
    F = O.fix_signs(U)
    assert np.array_equal(F[:, 0], [-0.6, 0.8, 0.0])
    assert np.array_equal(F[:, 1], [0.8, -0.6, 0.0])
    assert np.array_equal(F[:, 2], [0.5, -0.5, 0.0])


# --------------------------------------------------------------------------- xi_e (Sec. II, last paragraph)

def _untruncated(V, K, steps):
    """The oracle's state after `steps` steps from the fixed boundary with m large enough that
    nothing is cut (m = q^steps)."""
    q = len(V)
    o = O.OracleCTMRG(V, K, q ** steps, eig="lapack")
    for _ in range(steps):
        o.step()
    assert o.P.shape[1] == q ** steps
    return o


@pytest.mark.parametrize("name,T,steps", [("ising", 2.5, 1), ("ising", 2.0, 2), ("ising", 3.0, 3),
                                          ("ising", 1.7, 4), ("tetrahedron", 1.0, 2),
                                          ("dodecahedron", 0.44, 1)])
def test_row_transfer_matrix_brute_force(name, T, steps):
    """After k untruncated steps, sum_s P_s (x) P_s -- built from the rotated, normalized
    half-rows of the iteration -- has the spectrum (up to one scale) of the straight row of
    2k vertices with fixed ends, enumerated directly from the weights."""
    V = I.vertices(name)
    K = 1.0 / T
    o = _untruncated(V, K, steps)
    Tg = O.row_transfer_matrix(o.P)
    Tb = E.row_transfer_bruteforce(V, K, 0, 2 * steps)
    assert Tg.shape == Tb.shape
    a = np.linalg.eigvalsh(Tg)
    b = np.linalg.eigvalsh(Tb)
    a = a[np.argsort(-np.abs(a), kind="stable")]
    b = b[np.argsort(-np.abs(b), kind="stable")]
    a, b = a / a[0], b / b[0]
    assert np.abs(np.sort(a) - np.sort(b)).max() <= 1e-12
    # the operator form and the explicit matrix agree; ARPACK finds the same leading pair
    X = np.random.default_rng(7).standard_normal((o.P.shape[1],) * 2)
    assert np.allclose(O.row_transfer_apply(o.P, X).ravel(), Tg @ X.ravel(), rtol=0, atol=1e-13 * np.abs(Tg).max() * X.size)
    if Tg.shape[0] >= 16:
        lam_d, xi_d = O.correlation_length(o.P, "dense")
        lam_a, xi_a = O.correlation_length(o.P, "arpack")
        assert np.allclose(lam_a, lam_d, rtol=1e-11, atol=0)


def test_planted_row_transfer_mistakes():
    """A row made of two unrelated half-rows (no shared end spin), or of the boundary spin's
    half-row alone, fails the brute force."""
    V = I.ising()
    K = 1.0 / 2.0
    o = _untruncated(V, K, 3)
    P = o.P
    b = np.linalg.eigvalsh(E.row_transfer_bruteforce(V, K, 0, 6))
    b = np.sort(b / b[np.argmax(np.abs(b))])
    for bad in (sum(np.kron(P[s], P[t]) for s in range(2) for t in range(2)), np.kron(P[0], P[0])):
        a = np.linalg.eigvalsh(bad)
        a = np.sort(a / a[np.argmax(np.abs(a))])
        assert np.abs(a - b).max() > 1e-3


@pytest.mark.parametrize("T,ordered", [(4.0, False), (3.0, False), (1.8, True)])
def test_ising_correlation_length_closed_form(T, ordered):
    """q = 2: |lambda_2 / lambda_1| of the row-to-row transfer matrix tends, as m grows, to
    the exact value of the infinite lattice.  A row of vertices runs along a diagonal of the
    spin lattice, so the ratio is sinh^2(2K) above T_c (one free fermion at the bottom of its
    band) and sinh^-4(2K) below (two; the fixed boundary selects one ordered state).  The
    finite-m band of the transfer matrix starts above the exact edge, so the ratio approaches
    from below."""
    K = 1.0 / T
    exact = math.sinh(2 * K) ** (-4) if ordered else math.sinh(2 * K) ** 2
    prev = 0.0
    errs = []
    for m in (8, 16, 32):
        o, _ = O.run_fixed_point(I.ising(), K, m, tol=1e-13, max_steps=4000, eig="lapack")
        lam, xi = O.correlation_length(o.P)
        r = abs(lam[1] / lam[0])
        assert abs(xi - 1.0 / math.log(1.0 / r)) <= 1e-12 * xi
        errs.append(r / exact - 1.0)
        assert prev < r < exact
        prev = r
    assert abs(errs[-1]) <= (0.04 if ordered else 0.01)
    assert abs(errs[-1]) < abs(errs[0]) / 2.5


def test_impurity_energy_is_dF_dK_and_its_derivative_is_d2F_dK2_q20():
    """The identity the GPU's second derivative rests on (dF/dK equals the impurity energy E at
    every fixed point, so d2F/dK2 = dE/dK), on the oracle's own q = 20, m = 12 fixed points at
    K and K +- h (tests/golden, converged to 1e-13): the central difference of F equals E at K, and
    the second difference of F equals the central difference of E, to the accuracy of the
    differences (h^2 terms and 1e-13 / h^2 of convergence noise)."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "derivative_q20_m12_T0.40.npz")
    with np.load(path, allow_pickle=False) as z:
        r = {k: float(z[k]) for k in ("h", "F_0", "F_p", "F_m", "E_0", "E_p", "E_m")}
    h = r["h"]
    dF = (r["F_p"] - r["F_m"]) / (2 * h)
    d2F = (r["F_p"] - 2 * r["F_0"] + r["F_m"]) / h ** 2
    dE = (r["E_p"] - r["E_m"]) / (2 * h)
    assert abs(dF - r["E_0"]) <= 1e-7
    assert abs(d2F - dE) <= 2e-4 * abs(dE)
    # and not by accident: the energy is not the free energy's value, and E changes with K
    assert abs(r["E_0"] - r["F_0"]) > 1.0 and abs(dE) > 0.1
