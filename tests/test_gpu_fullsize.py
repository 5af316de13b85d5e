"""The FP64 path at the size the bench times: q = 20, m = 512 (C' 10240 x 10240), band 16, and at the
paper's largest cutoff, m = 800 (C' 16000 x 16000).

The oracle cannot run a step at this size in a test, so the checks are the outputs it can
compute one by one and properties that hold at any size:
  * sampled entries of C' against the oracle's one-entry formula, and the symmetry of C';
  * the spectrum of C' against its trace and Frobenius norm (sum lambda = Tr C',
    sum lambda^2 = ||C'||_F^2);
  * the kept eigenpairs: residuals ||C' u - lambda u|| and orthonormality;
  * the normalization omega = lambda / (sum lambda^4)^(1/4) and the symmetry of the new P slices;
  * that the kept set is the true top m_eff by modulus, from Sylvester's law of inertia: with t
    between |lambda_{m_eff}| and |lambda_{m_eff+1}|, the LDL^T factorizations (Bunch-Kaufman,
    on the host) of C' - t I and C' + t I count the eigenvalues above t and below -t, and
    together they must be m_eff;
  * n_C: sum lambda^4 against ||C'^2||_F^2 from one host product.
Tolerances: backward errors of order N u ||C'|| with N = 10240, u = 1.1e-16 (about 1e-12 ||C'||),
with a factor ten of margin.
"""
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


def _inertia(D):
    """(positive, negative) eigenvalue counts of the block-diagonal D of an LDL^T factorization
    (1 x 1 and 2 x 2 blocks)."""
    n = D.shape[0]
    sub = np.diag(D, -1)
    pos = neg = 0
    i = 0
    while i < n:
        if i + 1 < n and sub[i] != 0.0:
            ev = np.linalg.eigvalsh(np.array([[D[i, i], D[i + 1, i]], [D[i + 1, i], D[i + 1, i + 1]]]))
            pos += int(np.sum(ev > 0))
            neg += int(np.sum(ev < 0))
            i += 2
        else:
            pos += int(D[i, i] > 0)
            neg += int(D[i, i] < 0)
            i += 1
    return pos, neg


def test_fullsize_m512_step():
    ct = _lib()
    V = I.dodecahedron()
    q, m, K = 20, 512, 1.0 / 0.4398
    N = q * m
    say("[full size] q=20 m=512 T=0.4398: 5 steps")
    g = ct.CTMRG(V, K, m)
    g.step(5)
    st = g.export_state()
    P = g.P_slices()
    om = g.get("omega")
    say("  extended corner of the next step")
    g.extend()
    C = g.get("cext")
    cmax = float(np.abs(C).max())
    # sampled entries against the definition
    W = O.weight(V, K)
    rng = np.random.default_rng(0)
    worst = 0.0
    for _ in range(200):
        r, c = int(rng.integers(N)), int(rng.integers(N))
        worst = max(worst, abs(C[r, c] - O.extend_entry(W, P, om, r, c)))
    say(f"  sampled entries: max |C' - oracle| = {worst:.3e} (max |C'| = {cmax:.3e})")
    assert worst <= 1e-13 * cmax
    asym = 0.0
    for i0 in range(0, N, 1024):
        asym = max(asym, float(np.abs(C[i0:i0 + 1024, :] - C[:, i0:i0 + 1024].T).max()))
    say(f"  max |C' - C'^T| = {asym:.3e}")
    assert asym <= 1e-13 * cmax
    trace = float(np.trace(C))
    fro2 = float(np.sum(C * C))
    say("  one step from the same state")
    g.import_state(st)
    g.step(1)
    lam = g.get("spectrum")
    U = g.get("U")
    omn = g.get("omega")
    Pn = g.P_slices()
    g.close()
    me = int(np.count_nonzero(omn))
    l1 = float(np.abs(lam).max())
    say(f"  m_eff {me}; sum lambda {lam.sum():.15e} vs trace {trace:.15e}; "
        f"sum lambda^2 {np.sum(lam * lam):.15e} vs ||C'||_F^2 {fro2:.15e}")
    assert abs(lam.sum() - trace) <= 1e-11 * np.abs(lam).sum()
    assert abs(np.sum(lam * lam) - fro2) <= 1e-11 * fro2
    nC = float(np.sum(lam ** 4) ** 0.25)
    order = np.lexsort((-lam, -np.abs(lam)))
    lk = lam[order][:me]
    assert np.abs(omn[:me] - lk / nC).max() <= 1e-12
    Uk = U[:, :me]
    R = C @ Uk - Uk * lk[None, :]
    res = float(np.linalg.norm(R, axis=0).max())
    orth = float(np.abs(Uk.T @ Uk - np.eye(me)).max())
    say(f"  kept residual max ||C'u - lambda u|| = {res:.3e} (|lambda_1| = {l1:.3e}); ||U^T U - I|| = {orth:.3e}")
    assert res <= 1e-11 * l1
    assert orth <= 1e-11
    # the kept set is the top m_eff by modulus (inertia), and n_C from ||C'^2||_F
    from scipy import linalg
    mags = np.sort(np.abs(lam))[::-1]
    t = 0.5 * (mags[me - 1] + mags[me])
    say(f"  inertia at t = {t:.6e} (|lambda_m_eff| = {mags[me - 1]:.6e}, next {mags[me]:.6e})")
    Ct = C.copy()
    Ct[np.diag_indices(N)] -= t
    _, D, _ = linalg.ldl(Ct, lower=True, overwrite_a=True, check_finite=False)
    above, _ = _inertia(D)
    Ct = C.copy()
    Ct[np.diag_indices(N)] += t
    _, D, _ = linalg.ldl(Ct, lower=True, overwrite_a=True, check_finite=False)
    _, below = _inertia(D)
    del Ct, D
    say(f"  eigenvalues above t: {above}, below -t: {below}; m_eff {me}")
    assert above + below == me
    C2 = C @ C
    s4 = float(np.sum(C2 * C2))
    del C2
    say(f"  sum lambda^4 {np.sum(lam ** 4):.15e} vs ||C'^2||_F^2 {s4:.15e}")
    assert abs(np.sum(lam ** 4) - s4) <= 1e-12 * s4
    sym = float(np.abs(Pn - Pn.transpose(0, 2, 1)).max())
    say(f"  new P: max |P_s - P_s^T| = {sym:.3e}, max |P| = {np.abs(Pn).max():.3e}")
    assert sym <= 1e-12 * np.abs(Pn).max()
    assert abs(np.abs(Pn).max() - 1.0) <= 1e-15


def test_fullsize_m800_step():
    """The paper's largest cutoff, m = 800 (C' 16000 x 16000), FP64: the checks above that cost
    O(N^2 m) on the host (the inertia and ||C'^2||_F checks, O(N^3), are left to m = 512)."""
    ct = _lib()
    V = I.dodecahedron()
    q, m, K = 20, 800, 1.0 / 0.4398
    N = q * m
    say("[full size] q=20 m=800 T=0.4398: 4 steps")
    g = ct.CTMRG(V, K, m)
    g.step(4)
    st = g.export_state()
    P = g.P_slices()
    om = g.get("omega")
    g.extend()
    C = g.get("cext")
    cmax = float(np.abs(C).max())
    W = O.weight(V, K)
    rng = np.random.default_rng(1)
    worst = 0.0
    for _ in range(100):
        r, c = int(rng.integers(N)), int(rng.integers(N))
        worst = max(worst, abs(C[r, c] - O.extend_entry(W, P, om, r, c)))
    asym = max(float(np.abs(C[i0:i0 + 2000, :] - C[:, i0:i0 + 2000].T).max()) for i0 in range(0, N, 2000))
    say(f"  sampled entries: max |C' - oracle| = {worst:.3e}; max |C' - C'^T| = {asym:.3e} (max |C'| = {cmax:.3e})")
    assert worst <= 1e-13 * cmax
    assert asym <= 1e-13 * cmax
    trace = float(np.trace(C))
    fro2 = float(np.sum(C * C))
    g.import_state(st)
    g.step(1)
    lam = g.get("spectrum")
    U = g.get("U")
    omn = g.get("omega")
    Pn = g.P_slices()
    g.close()
    me = int(np.count_nonzero(omn))
    l1 = float(np.abs(lam).max())
    say(f"  m_eff {me}; trace identity {abs(lam.sum() - trace) / np.abs(lam).sum():.3e}, "
        f"Frobenius identity {abs(np.sum(lam * lam) - fro2) / fro2:.3e}")
    assert abs(lam.sum() - trace) <= 1e-11 * np.abs(lam).sum()
    assert abs(np.sum(lam * lam) - fro2) <= 1e-11 * fro2
    nC = float(np.sum(lam ** 4) ** 0.25)
    lk = lam[np.lexsort((-lam, -np.abs(lam)))][:me]
    assert np.abs(omn[:me] - lk / nC).max() <= 1e-12
    Uk = U[:, :me]
    res = float(np.linalg.norm(C @ Uk - Uk * lk[None, :], axis=0).max())
    orth = float(np.abs(Uk.T @ Uk - np.eye(me)).max())
    say(f"  kept residual max {res:.3e} (|lambda_1| = {l1:.3e}); ||U^T U - I|| = {orth:.3e}")
    assert res <= 1e-11 * l1
    assert orth <= 1e-11
    sym = float(np.abs(Pn - Pn.transpose(0, 2, 1)).max())
    assert sym <= 1e-12 * np.abs(Pn).max()
    assert abs(np.abs(Pn).max() - 1.0) <= 1e-15
