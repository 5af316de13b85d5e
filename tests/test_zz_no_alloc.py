"""ctmrg_eigh_topk_noalloc (the eigensolver entry point that allocates nothing) against
ctmrg_eigh_topk on the same matrices, through the C ABI: two calls in a row, the second with
a smaller input, so that the second call runs on the device array the first one left behind."""
import numpy as np
import pytest

import ctmrg_inputs as I

pytestmark = pytest.mark.gpu


def _lib():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2004_08669_amd import ctmrg
    ctmrg.load()
    return ctmrg


@pytest.mark.parametrize("band", [16, 32])
def test_noalloc_matches_allocating_entry_point(band):
    ct = _lib()
    cases = [(1000, 128, 11), (333, 40, 12)]  # the second call is smaller than the first
    for n, k, seed in cases:
        lam = I.graded_spectrum(seed, n, ratio=0.95)
        A = I.random_symmetric_with_spectrum(seed, lam)
        print(f"[noalloc] n={n} k={k} band={band} seed={seed}", flush=True)
        ev0, kept0, U0 = ct.eigh_topk(A, k, band)
        ev1, kept1, U1 = ct.eigh_topk_noalloc(A, k, band)
        scale = np.abs(lam).max()
        d_ev = float(np.abs(ev1 - ev0).max())
        d_kept = float(np.abs(kept1 - kept0).max())
        # eigenvectors: the same sign convention on both; compare projectors of each
        # exactly degenerate pair through the residual and the subspace instead of elements
        res = float(np.abs(A @ U1 - U1 * kept1).max())
        orth = float(np.abs(U1.T @ U1 - np.eye(k)).max())
        proj = float(np.abs(U1 @ U1.T - U0 @ U0.T).max())
        print(f"  |d evals| {d_ev:.2e} |d kept| {d_kept:.2e} residual {res:.2e} orth {orth:.2e} "
              f"|d projector| {proj:.2e} bitwise {np.array_equal(U0, U1)}", flush=True)
        assert d_ev <= 1e-13 * scale
        assert d_kept <= 1e-13 * scale
        assert res <= 1e-12 * scale * np.sqrt(n)
        assert orth <= 1e-12
        assert proj <= 1e-10


def test_noalloc_rejects_sizes_beyond_its_maximum():
    ct = _lib()
    lib = ct.load()
    n = 1100
    A = np.eye(n)
    ev, kept, vec = np.empty(n), np.empty(4), np.empty((n, 4))
    st = lib.ctmrg_eigh_topk_noalloc(n, ct._p(A), 4, 0, ct._p(ev), ct._p(kept), ct._p(vec))
    assert st == 1  # CTMRG_E_INVALID_ARG
