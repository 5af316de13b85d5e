"""A caller-owned device workspace (ctmrg_options.workspace) through the C ABI.

The context carves every buffer of ctmrg_init from the caller's memory (a torch tensor here);
the arithmetic is the same, so the steps, the state and the observables equal, bit for bit,
those of a context that allocates its own buffers.  A workspace smaller than
ctmrg_workspace_size is refused.
"""
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
    return ctmrg, torch


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("m,prec,eig", [(24, "fp64", "two_stage"), (24, "fp32", "warm"), (64, "fp64", "warm")])
def test_workspace_equals_own_buffers(m, prec, eig):
    ct, torch = _lib()
    V, K = I.dodecahedron(), 1.0 / 0.44
    nbytes = ct.workspace_size(20, m, precision=prec, eig=eig)
    say(f"[workspace] m={m} {prec} {eig}: {nbytes / 1e6:.1f} MB")
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    a = ct.CTMRG(V, K, m, precision=prec, eig=eig)
    b = ct.CTMRG(V, K, m, precision=prec, eig=eig, workspace=ws)
    a.step(30)
    b.step(30)
    oa, ob = a.observables(), b.observables()
    assert np.array_equal(a.get("P"), b.get("P"))
    assert np.array_equal(a.get("omega"), b.get("omega"))
    for key in ("f", "E", "M", "S_E", "xi_e"):
        assert oa[key] == ob[key], key
    a.close()
    b.close()
    del ws


def test_workspace_too_small():
    ct, torch = _lib()
    nbytes = ct.workspace_size(20, 16)
    ws = torch.empty(nbytes - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(ct.CTMRGError) as e:
        ct.CTMRG(I.dodecahedron(), 2.0, 16, workspace=ws)
    assert e.value.status == 1
