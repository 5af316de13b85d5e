"""Host logic of the sweep driver (paper_2004_08669_amd/sweep.py) with the library replaced by a
stand-in that returns fixed observables: one call per temperature, the central-difference checks
on the requested temperatures, the per-temperature summary (derivatives only where they were
computed) and the JSON written after every temperature.  No GPU."""
import json

import numpy as np

from paper_2004_08669_amd import sweep


class FakeContext:
    calls = []

    def __init__(self, V, K, m, precision="fp64", eig="two_stage", gap_tol=None):
        self.K = K
        self.state = None

    def sweep(self, Ts, tol, max_steps, warm_start=True, derivative=False):
        out = []
        for T in Ts:
            FakeContext.calls.append(T)
            K = 1.0 / T
            # F = K f = -K^2 (an exact quadratic: its central difference is exact)
            p = {"T": T, "steps": 10, "converged": T != 0.43, "delta": 1e-13, "m_eff": 4, "f": -K,
                 "E": -2.0 * K, "M": 0.5, "S_E": 0.1, "xi_e": 2.0}
            if derivative:
                ok = p["converged"]
                p["derivative"] = {"dF_dK": -2.0 * K if ok else 0.0, "d2F_dK2": -2.0 if ok else 0.0,
                                   "dM_dK": 0.1 if ok else 0.0, "iterations": 12 if ok else 0,
                                   "aligned_steps": 3, "status": 0}
            out.append(p)
        return out

    def export_state(self):
        return b"state"

    def import_state(self, st):
        self.state = st

    def close(self):
        pass


def test_sweep_driver_summary(tmp_path, monkeypatch):
    monkeypatch.setattr(sweep.ctmrg, "CTMRG", FakeContext)
    FakeContext.calls = []
    out = tmp_path / "s.json"
    Ts = [0.40, 0.43, 0.46]
    res = sweep.run(np.zeros((2, 1)), 8, Ts, 1e-12, 100, fd_every=2, dK=1e-3, out_path=str(out))
    # one call per temperature, then K +- dK around the checked ones (T = 0.40 and 0.46)
    assert FakeContext.calls[0] == 0.40 and 0.43 in FakeContext.calls and len(FakeContext.calls) == 3 + 2 * 2
    rows = res["points"]
    assert [r["T"] for r in rows] == Ts
    assert rows[1]["derivative"] is False and rows[1]["dF_dK"] is None
    assert rows[0]["derivative"] and abs(rows[0]["dF_dK"] - (-5.0)) < 1e-12
    assert abs(rows[0]["specific_heat"] - 2.0 / 0.40 ** 2) < 1e-12
    assert res["max_abs_dF_dK_minus_E"] == 0.0
    assert len(res["central_difference_checks"]) == 2
    for c in res["central_difference_checks"]:
        assert c["abs_diff"] < 1e-9
    on_disk = json.loads(out.read_text())
    assert on_disk["points"] == json.loads(json.dumps(rows))


def test_sweep_driver_grid(tmp_path, monkeypatch):
    """The (T, m) grid: one context per cutoff in order, observables only, the file holding every
    finished cutoff."""
    made = []

    class GridContext(FakeContext):
        def __init__(self, V, K, m, **kw):
            super().__init__(V, K, m, **kw)
            made.append(m)

    monkeypatch.setattr(sweep.ctmrg, "CTMRG", GridContext)
    FakeContext.calls = []
    out = tmp_path / "g.json"
    Ts = [0.40, 0.46]
    res = sweep.run_grid(np.zeros((2, 1)), [8, 16], Ts, 1e-12, 100, fd_every=1, dK=1e-3, out_path=str(out),
                         derivative=False)
    assert made == [8, 16]
    assert FakeContext.calls == Ts + Ts  # no central-difference contexts without derivatives
    assert [g["m"] for g in res["grid"]] == [8, 16]
    for g in res["grid"]:
        assert [r["T"] for r in g["points"]] == Ts
        assert all(r["derivative"] is False and r["dF_dK"] is None for r in g["points"])
        assert g["central_difference_checks"] == [] and g["max_abs_dF_dK_minus_E"] is None
    on_disk = json.loads(out.read_text())
    assert [g["m"] for g in on_disk["grid"]] == [8, 16]


def test_sweep_cli_cutoff_sets(monkeypatch):
    """--set A/B name the paper's two cutoff sets over 0.35 <= T <= 0.56."""
    seen = {}

    def fake_grid(V, ms, Ts, *a, **kw):
        seen.update(ms=list(ms), Ts=list(Ts), derivative=kw["derivative"])
        return {"grid": []}

    monkeypatch.setattr(sweep, "run_grid", fake_grid)
    monkeypatch.setattr(sweep, "vertex_set", lambda name: np.zeros((20, 3)))
    sweep.main(["--set", "A", "--n", "22", "--no-derivative"])
    assert seen["ms"] == [120, 240, 500, 800] and seen["derivative"] is False
    assert abs(seen["Ts"][0] - 0.35) < 1e-15 and abs(seen["Ts"][-1] - 0.56) < 1e-15 and len(seen["Ts"]) == 22
    sweep.main(["--set", "B", "--n", "3"])
    assert seen["ms"] == [500, 600, 700, 800] and seen["derivative"] is True


def test_sweep_cli_cutoff_list(monkeypatch):
    """--m takes one cutoff (a plain scan over 0.40-0.48) or a comma-separated list (a grid)."""
    seen = {}

    def fake_run(V, m, Ts, *a, **kw):
        seen.update(kind="run", ms=[m], Ts=list(Ts))
        return {"points": []}

    def fake_grid(V, ms, Ts, *a, **kw):
        seen.update(kind="grid", ms=list(ms), Ts=list(Ts))
        return {"grid": []}

    monkeypatch.setattr(sweep, "run", fake_run)
    monkeypatch.setattr(sweep, "run_grid", fake_grid)
    monkeypatch.setattr(sweep, "vertex_set", lambda name: np.zeros((20, 3)))
    sweep.main(["--m", "64", "--n", "5"])
    assert seen["kind"] == "run" and seen["ms"] == [64] and len(seen["Ts"]) == 5
    assert abs(seen["Ts"][0] - 0.40) < 1e-15 and abs(seen["Ts"][-1] - 0.48) < 1e-15
    sweep.main(["--m", "120,240", "--n", "2", "--T0", "0.5", "--T1", "0.6"])
    assert seen["kind"] == "grid" and seen["ms"] == [120, 240] and seen["Ts"] == [0.5, 0.6]
