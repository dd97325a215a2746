"""The 3d penny-crack convergence of Fig. 3 (Section 4.3) on one GPU under the quasi-static
reading of Sneddon's test: loading steps at the constant pressure until the phase field is
stationary (the first step sees the sharp initial band in its degradation and pressure terms;
the later ones relax it to the regularised profile).  Refs 7-9 in one batch and ref 10 alone:
the eps column of the table is reproduced (2 x the finest cell's diameter), the errors against
Sneddon's TCV are positive and shrink with eps as the table's do, and every ref's TCV is within
3 % of the table's value (measured: -2.2 %, -1.6 %, -1.4 %, -1.3 %; errors +32.0 / +11.7 /
+3.5 / +0.4 % against the table's +35.0 / +13.4 / +5.0 / +1.8 %).  A single Newton loop from the
sharp band (the first step) converges from below instead (-14.7 ... -5.5 %)."""
import os

import numpy as np
import pytest

from paper_1806_09924_amd import studies

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fig3_table.txt")
STEPS = 6


def _table():
    rows = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        rows[int(f[0])] = dict(ten_l0_over_h=int(f[1]), dofs=int(f[2]), eps=float(f[3]), tcv=float(f[4]),
                               err=float(f[5]) / 100)
    return rows


def _check_rows(rows, tab):
    for r in rows:
        t = tab[r["ref"]]
        assert r["ten_l0_over_h"] == t["ten_l0_over_h"]
        assert abs(r["eps"] / t["eps"] - 1) < 1e-4
        assert abs(r["tcv"] / t["tcv"] - 1) <= 0.03, (r["ref"], r["tcv"], t["tcv"])
        assert r["rel_error"] > 0                              # from above, as the table
        assert r["rel_error_first_step"] < 0                   # the sharp band alone: from below
        ts = r["tcv_steps"]
        assert abs(ts[-1] / ts[-2] - 1) <= 1e-8                # stationary


def test_convergence_3d_quasistatic_refs_7_to_10():
    tab = _table()
    out = studies.convergence_3d((7, 8, 9), refine_radius=0.4, precision=32, steps=STEPS)
    assert abs(out["exact"] / 5.12e-3 - 1) < 1e-12
    rows = out["rows"]
    _check_rows(rows, tab)
    # the finest mesh of the batch is of the table's size
    assert abs(rows[-1]["n_dofs"] / tab[9]["dofs"] - 1) <= 0.05
    out10 = studies.convergence_3d((10,), refine_radius=0.4, precision=32, steps=STEPS)
    _check_rows(out10["rows"], tab)
    errs = [r["rel_error"] for r in rows + out10["rows"]]
    assert all(a > b for a, b in zip(errs, errs[1:]))
    assert errs[-1] <= 0.02


def test_convergence_3d_ref_11_at_the_table_size():
    """Ref 11 (h_min = 10/2048) with the refinement radius cut to 0.12 so that the mesh has the
    table's size (34.8 M DoFs against 30.3 M; radius 0.4 would need about 4x that, beyond one
    GPU's memory for the 3d hierarchy).  The eps column and the table's TCV within 3 % hold and
    the phase field is stationary; the error against Sneddon is -1.3 % here, below the table's
    +0.72 %: with the mesh coarsened 0.12 away from the crack the far field's discretisation
    error (which lowers the TCV) outweighs the eps error at this size (ref 10 with radius 0.4:
    +0.4 %).  The device pool is handed back at the end."""
    tab = _table()
    try:
        out = studies.convergence_3d((11,), refine_radius=0.12, precision=32, steps=STEPS)
        (r,) = out["rows"]
        t = tab[11]
        assert r["ten_l0_over_h"] == t["ten_l0_over_h"]
        assert abs(r["eps"] / t["eps"] - 1) < 1e-4
        assert abs(r["n_dofs"] / t["dofs"] - 1) <= 0.20
        assert abs(r["tcv"] / t["tcv"] - 1) <= 0.03, (r["tcv"], t["tcv"])
        assert abs(r["rel_error"]) <= 0.02
        ts = r["tcv_steps"]
        assert abs(ts[-1] / ts[-2] - 1) <= 1e-8
    finally:
        import gc
        from paper_1806_09924_amd import binding as B
        gc.collect()
        B.trim_pool()
