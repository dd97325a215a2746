"""COD convergence under adaptive and global refinement (Section 4.4) on a 10 x 10 domain with
l0 = 1, eps = 2 h_min: the errors against each family's Richardson reference fall faster than
linearly in h at the crack centre and half-way to the tip, half-way to the tip the adaptive family
converges quadratically in h (the paper's statement), both families agree at every common h
(the same resolution at the crack), and the adaptive family gets there with fewer DoFs.  The
Newton solves themselves are parity-checked against the oracle elsewhere."""
import numpy as np
import pytest

from paper_1806_09924_amd import studies
from inputs import cod_study

pytestmark = pytest.mark.gpu


def test_cod_convergence_adaptive_and_global():
    c = cod_study()
    out = studies.cod_convergence(c["half_width"], c["levels"], c["refine_radius"])
    ad, gl = out["adaptive"], out["global_"]
    for fam in (ad, gl):
        for k in range(len(out["xs"])):
            assert all(o > 1.1 for o in fam["orders"][k]["vs_h"]), fam["orders"][k]
    assert 1.5 <= ad["order_richardson"][1] <= 2.5, ad["order_richardson"]
    n = len(gl["h"])
    assert ad["h"][:n] == gl["h"]
    for k in range(len(out["xs"])):
        a, g = np.array(ad["cod"][k][:n]), np.array(gl["cod"][k])
        assert np.abs(a / g - 1).max() <= 5e-3
        assert abs(ad["reference"][k] / gl["reference"][k] - 1) <= 5e-3
    assert all(a < g for a, g in zip(ad["n_dofs"][:n], gl["n_dofs"]))
    # Sneddon's centre opening 2 p l0 (1 - nu^2) / E, less the finite-domain effect
    exact = 2 * 1e-3 * 1.0 * (1 - 0.2 ** 2)
    assert 0.0 < 1 - ad["reference"][0] / exact <= 0.08
