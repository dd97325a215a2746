"""Host arithmetic of the studies: Richardson extrapolation (Section 4.2 and 4.4 reference
values) against sequences with a known limit and order."""
import numpy as np
import pytest

from paper_1806_09924_amd.studies import richardson


@pytest.mark.parametrize("q", [1.0, 1.5, 2.0, 3.0])
def test_richardson_recovers_limit_and_order(q):
    c_star, a = 1.8877e-3, -2.3e-4
    h = 0.125 / 2.0 ** np.arange(5)
    c = c_star + a * h ** q
    ref, order = richardson(c)
    assert abs(order - q) <= 1e-9
    assert abs(ref - c_star) <= 1e-12 * abs(c_star)


def test_richardson_rejects_non_monotone_sequences():
    with pytest.raises(ValueError):
        richardson([1.0, 1.1, 1.05])
    with pytest.raises(ValueError):
        richardson([1.0, 1.0, 1.0])
