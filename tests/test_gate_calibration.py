"""The surrogate gate's change threshold (host logic, no GPU): the largest
predicted change among calibration hops within the error bar that lies below the
change of every hop outside it."""
import numpy as np
import pytest

from paper_2004_11286_amd.surrogate import calibrate_change_tol


def hop(err, chg):
    return {"X_linf": err, "state_change": chg}


def test_no_hops_or_no_good_hop_gives_zero():
    assert calibrate_change_tol([]) == 0.0
    assert calibrate_change_tol([hop(2e-3, 1e-3), hop(5e-2, 0.2)]) == 0.0


def test_largest_good_change_below_every_bad_one():
    hops = [hop(5e-2, 0.2), hop(3e-3, 6e-3), hop(8e-4, 2e-3), hop(5e-4, 1e-3), hop(9e-4, 3e-3)]
    assert calibrate_change_tol(hops) == 3e-3
    # a bad hop with a smaller change caps the threshold below it
    hops.append(hop(1.2e-3, 2.5e-3))
    assert calibrate_change_tol(hops) == 2e-3


def test_a_good_hop_tied_with_a_bad_one_is_not_admitted():
    assert calibrate_change_tol([hop(1e-4, 2e-3), hop(2e-3, 2e-3), hop(1e-4, 1e-3)]) == 1e-3


def test_the_bar_is_inclusive():
    assert calibrate_change_tol([hop(1e-3, 4e-3), hop(1.0000001e-3, 5e-3)]) == 4e-3


@pytest.mark.parametrize("seed", range(20))
def test_every_admitted_calibration_hop_is_within_the_bar(seed):
    """On random hop sets (error loosely growing with the change, as the
    network's does), every hop whose change is at most the threshold is good,
    and no larger threshold has that property."""
    rng = np.random.default_rng(seed)
    chg = 10.0 ** rng.uniform(-3.5, -0.5, size=int(rng.integers(1, 40)))
    err = chg * 10.0 ** rng.uniform(-1.0, 0.2, size=chg.size)
    hops = [hop(float(e), float(c)) for e, c in zip(err, chg)]
    tol = calibrate_change_tol(hops)
    admitted = [h for h in hops if h["state_change"] <= tol]
    assert all(h["X_linf"] <= 1e-3 for h in admitted)
    bigger = sorted(h["state_change"] for h in hops if h["state_change"] > tol)
    if bigger:
        assert any(h["X_linf"] > 1e-3 for h in hops if h["state_change"] <= bigger[0])
