"""Comoving kick and drift factors (the symplectic integrator of paper
Sec. 2.1 run in the comoving volumes of Sec. 3): K = int da / (a^2 H) and
D = int da / (a^3 H).  The oracle's quadrature and the library's host-side
factors are pinned to the closed forms of three backgrounds, checked against
each other on the paper's (omega_m, omega_lambda) = (0.295, 0.705), and the
oracle's comoving leapfrog is checked for time reversibility."""
import math

import numpy as np
import pytest

import oracle
import workloads
from paper_1407_2600_amd import hot


def _closed(a1, a2, bg, h0):
    """(K, D) in closed form: Einstein-de Sitter (H = h0 a^-3/2), de Sitter
    (H = h0) and the empty Milne background (H = h0 / a)."""
    if bg == "eds":
        return (2.0 * (math.sqrt(a2) - math.sqrt(a1)) / h0,
                2.0 * (1.0 / math.sqrt(a1) - 1.0 / math.sqrt(a2)) / h0)
    if bg == "ds":
        return (1.0 / a1 - 1.0 / a2) / h0, 0.5 * (1.0 / a1 ** 2 - 1.0 / a2 ** 2) / h0
    return math.log(a2 / a1) / h0, (1.0 / a1 - 1.0 / a2) / h0


BACKGROUNDS = {"eds": (1.0, 0.0), "ds": (0.0, 1.0), "milne": (0.0, 0.0)}
INTERVALS = [(0.01, 0.0105), (0.1, 0.3), (0.5, 1.0), (0.02, 1.0), (1.0, 0.4)]


@pytest.mark.parametrize("bg", sorted(BACKGROUNDS))
@pytest.mark.parametrize("a1,a2", INTERVALS)
def test_factors_closed_forms(bg, a1, a2):
    om, ol = BACKGROUNDS[bg]
    h0 = 1.7
    k, d = _closed(a1, a2, bg, h0)
    for name, f in (("oracle", oracle.comoving_factors), ("library", hot.comoving_factors)):
        kk, dd = f(a1, a2, om, ol, h0)
        assert abs(kk - k) <= 1e-13 * abs(k), (name, kk, k)
        assert abs(dd - d) <= 1e-13 * abs(d), (name, dd, d)


@pytest.mark.parametrize("a1,a2", INTERVALS)
def test_factors_library_matches_oracle_lcdm(a1, a2):
    om, ol, h0 = 0.295, 0.705, 0.688
    ko, do = oracle.comoving_factors(a1, a2, om, ol, h0)
    kl, dl = hot.comoving_factors(a1, a2, om, ol, h0)
    assert abs(kl - ko) <= 1e-12 * abs(ko) and abs(dl - do) <= 1e-12 * abs(do)
    # additive over intervals, zero on an empty one
    am = 0.5 * (a1 + a2)
    k1, d1 = hot.comoving_factors(a1, am, om, ol, h0)
    k2, d2 = hot.comoving_factors(am, a2, om, ol, h0)
    assert abs(k1 + k2 - kl) <= 1e-13 * abs(kl) and abs(d1 + d2 - dl) <= 1e-13 * abs(dl)
    assert hot.comoving_factors(a1, a1, om, ol, h0) == (0.0, 0.0)


@pytest.mark.parametrize("bad", [(0.0, 1.0, 0.3, 0.7, 1.0), (-0.1, 1.0, 0.3, 0.7, 1.0),
                                 (0.5, 1.0, 0.3, 0.7, 0.0), (0.5, 1.0, float("nan"), 0.7, 1.0),
                                 (0.5, float("inf"), 0.3, 0.7, 1.0),
                                 # a background that recollapses before a = 2:
                                 # H^2 < 0 on the interval
                                 (0.5, 2.0, 0.1, -2.0, 1.0)])
def test_factors_reject_bad_backgrounds(bad):
    with pytest.raises(hot.HotError) as e:
        hot.comoving_factors(*bad)
    assert e.value.status == hot.HOT_EINVAL


def test_oracle_comoving_leapfrog_is_reversible():
    """Stepping back with -da from the end state returns to the start (the
    kicks and the drift of a step undo each other exactly in exact arithmetic;
    here to rounding)."""
    pos, mass, prm = workloads.make("zeldovich128", n_side=6)
    prm = dict(prm, theta=0.5)
    rng = np.random.default_rng(4)
    vel = rng.normal(scale=0.02, size=pos.shape)
    h0 = math.sqrt(8.0 * math.pi / (3.0 * 0.295))  # G = 1, mean density 1
    x1, v1, a1, _ = oracle.kdk_comoving(pos, vel, mass, prm, 0.2, 0.05, 3, 0.295, 0.705, h0)
    x0, v0, _, _ = oracle.kdk_comoving(x1, v1, mass, prm, 0.35, -0.05, 3, 0.295, 0.705, h0,
                                       acc=a1)
    d = x0 - pos
    d -= np.round(d)
    assert np.max(np.abs(d)) < 1e-12
    assert np.max(np.abs(v0 - vel)) < 1e-10 * np.max(np.abs(vel))
