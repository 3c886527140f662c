"""Pins for the oracle's point kernels (Section 2, Eq. 3): finite differences,
the kappa -> 0 limit, and high-precision (decimal) evaluation of the
cancellation-free difference factors."""
from decimal import Decimal, getcontext

import numpy as np
import pytest

import oracle as O

RNG = np.random.default_rng(11)


def _unit(v):
    v = np.asarray(v, float)
    return v / np.linalg.norm(v)


def _cases(n=12):
    out = []
    for _ in range(n):
        x = RNG.normal(size=3)
        y = x + _unit(RNG.normal(size=3)) * RNG.uniform(0.3, 6.0)
        out.append((x, _unit(RNG.normal(size=3)), y, _unit(RNG.normal(size=3)),
                    RNG.uniform(0.02, 1.5)))
    return out


@pytest.mark.parametrize("x,nx,y,ny,kappa", _cases())
def test_normal_derivatives_by_finite_differences(x, nx, y, ny, kappa):
    h = 1e-5
    k0 = O.kernels(x, nx, y, ny, kappa)

    def at(xx, yy):
        return O.kernels(xx, nx, yy, ny, kappa)

    # source-normal derivatives: d/dt K(x, y + t ny)
    kp, km = at(x, y + h * ny), at(x, y - h * ny)
    for k, dk in (("G", "dG_dny"), ("u", "du_dny")):
        fd = (kp[k] - km[k]) / (2 * h)
        assert fd == pytest.approx(k0[dk], rel=1e-6, abs=1e-12)
    # target-normal derivatives: d/dt K(x + t nx, y)
    kp, km = at(x + h * nx, y), at(x - h * nx, y)
    for k, dk in (("G", "dG_dnx"), ("u", "du_dnx")):
        fd = (kp[k] - km[k]) / (2 * h)
        assert fd == pytest.approx(k0[dk], rel=1e-6, abs=1e-12)
    # mixed second derivative: d/dt of the source-normal derivative at x + t nx
    for k, dk in (("dG_dny", "d2G"), ("du_dny", "d2u")):
        fd = (kp[k] - km[k]) / (2 * h)
        assert fd == pytest.approx(k0[dk], rel=1e-5, abs=1e-11)


@pytest.mark.parametrize("x,nx,y,ny,kappa", _cases(6))
def test_difference_forms_match_plain_differences_without_cancellation(x, nx, y, ny, kappa):
    kappa = 2.0 / np.linalg.norm(np.asarray(x) - np.asarray(y))  # kappa r = 2
    k = O.kernels(x, nx, y, ny, kappa)
    assert k["G_minus_u"] == pytest.approx(k["G"] - k["u"], rel=1e-13)
    assert k["d2G_minus_d2u"] == pytest.approx(k["d2G"] - k["d2u"], rel=1e-12, abs=1e-15)


def test_kappa_zero_gives_identical_kernels():
    for x, nx, y, ny, _ in _cases(5):
        k = O.kernels(x, nx, y, ny, 0.0)
        assert k["u"] == k["G"] and k["du_dny"] == k["dG_dny"]
        assert k["du_dnx"] == k["dG_dnx"]
        assert k["G_minus_u"] == 0.0 and k["d2G_minus_d2u"] == 0.0


def _a_b_decimal(s):
    getcontext().prec = 60
    s = Decimal(repr(s))
    e = (-s).exp()
    a = 1 - e * (1 + s)
    b = 3 - e * (3 + 3 * s + s * s)
    return float(a), float(b)


@pytest.mark.parametrize("s", [1e-6, 1e-4, 3e-3, 0.05, 0.0999, 0.1, 0.3, 2.0, 9.0])
def test_difference_factors_against_60_digit_decimal(s):
    # Along a geometry where R.nx = R.ny = 0 and nx.ny = 1 the second
    # difference kernel is a(s)/(4 pi r^3); with R.nx = R.ny = r (nx = ny =
    # R/r) it is (a(s) - b(s))/(4 pi r^3).
    r = 1.0
    kappa = s / r
    x, y = np.array([r, 0, 0.0]), np.zeros(3)
    a_ref, b_ref = _a_b_decimal(s)
    k1 = O.kernels(x, [0, 0, 1.0], y, [0, 0, 1.0], kappa)
    assert k1["d2G_minus_d2u"] * 4 * np.pi * r ** 3 == pytest.approx(a_ref, rel=2e-14)
    k2 = O.kernels(x, [1.0, 0, 0], y, [1.0, 0, 0], kappa)
    assert k2["d2G_minus_d2u"] * 4 * np.pi * r ** 3 == pytest.approx(a_ref - b_ref, rel=1e-13)
    getcontext().prec = 60
    gmu = float((1 - (-Decimal(repr(kappa)) * Decimal(repr(r))).exp()) / Decimal(repr(r)))
    assert k1["G_minus_u"] * 4 * np.pi == pytest.approx(gmu, rel=1e-14)
