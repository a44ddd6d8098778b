"""Pins of the oracle's 1D kernels W_l, C_l, T_l against what the paper fixes
independently of the oracle's own code: the printed T_1..T_4 (Sec. 2), the
Fourier symbols s_l (Eq. s_l) and tau_l (Eq. tau_l), the momentum-conserving
limit a = 1/2 (Sec. 2, after Eq. tau_l), the support width l + 2a, and the
cancellation of Appendix A."""
import os

import numpy as np
import pytest

from tests.paper_printed import PRINTED_T

ORDERS = [1, 2, 3, 4]
A_VALUES = [0.02, 0.1, 0.25, 0.3, 0.45, 0.5]


def _breakpoints_T(l, a):
    pts = set()
    for j in range(l + 1):
        for s in (-a, a):
            pts.add(j - 0.5 * l + s)
    return np.array(sorted(pts))


def _ft(f, pts, k, nq=24):
    """Integral of f(y) exp(-i k y) dy over the support, Gauss-Legendre per
    polynomial piece (exact for the piecewise polynomials up to rounding)."""
    xg, wg = np.polynomial.legendre.leggauss(nq)
    tot = 0.0 + 0.0j
    for lo, hi in zip(pts[:-1], pts[1:]):
        y = 0.5 * (hi - lo) * xg + 0.5 * (hi + lo)
        tot += np.sum(wg * 0.5 * (hi - lo) * f(y) * np.exp(-1j * k * y))
    return tot


def _sinc(x):
    return np.sinc(x / np.pi)


@pytest.mark.parametrize("l", ORDERS)
@pytest.mark.parametrize("a", [0.02, 0.1, 0.25, 0.3, 0.45, 0.5])
def test_T_matches_printed_polynomials(orc, l, a):
    y = np.linspace(-(l / 2 + a) - 0.3, l / 2 + a + 0.3, 2001)
    ref = PRINTED_T[l](y, a)
    got = orc.T(l, a, y)
    assert np.max(np.abs(got - ref)) <= 1e-12


def test_printed_fixture(orc):
    """Values of the printed T_l stored in tests/golden (written by
    tests/golden/make_printed_T.py from the printed equations)."""
    path = os.path.join(os.path.dirname(__file__), "golden", "printed_T.txt")
    data = np.loadtxt(path)
    for l, a, y, t in data:
        assert abs(orc.T(int(l), a, np.array([y]))[0] - t) <= 1e-12


@pytest.mark.parametrize("l", ORDERS)
def test_T_equals_W_at_half_courant(orc, l):
    """For c dt = dx/2, tau_l = s_l and WT reduces to MC."""
    y = np.linspace(-3, 3, 4001)
    assert np.max(np.abs(orc.T(l, 0.5, y) - orc.W(l, y))) <= 1e-14


@pytest.mark.parametrize("l", ORDERS)
def test_T_small_dt_limit(orc, l):
    """tau_l -> sinc^l as dt -> 0, i.e. T_l -> W_{l-1}."""
    y = np.linspace(-3, 3, 4001)
    a = 1e-5
    assert np.max(np.abs(orc.T(l, a, y) - orc.W(l - 1, y))) <= 2e-5


@pytest.mark.parametrize("l", ORDERS)
@pytest.mark.parametrize("a", [0.1, 0.3, 0.5, 0.7, 0.9])
def test_T_support_width(orc, l, a):
    """T_l vanishes outside |y| < l/2 + a (width l dx + 2 c dt)."""
    h = l / 2 + a
    y_out = np.concatenate([np.linspace(h + 1e-12, h + 2, 50), -np.linspace(h + 1e-12, h + 2, 50)])
    assert np.all(orc.T(l, a, y_out) == 0.0)
    y_in = np.linspace(-h + 1e-3, h - 1e-3, 200)
    assert np.all(orc.T(l, a, y_in) > 0.0)


@pytest.mark.parametrize("l", ORDERS)
def test_W_fourier_transform_is_s_l(orc, l):
    pts = np.arange(-(l + 1) / 2, (l + 1) / 2 + 0.5, 1.0)
    for k in np.linspace(0.05, 12.0, 37):
        ft = _ft(lambda y: orc.W(l, y), pts, k)
        assert abs(ft - _sinc(k / 2) ** (l + 1)) <= 1e-13


@pytest.mark.parametrize("l", ORDERS)
@pytest.mark.parametrize("a", [0.05, 0.2, 0.45, 0.5, 0.7])
def test_T_fourier_transform_is_tau_l(orc, l, a):
    pts = _breakpoints_T(l, a)
    for k in np.linspace(0.05, 12.0, 37):
        ft = _ft(lambda y: orc.T(l, a, y), pts, k)
        tau = _sinc(k / 2) ** l * _sinc(k * a)
        assert abs(ft - tau) <= 1e-12


@pytest.mark.parametrize("l", ORDERS)
@pytest.mark.parametrize("a", [0.1, 0.35, 0.5, 0.7])
def test_partition_of_unity_and_linear_reproduction(orc, l, a):
    x = np.random.default_rng(5).random(64) * 7 - 3
    for xv in x:
        n = np.arange(np.floor(xv) - 5, np.floor(xv) + 6)
        w = orc.W(l, xv - n)
        t = orc.T(l, a, xv - n)
        assert abs(w.sum() - 1) <= 1e-14
        assert abs(t.sum() - 1) <= 1e-14
        assert abs((n * w).sum() - xv) <= 1e-13
        if l >= 2 or a == 0.5:
            assert abs((n * t).sum() - xv) <= 1e-13
    if l == 1 and a != 0.5:
        # the first moment is not reproduced by T_1 away from the MC limit
        xv = 0.3
        n = np.arange(-5, 6)
        assert abs((n * orc.T(1, a, xv - n)).sum() - xv) > 1e-3


@pytest.mark.parametrize("l", [2, 3, 4])
def test_C_is_integral_of_lower_spline(orc, l):
    xg, wg = np.polynomial.legendre.leggauss(20)
    for z in np.linspace(-l / 2 - 0.5, l / 2 + 0.5, 23):
        knots = np.arange(-l / 2, l / 2 + 0.5, 1.0)
        pts = np.concatenate([[-l / 2], knots[(knots > -l / 2) & (knots < z)], [z]]) if z > -l / 2 else None
        ref = 0.0
        if pts is not None:
            for lo, hi in zip(pts[:-1], pts[1:]):
                y = 0.5 * (hi - lo) * xg + 0.5 * (hi + lo)
                ref += np.sum(wg * 0.5 * (hi - lo) * orc.W(l - 1, y))
        assert abs(orc.C(l, np.array([z]))[0] - ref) <= 1e-14


def _symbols(orc, l, k1p, a, pts_T, pts_W):
    """s_{l,1} and tau_{l,1} at k'_1 from the oracle's real-space kernels."""
    s = _ft(lambda y: orc.W(l, y), pts_W, k1p).real
    tau = _ft(lambda y: orc.T(l, a, y), pts_T, k1p).real
    return s, tau


@pytest.mark.parametrize("l", [2, 4])
def test_appendix_A_cancellation(orc, l):
    """S_B3 xi_0 - S_E2 [k]_B1 c = 0 on the beam resonance omega' = c k'_1 for
    WT (any dt, any alias nu_1), and not for MC unless c dt = dx/2.  The
    common factors s_{l,2} tau_{l,3} eta_2 are dropped; tau_{l,1}, s_{l,1} come
    from the oracle's T_l and W_l by numerical Fourier transform.  dx = c = 1."""
    rng = np.random.default_rng(7)
    pts_W = np.arange(-(l + 1) / 2, (l + 1) / 2 + 0.5, 1.0)
    for _ in range(12):
        a = rng.uniform(0.05, 0.5)
        dt = a
        k1 = rng.uniform(0.05, np.pi)
        nu = int(rng.integers(-2, 3))
        k1p = k1 + 2 * np.pi * nu
        s1, tau1 = _symbols(orc, l, k1p, a, _breakpoints_T(l, a), pts_W)
        eta1 = (-1.0) ** nu
        xi0 = np.sin(k1p * dt / 2) / (dt / 2)
        kB1 = np.sin(k1 / 2) / 0.5
        cosw = np.cos(k1p * dt / 2)
        wt = cosw * s1 * eta1 * xi0 - tau1 * kB1
        mc = cosw * s1 * eta1 * xi0 - s1 * kB1
        assert abs(wt) <= 1e-11
        if abs(np.sin(k1p * a) / a - 2 * np.sin(k1p / 2)) > 1e-3:
            assert abs(mc) > 1e-9
