"""Pins of the oracle's bubble weights against definitions it does not use.

The oracle evaluates chi and T d/dT chi through a cancellation-free identity for the divided
difference of phi(u) = u sech^2 u.  Here they are checked against (i) the Fermi-function
definition chi = -(f(x) - f(y))/(x - y) evaluated in 600-digit decimal arithmetic (enough to resolve differences of tanh near 1 at T = 0.01), (ii) the
closed forms chi(x,x) = -f'(x) and chi(x,-x) = tanh(x/2T)/(2x), (iii) a centred finite
difference in T, (iv) the particle-hole symmetry of the weights, and (v) the q = 0
particle-hole loop sum against (1/L^2) sum_j of the closed form T d/dT(-f'(xi_j)) and, for
large L, against the density-of-states integral with the square-lattice DOS.
"""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest
from scipy import integrate, special

from oracle import oracle as O

getcontext().prec = 600


def _dtanh(u):
    e2 = (2 * u).exp()
    return (e2 - 1) / (e2 + 1)


def chi_decimal(x, y, T):
    """(tanh(x/2T) - tanh(y/2T)) / (2 (x - y)), i.e. -(f(x)-f(y))/(x-y), 600 digits."""
    x, y, T = Decimal(x), Decimal(y), Decimal(T)
    if x == y:
        s = 1 / ((x / (2 * T)).exp() + (-x / (2 * T)).exp())
        return float(4 * s * s / (4 * T))
    return float((_dtanh(x / (2 * T)) - _dtanh(y / (2 * T))) / (2 * (x - y)))


def phi_dd_decimal(a, b):
    """(a sech^2 a - b sech^2 b)/(a - b) with 600 digits (a != b)."""
    a, b = Decimal(a), Decimal(b)

    def phi(u):
        s = 2 / (u.exp() + (-u).exp())
        return u * s * s
    return float((phi(a) - phi(b)) / (a - b))


CASES = [(0.3, 0.7), (0.3, -0.29), (1.0, 1.0 + 1e-9), (2.5, 2.5 - 1e-4), (-3.0, 3.0 + 1e-6),
         (12.0, 12.001), (40.0, -39.5), (0.0, 1e-7), (5.0, -0.1), (80.0, 81.0), (0.77, 0.78)]


@pytest.mark.parametrize("a,b", CASES)
def test_phi_divided_difference_vs_decimal(a, b):
    ref = phi_dd_decimal(a, b)
    got = O.phi_dd(a, b)
    scale = max(abs(ref), 1e-300)
    # relative accuracy where the value is representable, absolute 1e-16 otherwise
    assert abs(got - ref) <= 1e-13 * scale + 1e-17, (a, b, got, ref)
    assert abs(O.phi_dd(b, a) - ref) <= 1e-13 * scale + 1e-17


@pytest.mark.parametrize("x,y,T", [(0.3, 0.7, 0.1), (-1.2, 0.4, 0.05), (0.5, 0.5, 0.2),
                                   (3.0, 3.0 + 1e-10, 0.01), (2.0, -1.9999, 0.01),
                                   (-3.9, 3.9, 0.01), (0.01, -0.02, 1.0)])
def test_chi_vs_decimal(x, y, T):
    ref = chi_decimal(x, y, T)
    assert abs(O.chi_ph(x, y, T) - ref) <= 1e-13 * abs(ref) + 1e-300
    ref_pp = chi_decimal(x, -y, T)
    assert abs(O.chi_pp(x, y, T) - ref_pp) <= 1e-13 * abs(ref_pp) + 1e-300


@pytest.mark.parametrize("x,T", [(0.0, 0.1), (0.3, 0.1), (-2.0, 0.5), (1.5, 0.01)])
def test_closed_forms(x, T):
    fprime = -1.0 / (4 * T * math.cosh(x / (2 * T)) ** 2)
    assert O.chi_ph(x, x, T) == pytest.approx(-fprime, rel=1e-14)
    if x != 0.0:
        assert O.chi_pp(x, x, T) == pytest.approx(math.tanh(x / (2 * T)) / (2 * x), rel=1e-14)
    # coincident limit of T d/dT chi:  (1/4T) sech^2 a (2 a tanh a - 1), a = x/2T
    a = x / (2 * T)
    cl = (2 * a * math.tanh(a) - 1) / (4 * T * math.cosh(a) ** 2)
    assert O.chidot_ph(x, x, T) == pytest.approx(cl, rel=1e-13, abs=1e-300)


@pytest.mark.parametrize("x,y,T", [(0.3, -0.7, 0.1), (1.0, 1.3, 0.05), (-0.2, -0.2, 0.3),
                                   (2.0, -2.0001, 0.2), (0.05, 3.0, 1.0)])
def test_chidot_is_T_derivative(x, y, T):
    """T d/dT chi against a centred difference in ln T of the decimal chi."""
    d = 1e-5
    for pp in (False, True):
        yy = -y if pp else y
        fd = (chi_decimal(x, yy, T * math.exp(d)) - chi_decimal(x, yy, T * math.exp(-d))) / (2 * d)
        got = O.chidot_pp(x, y, T) if pp else O.chidot_ph(x, y, T)
        assert got == pytest.approx(fd, rel=1e-8, abs=1e-12)


def test_weight_symmetries():
    rng = np.random.default_rng(3)
    for _ in range(200):
        x, y = rng.uniform(-4, 4, 2)
        T = math.exp(rng.uniform(math.log(0.01), 0.0))
        for f in (O.chidot_ph, O.chidot_pp, O.chi_ph, O.chi_pp):
            assert f(-x, -y, T) == f(x, y, T)          # xi -> -xi (half filling)
            # symmetric to rounding on the weight scale 1/(4T)
            assert f(y, x, T) == pytest.approx(f(x, y, T), rel=1e-13, abs=1e-15 / T)
        assert O.chi_ph(x, y, T) >= 0.0 and O.chi_pp(x, y, T) >= 0.0 or abs(x + y) < 1e-12


def _grid_xi(L):
    k = -math.pi + 2 * math.pi * (np.arange(L) + 0.5) / L
    return (-2 * (np.cos(k)[None, :] + np.cos(k)[:, None])).ravel()


@pytest.mark.parametrize("L,T", [(32, 0.5), (64, 0.1), (16, 0.02)])
def test_q0_particle_hole_loop_sum(L, T):
    """N = 1 and the crossed channel only: dV/dlnT = V^2 (1/L^2) sum_j T d/dT(-f'(xi_j))."""
    m = O.model(1, L, channels=O.CH_CR)
    got = O.rhs(m, T, np.ones((1, 1, 1)))[0, 0, 0]
    a = _grid_xi(L) / (2 * T)
    ref = np.mean((2 * a * np.tanh(a) - 1) / (4 * T * np.cosh(a) ** 2))
    assert got == pytest.approx(ref, rel=1e-12)


def test_q0_loop_sum_converges_to_dos_integral():
    """(1/L^2) sum_j w(xi_j) -> int rho(e) w(e) de with rho(e) = K(1 - e^2/16) / (2 pi^2)."""
    T = 0.5
    w = lambda e: (2 * (e / 2 / T) * math.tanh(e / 2 / T) - 1) / (4 * T * math.cosh(e / 2 / T) ** 2)
    rho = lambda e: special.ellipk(1 - e * e / 16) / (2 * math.pi ** 2)
    ref = 2 * integrate.quad(lambda e: rho(e) * w(e), 0, 4, limit=400, )[0]
    # the half-shifted grid is a periodic trapezoid rule for a smooth integrand: the grid
    # sum reaches the integral to quadrature accuracy already at moderate L
    for L in (64, 128, 256):
        m = O.model(1, L, channels=O.CH_CR)
        got = O.rhs(m, T, np.ones((1, 1, 1)))[0, 0, 0]
        assert abs(got - ref) < 1e-10 * abs(ref), (L, got, ref)
