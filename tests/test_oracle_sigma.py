"""Pins of the oracle's quasi-particle weight provider: the second-order self-energy on the
real axis, Kramers-Kronig, and Z from the slope outside the 2T window (Sec. 3.1; App. A,
Eq. definition_Z).

* Sum rule: -(1/pi) int Im Sigma dw = U^2 n (1 - n), n the mean occupation of the loop grid,
  exactly on the lattice for every external point (catches a dropped thermal term, a wrong
  normalisation, lost weight in the frequency binning).
* Im Sigma(w) = Im Sigma(-w) at half filling on the Fermi surface (particle-hole symmetry;
  k + Q is a point-group image of k there), so Re Sigma is odd.
* Kramers-Kronig against the Hilbert transform of a Gaussian, 2/sqrt(pi) times Dawson's
  function (scipy.special.dawsn).
* The literal brute force at N = 4, L = 4 and under identity patching at L = 4: the binned
  Im Sigma from a Python loop over the loop points, with cos per momentum.
* The vertex form: V = U gives the bare result bit for bit; Im Sigma scales as U^2; Z tends
  to 1 as U^2 (1 - Z proportional to U^2 at small U) and lies in (0, 1).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2005_00827_amd import inputs


def occupation(m, T):
    xi, _, _, _ = O.geometry(m)
    return float(np.mean(0.5 * (1.0 - np.tanh(0.5 * xi / T))))


@pytest.mark.parametrize("T,tp,mu", [(0.3, 0.0, 0.0), (0.1, 0.0, 0.0), (0.2, -0.3, -0.4)])
def test_sum_rule_on_grid_points(T, tp, mu):
    L = 6
    m = O.model(L * L, L, tp=tp, mu=mu, identity=True)
    U = 1.7
    w, im, _, _ = O.sigma2(m, T, U, n_w=512)
    n = occupation(m, T)
    total = -np.trapezoid(im, w, axis=1) / math.pi
    assert np.abs(total - U * U * n * (1 - n)).max() <= 1e-12


def test_sum_rule_angular_patches():
    """For any external point: the terms f2 (f3 - f1) cancel in pairs under
    (p1, p3) -> (-p3, -p1), which keeps p2 = k + p1 - p3 and swaps xi1 and xi3, so the rule
    is exact for the off-grid representative points too, also away from half filling."""
    for tp, mu in ((0.0, 0.0), (-0.3, -0.4)):
        m = O.model(8, 16, tp=tp, mu=mu)
        w, im, _, _ = O.sigma2(m, 0.2, 1.3, n_w=512)
        n = occupation(m, 0.2)
        total = -np.trapezoid(im, w, axis=1) / math.pi
        assert np.abs(total - 1.69 * n * (1 - n)).max() <= 1e-12


def test_particle_hole_symmetry_at_half_filling():
    m = O.model(16, 32)
    w, im, re, Z = O.sigma2(m, 0.15, 2.0, n_w=1024)
    assert np.abs(im - im[:, ::-1]).max() <= 1e-11 * np.abs(im).max()
    assert np.abs(re + re[:, ::-1]).max() <= 1e-10 * np.abs(re).max()
    assert (im <= 0.0).all()


def test_kramers_kronig_of_a_gaussian():
    """The piecewise-linear principal value converges to the exact transform at second
    order in the node spacing."""
    from scipy.special import dawsn
    errs = []
    for n_w in (1025, 2049):
        W0 = 12.0
        dw = 2 * W0 / (n_w - 1)
        w = -W0 + dw * np.arange(n_w)
        s = 0.3
        im = -np.exp(-(w / s) ** 2)
        re = O.kramers_kronig(-W0, dw, im)
        # Re(w) = -(1/pi) P int Im(x)/(w - x) dx = (2/sqrt(pi)) D(w/s) for Im = -exp(-(x/s)^2)
        errs.append(np.abs(re - 2.0 / math.sqrt(math.pi) * dawsn(w / s)).max())
    assert errs[1] <= 3e-4 and 3.5 < errs[0] / errs[1] < 4.5, errs


def _brute_im(N, L, T, U, n_w, identity=False):
    """Literal loops: Python cos per momentum and the linear split of each term's weight.
    The external point is the Fermi point on the patch's centre ray, or under identity
    patching the loop point of the patch itself."""
    xi_of = lambda kx, ky: -2.0 * (math.cos(kx) + math.cos(ky))
    kg = [-math.pi + 2 * math.pi * (j + 0.5) / L for j in range(L)]
    W0 = 3.0001 * 4.0
    dw = 2 * W0 / (n_w - 1)
    f = lambda x: 0.5 * (1.0 - math.tanh(0.5 * x / T))
    out = np.zeros((N, n_w))
    for a in range(N):
        if identity:
            kx, ky = kg[a % L], kg[a // L]
        else:
            th = math.pi / N + 2 * math.pi * a / N        # N % 8 == 4: centres off the axes
            r = math.pi / (abs(math.cos(th)) + abs(math.sin(th)))   # the half-filled diamond
            kx, ky = r * math.cos(th), r * math.sin(th)
        h = np.zeros(n_w)
        for y1 in kg:
            for x1 in kg:
                for y3 in kg:
                    for x3 in kg:
                        e1, e3 = xi_of(x1, y1), xi_of(x3, y3)
                        e2 = xi_of(kx + x1 - x3, ky + y1 - y3)
                        F = f(e1) * (1 - f(e2)) * (1 - f(e3)) + (1 - f(e1)) * f(e2) * f(e3)
                        x = (e2 + e3 - e1 + W0) / dw
                        i = math.floor(x)
                        h[i] += (1 - (x - i)) * U * U * F
                        h[i + 1] += (x - i) * U * U * F
        out[a] = -math.pi * h / (L ** 4 * dw)
    return out


def test_im_sigma_brute_force():
    N, L, T, U = 4, 4, 0.4, 1.3
    _, im, _, _ = O.sigma2(O.model(N, L), T, U, n_w=256)
    ref = _brute_im(N, L, T, U, 256)
    # the Fermi point is found by bisection in the oracle and in closed form here
    assert np.abs(im - ref).max() <= 1e-9 * np.abs(ref).max()


def test_im_sigma_brute_force_identity_patches():
    """Under identity patching every patch is a loop point, and so is its external point."""
    L, T, U = 4, 0.4, 1.3
    _, im, _, _ = O.sigma2(O.model(L * L, L, identity=True), T, U, n_w=256)
    ref = _brute_im(L * L, L, T, U, 256, identity=True)
    assert np.abs(im - ref).max() <= 1e-12 * np.abs(ref).max()


def test_unresolved_slope_gives_no_z():
    """Z needs at least 8 nodes in the window 2T <= |w| <= 4T: with 512 nodes (spacing 0.047)
    T = 0.05 has about 4 there, T = 0.2 about 17."""
    m = O.model(8, 16)
    w, _, re, Z = O.sigma2(m, 0.05, 2.0, n_w=512)
    assert ((np.abs(w) >= 0.1) & (np.abs(w) <= 0.2)).sum() < 8
    assert np.isnan(Z).all() and np.isfinite(re).all()
    w, _, _, Z = O.sigma2(m, 0.2, 2.0, n_w=512)
    assert ((np.abs(w) >= 0.4) & (np.abs(w) <= 0.8)).sum() >= 8 and np.isfinite(Z).all()


def test_vertex_form_and_scaling():
    m = O.model(16, 32)
    T = 0.2
    w, im1, re1, Z1 = O.sigma2(m, T, 1.0, n_w=512)
    _, imv, rev, Zv = O.sigma2(m, T, 1.0, V=inputs.constant_state(16, 1.0), n_w=512)
    assert np.array_equal(im1, imv) and np.array_equal(Z1, Zv)
    _, im2, _, Z2 = O.sigma2(m, T, 2.0, n_w=512)
    assert np.abs(im2 - 4.0 * im1).max() <= 1e-13 * np.abs(im2).max()
    _, _, _, Zh = O.sigma2(m, T, 0.5, n_w=512)
    assert ((Z2 > 0) & (Z2 < 1)).all()
    # 1 - Z = U^2 c + O(U^4)
    r = (1 - Zh) / 0.25 / ((1 - Z1) / 1.0)
    assert np.abs(r - 1.0).max() < 0.05, r
    # a vertex that is not constant changes the weights
    _, imn, _, _ = O.sigma2(m, T, 1.0, V=inputs.noisy_state(16, 1.0), n_w=512)
    assert np.abs(imn - im1).max() > 1e-3 * np.abs(im1).max()
