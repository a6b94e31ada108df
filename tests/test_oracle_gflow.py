"""Pins of the oracle's interaction flow (Sec. 2.2; App. A, Steps 1 and 2): the one-loop
vertex flow at fixed T in the propagator scale g, lines G_g = g Z G0 and S_g = Z^2 G0, so
the internal line pair carries g Z_a Z_b (Z_a + Z_b) chi (2 g chi without Z).

* N = 1: dv/dg = 2 g c v^2 with c = chi_ph(q=0) - chi_pp(q_pp) as grid sums at T, so
  1/v(g) = 1/U - g^2 c exactly.  Checks the RK4 order, the adaptive integrator, and the
  crossing g* of the stop rule for an attractive U (1/max|V| is exactly linear in g^2).
* scaling: without Z, g^2 V_g depends on g^2 U only.  For the discrete RK4 map too, since
  the right-hand side is 2 g times a quadratic form in V: the flow of 4U to g/2 is four
  times the flow of U to g, bit for bit.  A wrong power of g breaks this.
* small U: V(g = 1) - U against second-order perturbation theory at T,
  U^2 [chi_ph(k3 - k2) - chi_pp(k1 + k2)] (the right-hand side at the start of the flow is
  second-order perturbation theory up to a factor, Sec. 3.1), residual ~ U^3.  Fixes the
  factor 2 and the signs.
* stop rule: relative to the bare coupling, max|V| > v_rel |U| (Sec. 3.2), so that the
  crossover coupling U* = g*^2 U is the same for every bare U above it (without Z).
* Z: Z = 1 tables bitwise equal no feedback; constant Z = z gives
  V_z(g; U) = V_1(g; z^3 U) / z^3; a g- and patch-dependent table gives the O(U^2) term
  int_0^1 g Z_a Z_b (Z_a + Z_b) chi dg, by quadrature of oracle-independent bubble sums.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O


def _fermi(x, T):
    return 0.5 * (1.0 - np.tanh(x / (2 * T)))


def _chi(x, y, T):
    """Static bubble -(f(x) - f(y))/(x - y), -f'(x) on the diagonal (plain numpy)."""
    d = x - y
    same = np.abs(d) < 1e-12
    num = -(_fermi(x, T) - _fermi(y, T))
    fp = _fermi(x, T) * (1 - _fermi(x, T)) / T
    return np.where(same, fp, num / np.where(same, 1.0, d))


def _xi(L):
    k = -math.pi + 2 * math.pi * (np.arange(L) + 0.5) / L
    return -2 * (np.cos(k)[None, :] + np.cos(k)[:, None])      # [jy, jx]


def _partner(L, m, pp):
    jy, jx = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    if pp:
        return (m[0] - jx - 1) % L, (m[1] - jy - 1) % L
    return (jx + m[0]) % L, (jy + m[1]) % L


def loop_sum(L, m, T, pp):
    xi = _xi(L)
    px, py = _partner(L, m, pp)
    return np.mean(_chi(xi, -xi[py, px] if pp else xi[py, px], T))


def gcfg(T, U, **kw):
    kw.setdefault("v_rel", 1e300)
    return O.flowcfg(T0=T, U=U, gflow=True, **kw)


# --------------------------------------------------------------------------------------
# N = 1 closed form
# --------------------------------------------------------------------------------------
L1 = 32


def c_n1(T):
    # one patch centred on theta = 0: k_F = (pi, 0), so q_pp = 2 k_F = 0 on the grid
    return loop_sum(L1, (0, 0), T, False) - loop_sum(L1, (0, 0), T, True)


def test_n1_rk4_fourth_order_and_closed_form():
    # an attractive U that stays finite up to g = 1 with 1/v(1) = 1/(5U): a steep flow
    T = 0.1
    c = c_n1(T)
    assert c < 0
    U = -1.0 / (1.25 * abs(c))
    exact = 1.0 / (1.0 / U - c)
    errs = []
    for n in (20, 40, 80):
        V, res, _ = O.flow(O.model(1, L1), gcfg(T, U, n_steps=n), U)
        assert res["status"] == O.REACHED_TEND and res["g_final"] == 1.0
        assert math.isnan(res["g_c"]) and math.isnan(res["T_c"]) and res["T_final"] == T
        errs.append(abs(V[0, 0, 0] - exact))
    r1, r2 = math.log2(errs[0] / errs[1]), math.log2(errs[1] / errs[2])
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, (errs, r1, r2)
    V, res, tr = O.flow(O.model(1, L1), gcfg(T, U, integrator=1, rtol=1e-10), U)
    assert V[0, 0, 0] == pytest.approx(exact, rel=1e-8)
    for g, mv in tr:
        assert mv == pytest.approx(abs(1.0 / (1.0 / U - g * g * c_n1(T))), rel=1e-8)


@pytest.mark.parametrize("integrator,n", [(0, 200), (1, 0)])
def test_n1_attractive_crossing(integrator, n):
    T, U, vmax = 0.1, -4.0, 20.0
    c = c_n1(T)
    # |v| = v_max with v < 0: 1/U - g^2 c = -1/v_max
    g2 = (1.0 / U + 1.0 / vmax) / c
    assert 0.05 < g2 < 0.9, (c, g2)
    cfg = gcfg(T, U, integrator=integrator, n_steps=n, v_rel=vmax / abs(U), rtol=1e-10)
    V, res, tr = O.flow(O.model(1, L1), cfg, U)
    assert res["status"] == O.DIVERGED
    assert res["g_c"] == pytest.approx(math.sqrt(g2), rel=1e-7)
    assert res["U_star"] == pytest.approx(g2 * U, rel=1e-7)
    (g0, m0), (g1, m1) = tr[-2], tr[-1]
    assert m0 <= vmax < m1
    # the crossing of 1/max|V| = 1/v_max on the parabola in g^2 through the last three
    # accepted points, inside the last step (exactly linear for N = 1 up to the integrator's
    # own error, so the straight line through the last two agrees closely)
    coef = np.polyfit(tr[-3:, 0] ** 2, 1.0 / tr[-3:, 1], 2)
    roots = [r.real for r in np.roots(coef - np.array([0.0, 0.0, 1.0 / vmax]))
             if abs(r.imag) < 1e-12 and g0 ** 2 <= r.real <= g1 ** 2]
    assert len(roots) == 1
    assert res["g_c"] == pytest.approx(math.sqrt(roots[0]), abs=1e-10)
    assert res["g_c"] == pytest.approx(O.gc_interp(g0, m0, g1, m1, vmax), abs=1e-8)


def test_stop_at_start():
    _, res, _ = O.flow(O.model(1, L1), gcfg(0.2, 3.0, v_rel=0.5), 3.0)
    assert res["status"] == O.DIVERGED and res["g_c"] == 0.0 and res["U_star"] == 0.0


def test_relative_threshold_makes_ustar_independent_of_bare_u():
    """With max|V| > v_rel |U|, the flows of two bare couplings above U*(T) cross at the same
    g*^2 U; an absolute threshold would not."""
    N, L, T = 8, 16, 0.1
    us = []
    for U in (6.0, 9.0):
        _, r, _ = O.flow(O.model(N, L), gcfg(T, U, integrator=1, rtol=1e-10, v_rel=100.0), U)
        assert r["status"] == O.DIVERGED and 0.0 < r["g_c"] < 1.0
        us.append(r["U_star"])
    assert us[0] == pytest.approx(us[1], rel=1e-7)
    ab = []
    for U in (6.0, 9.0):
        _, r, _ = O.flow(O.model(N, L), gcfg(T, U, integrator=1, rtol=1e-10, v_rel=20.0 / U), U)
        ab.append(r["U_star"])
    assert abs(ab[0] / ab[1] - 1.0) > 1e-3


# --------------------------------------------------------------------------------------
# g^2 U scaling
# --------------------------------------------------------------------------------------
def test_g2u_scaling_bitwise_for_rk4():
    N, L, T, U = 8, 16, 0.2, 1.0
    VA, ra, _ = O.flow(O.model(N, L), gcfg(T, U, n_steps=50), U)
    VB, rb, _ = O.flow(O.model(N, L), gcfg(T, 4 * U, n_steps=50, g_end=0.5), 4 * U)
    assert np.abs(VA - U).max() > 0.05
    assert np.array_equal(VB / 4.0, VA)


def test_g2u_scaling_adaptive():
    N, L, T, U = 8, 16, 0.2, 1.0
    VA, _, _ = O.flow(O.model(N, L), gcfg(T, U, integrator=1, rtol=1e-11), U)
    k = 2.25
    VB, _, _ = O.flow(O.model(N, L), gcfg(T, k * U, integrator=1, rtol=1e-11,
                                           g_end=1.0 / math.sqrt(k)), k * U)
    assert np.abs(VB / k - VA).max() <= 1e-8 * np.abs(VA).max()


# --------------------------------------------------------------------------------------
# second order in U at g = 1
# --------------------------------------------------------------------------------------
def test_second_order_perturbation_theory_at_g1():
    N, L, T = 8, 16, 0.3
    _, _, anchor, _ = O.geometry(O.model(N, L))
    cache = {}

    def s(m, pp):
        if (m, pp) not in cache:
            cache[(m, pp)] = loop_sum(L, m, T, pp)
        return cache[(m, pp)]
    pred = np.zeros((N, N, N))
    for a in range(N):
        for b in range(N):
            qpp = tuple((anchor[a] + anchor[b]) % L)
            for c in range(N):
                pred[a, b, c] = s(tuple((anchor[c] - anchor[b]) % L), False) - s(qpp, True)
    res = []
    for U in (0.02, 0.04, 0.08):
        V, r, _ = O.flow(O.model(N, L), gcfg(T, U, n_steps=50), U)
        res.append(np.abs(V - U - U * U * pred).max())
        assert np.abs(V - U).max() > 10 * res[-1]
    s1, s2 = math.log2(res[1] / res[0]), math.log2(res[2] / res[1])
    assert abs(s1 - 3) < 0.1 and abs(s2 - 3) < 0.1, (res, s1, s2)


def test_rhs_at_g_is_2g_times_sopt_kernel_for_constant_v():
    """For V = U the direct bracket vanishes, so dV/dg = 2 g U^2 [chi_ph - chi_pp]."""
    N, L, T, U, g = 8, 16, 0.25, 1.3, 0.7
    _, _, anchor, _ = O.geometry(O.model(N, L))
    dV = O.rhs_g(O.model(N, L), T, g, np.full((N, N, N), U))
    for a, b, c in [(0, 0, 0), (1, 3, 5), (7, 2, 4), (4, 4, 0)]:
        qpp = tuple((anchor[a] + anchor[b]) % L)
        qcr = tuple((anchor[c] - anchor[b]) % L)
        want = 2 * g * U * U * (loop_sum(L, qcr, T, False) - loop_sum(L, qpp, T, True))
        assert dV[a, b, c] == pytest.approx(want, rel=1e-12, abs=1e-14)


# --------------------------------------------------------------------------------------
# Z insertion
# --------------------------------------------------------------------------------------
def test_z_one_is_bitwise_no_feedback():
    N, L, T, U = 8, 16, 0.2, 2.0
    gs = np.linspace(0.0, 1.0, 5)
    V0, _, _ = O.flow(O.model(N, L), gcfg(T, U, n_steps=30), U)
    V1, _, _ = O.flow(O.model(N, L), gcfg(T, U, n_steps=30, z_lnT=gs, z_tab=np.ones((5, N))), U)
    assert np.abs(V0 - U).max() > 0.1
    assert np.array_equal(V0, V1)


def test_constant_z_scaling():
    N, L, T, U, z = 8, 16, 0.15, 1.5, 0.8
    gs = np.linspace(0.0, 1.0, 3)
    Vz, _, _ = O.flow(O.model(N, L), gcfg(T, U, n_steps=40, z_lnT=gs,
                                          z_tab=np.full((3, N), z)), U)
    assert np.abs(Vz - U).max() > 0.1
    V1, _, _ = O.flow(O.model(N, L), gcfg(T, z ** 3 * U, n_steps=40), z ** 3 * U)
    assert np.abs(Vz - V1 / z ** 3).max() <= 1e-12 * np.abs(Vz).max()


def test_tabulated_z_second_order():
    """V(1) - U = U^2 int_0^1 sum_j g Z_j Z_j' (Z_j + Z_j') chi dg + O(U^3) with a table
    that varies with g and with the patch; Simpson quadrature in g.  U is small enough that
    the U^3 term stays below 1e-4 of the U^2 term also where the channels nearly cancel."""
    N, L, T, U = 8, 16, 0.25, 1e-6
    gs = np.linspace(0.0, 1.0, 6)
    tab = np.array([[1.0 - 0.3 * g * (1.0 + 0.25 * (a % 3)) for a in range(N)] for g in gs])
    V, _, _ = O.flow(O.model(N, L), gcfg(T, U, n_steps=60, z_lnT=gs, z_tab=tab), U)
    xi, patch, anchor, _ = O.geometry(O.model(N, L))
    P, X = patch.reshape(L, L), xi.reshape(L, L)

    def integrand(g, m, pp):
        Z = np.array([np.interp(g, gs, tab[:, a]) for a in range(N)])
        px, py = _partner(L, m, pp)
        za, zb = Z[P], Z[P[py, px]]
        y = -X[py, px] if pp else X[py, px]
        return np.mean(g * za * zb * (za + zb) * _chi(X, y, T))

    gg = np.linspace(0.0, 1.0, 201)
    wts = np.ones_like(gg)
    wts[1:-1:2], wts[2:-1:2] = 4, 2
    hs = (gg[1] - gg[0]) / 3
    for a, b, c in [(0, 0, 0), (1, 3, 5), (7, 2, 4), (4, 4, 0)]:
        qpp = tuple((anchor[a] + anchor[b]) % L)
        qcr = tuple((anchor[c] - anchor[b]) % L)
        cr = hs * sum(w * integrand(g, qcr, False) for g, w in zip(gg, wts))
        pp = hs * sum(w * integrand(g, qpp, True) for g, w in zip(gg, wts))
        assert (V[a, b, c] - U) / U ** 2 == pytest.approx(cr - pp, rel=1e-4, abs=1e-6)


def test_step_matches_flow():
    """One oracle step in g from 0 reproduces the first accepted step of the flow."""
    N, L, T, U = 4, 8, 0.2, 2.0
    cfg = gcfg(T, U, integrator=1, v_rel=10.0)
    V, res, tr = O.flow(O.model(N, L), cfg, U)
    g1 = tr[1][0]
    gn, hn, Vs, acc, err = O.step(O.model(N, L), cfg, 0.0, g1, np.full((N, N, N), U))
    assert acc and gn == pytest.approx(g1, abs=1e-15)
    assert np.abs(Vs).max() == pytest.approx(tr[1][1], rel=1e-14)
