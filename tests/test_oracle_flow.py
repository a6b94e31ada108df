"""Pins of the oracle's flows (integrators, stop rule, Z insertion) against closed forms.

* N = 1: the flow reduces to dv/ds = v^2 c'(s) with c = chi_ph(q=0) - chi_pp(q_pp) as grid
  sums, so 1/v(T) = 1/U - [c(T) - c(T0)] exactly.  Checks the RK4 error order (h^4), the
  adaptive integrator's accuracy, and T_c from the stop rule against the closed-form root
  for an attractive U.
* small U: V(T) - U against second-order perturbation theory
  U^2 [Delta chi_ph(k3 - k2) - Delta chi_pp(k1 + k2)] (the flow's right-hand side at the
  start is second-order perturbation theory, Sec. 3.1), with a residual that scales as U^3.
* Z insertion: Z = 1 tables are bit-identical to no feedback; a constant Z = z gives
  V_z(T; U) = V_1(T; z^2 U) / z^2; with a tabulated Z(T) the O(U^2) term is the
  Z-weighted integral of the bubble derivative.
* Dormand-Prince 5(4): the tableau satisfies every order condition up to order 5 (order 4
  for the embedded weights).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2005_00827_amd import inputs


def _fermi(x, T):
    return 0.5 * (1.0 - np.tanh(x / (2 * T)))


def _chi(x, y, T):
    d = x - y
    same = np.abs(d) < 1e-12
    num = -(_fermi(x, T) - _fermi(y, T))
    fp = _fermi(x, T) * (1 - _fermi(x, T)) / T
    return np.where(same, fp, num / np.where(same, 1.0, d))


def _xi(L):
    k = -math.pi + 2 * math.pi * (np.arange(L) + 0.5) / L
    return -2 * (np.cos(k)[None, :] + np.cos(k)[:, None])      # [jy, jx]


def loop_sum(L, m, T, pp):
    xi = _xi(L)
    jy, jx = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    if pp:
        px, py = (m[0] - jx - 1) % L, (m[1] - jy - 1) % L
        return np.mean(_chi(xi, -xi[py, px], T))
    px, py = (jx + m[0]) % L, (jy + m[1]) % L
    return np.mean(_chi(xi, xi[py, px], T))


# --------------------------------------------------------------------------------------
# N = 1 closed form
# --------------------------------------------------------------------------------------
L1 = 32


def c_n1(T):
    # one patch centred on theta = 0: k_F = (pi, 0), so q_pp = 2 k_F = 0 on the grid
    return loop_sum(L1, (0, 0), T, False) - loop_sum(L1, (0, 0), T, True)


def v_exact(U, T, T0=1.0):
    return 1.0 / (1.0 / U - (c_n1(T) - c_n1(T0)))


def test_n1_rk4_converges_at_fourth_order():
    U = 1.5
    errs = []
    for n in (25, 50, 100):
        cfg = O.flowcfg(T0=1.0, T_end=0.05, n_steps=n, v_max=1e300, U=U)
        V, res, tr = O.flow(O.model(1, L1), cfg, U)
        assert res["status"] == O.REACHED_TEND
        errs.append(abs(V[0, 0, 0] - v_exact(U, 0.05)))
    r1, r2 = math.log2(errs[0] / errs[1]), math.log2(errs[1] / errs[2])
    assert 3.7 < r1 < 4.3 and 3.7 < r2 < 4.3, (errs, r1, r2)


def test_n1_dopri_accuracy_and_repulsive_no_divergence():
    U = 2.0
    cfg = O.flowcfg(T0=1.0, T_end=0.01, integrator=1, rtol=1e-9, U=U)
    V, res, tr = O.flow(O.model(1, L1), cfg, U)
    # repulsive U at N = 1: 1/v grows (chi_pp(0) outgrows chi_ph(0)), no instability
    assert res["status"] == O.REACHED_TEND and math.isnan(res["T_c"])
    assert V[0, 0, 0] == pytest.approx(v_exact(U, 0.01), rel=1e-7)
    for s, mv in tr[:: max(1, len(tr) // 10)]:
        assert mv == pytest.approx(abs(v_exact(U, math.exp(s))), rel=1e-7)


def _tc_exact(U, v_max, T0=1.0):
    # |v| = v_max with v keeping the sign of U: 1/U - [c(T) - c(T0)] = sign(U)/v_max
    g = lambda s: 1.0 / U - (c_n1(math.exp(s)) - c_n1(T0)) - math.copysign(1.0, U) / v_max
    lo, hi = math.log(0.01), math.log(T0)
    assert g(lo) * g(hi) < 0
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        if g(mid) * g(hi) < 0:
            lo = mid
        else:
            hi = mid
    return math.exp(0.5 * (lo + hi))


@pytest.mark.parametrize("integrator,n", [(0, 400), (1, 0)])
def test_n1_attractive_tc(integrator, n):
    U, vmax = -2.0, 20.0
    tc = _tc_exact(U, vmax)
    cfg = O.flowcfg(T0=1.0, T_end=0.01, integrator=integrator, n_steps=n, v_max=vmax, U=U)
    V, res, tr = O.flow(O.model(1, L1), cfg, U)
    assert res["status"] == O.DIVERGED
    assert res["T_c"] == pytest.approx(tc, rel=1e-3)
    # the stop rule: the crossing of 1/max|V| = 1/v_max on the parabola in ln T through the
    # last three accepted points, inside the last step
    (s0, m0), (s1, m1) = tr[-2], tr[-1]
    assert m0 <= vmax < m1
    coef = np.polyfit(tr[-3:, 0], 1.0 / tr[-3:, 1], 2)
    coef[-1] -= 1.0 / vmax
    roots = [r.real for r in np.roots(coef) if abs(r.imag) < 1e-12 and s1 <= r.real <= s0]
    assert len(roots) == 1
    assert math.log(res["T_c"]) == pytest.approx(roots[0], abs=1e-10)


@pytest.mark.parametrize("rtol", [1e-4, 1e-6])
def test_n1_crossing_through_three_points_tracks_the_closed_form(rtol):
    """With long steps near the instability (loose rtol), the crossing on the parabola
    through the last three points stays within 1e-4 of the closed-form T_c; the straight line
    through the last two is what the curvature of 1/max|V| over the step moves."""
    U, vmax = -2.0, 20.0
    tc = _tc_exact(U, vmax)
    cfg = O.flowcfg(T0=1.0, T_end=0.01, integrator=1, rtol=rtol, v_max=vmax, U=U)
    _, res, tr = O.flow(O.model(1, L1), cfg, U)
    assert res["status"] == O.DIVERGED
    assert abs(res["T_c"] / tc - 1.0) < 1e-4, (res["T_c"], tc)
    lin = math.exp(O.tc_interp(tr[-2, 0], tr[-2, 1], tr[-1, 0], tr[-1, 1], vmax))
    assert abs(res["T_c"] / tc - 1.0) <= abs(lin / tc - 1.0)


def test_stop_at_start_and_stepfail():
    cfg = O.flowcfg(T0=1.0, T_end=0.1, v_max=1.0, U=3.0)
    _, res, _ = O.flow(O.model(1, L1), cfg, 3.0)
    assert res["status"] == O.DIVERGED and res["T_c"] == pytest.approx(1.0)
    cfg = O.flowcfg(T0=1.0, T_end=0.1, integrator=1, h_min=10.0, U=1.0)
    _, res, _ = O.flow(O.model(1, L1), cfg, 1.0)
    assert res["status"] == O.STEPFAIL


# --------------------------------------------------------------------------------------
# second order in U
# --------------------------------------------------------------------------------------
def _second_order(N, L, T, T0, Zfun=None):
    _, _, anchor, _ = O.geometry(O.model(N, L))
    pred = np.zeros((N, N, N))
    cache = {}

    def d(m, pp):
        key = (m, pp)
        if key not in cache:
            cache[key] = loop_sum(L, m, T, pp) - loop_sum(L, m, T0, pp)
        return cache[key]
    for a in range(N):
        for b in range(N):
            qpp = tuple((anchor[a] + anchor[b]) % L)
            for c in range(N):
                qcr = tuple((anchor[c] - anchor[b]) % L)
                pred[a, b, c] = d(qcr, False) - d(qpp, True)
    return pred


def test_second_order_perturbation_theory():
    N, L, T0, T1 = 8, 16, 1.0, 0.1
    pred = _second_order(N, L, T1, T0)
    res = []
    for U in (0.02, 0.04, 0.08):
        cfg = O.flowcfg(T0=T0, T_end=T1, n_steps=100, v_max=1e300, U=U)
        V, r, _ = O.flow(O.model(N, L), cfg, U)
        res.append(np.abs(V - U - U * U * pred).max())
        # the second-order term itself is resolved
        assert np.abs(V - U).max() > 10 * res[-1]
    s1, s2 = math.log2(res[1] / res[0]), math.log2(res[2] / res[1])
    assert abs(s1 - 3) < 0.1 and abs(s2 - 3) < 0.1, (res, s1, s2)


# --------------------------------------------------------------------------------------
# Z insertion
# --------------------------------------------------------------------------------------
def test_z_one_is_bitwise_no_feedback():
    N, L, U = 8, 16, 2.0
    lnT = np.linspace(math.log(0.2), 0.0, 5)
    cfg0 = O.flowcfg(T0=1.0, T_end=0.2, n_steps=30, v_max=1e300, U=U)
    cfg1 = O.flowcfg(T0=1.0, T_end=0.2, n_steps=30, v_max=1e300, U=U, z_lnT=lnT,
                     z_tab=np.ones((5, N)))
    V0, _, _ = O.flow(O.model(N, L), cfg0, U)
    V1, _, _ = O.flow(O.model(N, L), cfg1, U)
    assert np.all(np.isfinite(V0)) and np.abs(V0 - U).max() > 0.1
    assert np.array_equal(V0, V1)


def test_constant_z_scaling():
    N, L, U, z = 8, 16, 1.5, 0.8
    lnT = np.linspace(math.log(0.05), 0.0, 3)
    cfgz = O.flowcfg(T0=1.0, T_end=0.05, n_steps=40, v_max=1e300, U=U, z_lnT=lnT,
                     z_tab=np.full((3, N), z))
    Vz, _, _ = O.flow(O.model(N, L), cfgz, U)
    assert np.all(np.isfinite(Vz)) and np.abs(Vz - U).max() > 0.1
    cfg1 = O.flowcfg(T0=1.0, T_end=0.05, n_steps=40, v_max=1e300, U=z * z * U)
    V1, _, _ = O.flow(O.model(N, L), cfg1, z * z * U)
    assert np.abs(Vz - V1 / (z * z)).max() <= 1e-12 * np.abs(Vz).max()


def test_tabulated_z_second_order():
    """dV/ds = U^2 sum_j Z_a' Z_b' chidot + O(U^3): with a patch- and T-dependent table the
    O(U^2) term is int ds of the Z-weighted bubble derivative, here by Simpson quadrature
    of the oracle-independent bubble sums."""
    N, L, T0, T1, U = 8, 16, 1.0, 0.2, 1e-4
    lnT, tab = inputs.synthetic_z_table(N, 3.0, T0, T1, n_nodes=9)
    cfg = O.flowcfg(T0=T0, T_end=T1, n_steps=60, v_max=1e300, U=U, z_lnT=lnT, z_tab=tab)
    V, _, _ = O.flow(O.model(N, L), cfg, U)
    xi, patch, anchor, _ = O.geometry(O.model(N, L))
    P = patch.reshape(L, L)
    X = xi.reshape(L, L)
    jy, jx = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")

    def z_at(s):
        return np.array([np.interp(s, lnT, tab[:, a]) for a in range(N)])

    def integrand(s, m, pp):
        T, h = math.exp(s), 1e-5
        Z = z_at(s)
        if pp:
            px, py = (m[0] - jx - 1) % L, (m[1] - jy - 1) % L
            y = -X[py, px]
        else:
            px, py = (jx + m[0]) % L, (jy + m[1]) % L
            y = X[py, px]
        w = Z[P] * Z[P[py, px]]
        dchi = (_chi(X, y, T * math.exp(h)) - _chi(X, y, T * math.exp(-h))) / (2 * h)
        return np.mean(w * dchi)

    ss = np.linspace(math.log(T0), math.log(T1), 241)
    wts = np.ones_like(ss)
    wts[1:-1:2], wts[2:-1:2] = 4, 2
    hs = (ss[1] - ss[0]) / 3
    for a, b, c in [(0, 0, 0), (1, 3, 5), (7, 2, 4), (4, 4, 0)]:
        qpp = tuple((anchor[a] + anchor[b]) % L)
        qcr = tuple((anchor[c] - anchor[b]) % L)
        cr = hs * sum(w * integrand(s, qcr, False) for s, w in zip(ss, wts))
        pp = hs * sum(w * integrand(s, qpp, True) for s, w in zip(ss, wts))
        assert (V[a, b, c] - U) / U ** 2 == pytest.approx(cr - pp, rel=1e-3, abs=2e-5)


# --------------------------------------------------------------------------------------
# Dormand-Prince tableau
# --------------------------------------------------------------------------------------
def test_dopri_order_conditions():
    c, A, e = O.dopri_tableau()
    Af = np.zeros((7, 7))
    Af[:, :6] = A
    b = Af[6].copy()
    bh = b - e
    assert np.allclose(Af.sum(1), c, atol=1e-15)

    def conds(w, order):
        out = [(w.sum(), 1.0), (w @ c, 1 / 2), (w @ c ** 2, 1 / 3), (w @ Af @ c, 1 / 6)]
        if order >= 4:
            out += [(w @ c ** 3, 1 / 4), (w @ (c * (Af @ c)), 1 / 8), (w @ Af @ c ** 2, 1 / 12),
                    (w @ Af @ Af @ c, 1 / 24)]
        if order >= 5:
            Ac = Af @ c
            out += [(w @ c ** 4, 1 / 5), (w @ (c ** 2 * Ac), 1 / 10), (w @ Ac ** 2, 1 / 20),
                    (w @ (c * (Af @ c ** 2)), 1 / 15), (w @ Af @ c ** 3, 1 / 20),
                    (w @ (c * (Af @ Ac)), 1 / 30), (w @ Af @ (c * Ac), 1 / 40),
                    (w @ Af @ Af @ c ** 2, 1 / 60), (w @ Af @ Af @ Af @ c, 1 / 120)]
        return out
    for got, want in conds(b, 5):
        assert got == pytest.approx(want, abs=1e-14)
    for got, want in conds(bh, 4):
        assert got == pytest.approx(want, abs=1e-14)
    # the embedded pair differs at fifth order
    assert abs(bh @ c ** 4 - 1 / 5) > 1e-6


def test_step_matches_flow():
    """orc_step (no carry-over) reproduces the flow's first accepted steps."""
    N, L, U = 8, 16, 2.0
    m = O.model(N, L)
    cfg = O.flowcfg(T0=1.0, T_end=0.05, integrator=1, v_max=1e300, U=U)
    _, _, tr = O.flow(m, cfg, U)
    lnT, h, V = 0.0, math.log(0.05) / 200, np.full((N, N, N), U)
    k = 1
    while k < 4:
        lnT2, h2, V2, acc, err = O.step(m, cfg, lnT, h, V)
        if acc:
            assert lnT2 == pytest.approx(tr[k][0], abs=1e-15)
            assert np.abs(V2).max() == pytest.approx(tr[k][1], rel=1e-15)
            lnT, V, k = lnT2, V2, k + 1
        h = h2


# --------------------------------------------------------------------------------------
# flows on one shared step schedule
# --------------------------------------------------------------------------------------
def test_sync_batch_of_one_is_the_plain_flow():
    """One flow on a 'shared' schedule takes exactly the plain Dormand-Prince flow's steps."""
    m = O.model(16, 32)
    V1, r1, _ = O.flow(m, O.flowcfg(U=2.5, integrator=1), 2.5)
    Vs, rs = O.flow_sync(m, O.flowcfg(integrator=1, atol=0.0), [2.5])
    assert np.array_equal(V1, Vs[0])
    for k in ("status", "T_c", "T_final", "n_accepted", "n_rejected", "n_rhs", "max_abs_V"):
        assert rs[0][k] == r1[k], k


def test_sync_batch_closed_form_and_shared_steps():
    """Attractive one-patch flows of different U on one schedule: each reaches its own
    closed-form T_c (the stop rule stays per flow), every running flow makes every attempt
    (equal counts while both run), and the group takes at least as many steps as either
    flow alone (its step is the smallest either proposes)."""
    m = O.model(1, L1)
    Us = [-3.0, -2.0]
    _, rs = O.flow_sync(m, O.flowcfg(T0=1.0, T_end=0.01, integrator=1, atol=0.0), Us)
    for U, r in zip(Us, rs):
        assert r["status"] == O.DIVERGED
        assert r["T_c"] == pytest.approx(_tc_exact(U, 20.0), rel=1e-3)
        _, r1, _ = O.flow(m, O.flowcfg(T0=1.0, T_end=0.01, integrator=1, U=U), U)
        assert r["n_accepted"] + r["n_rejected"] >= r1["n_accepted"] + r1["n_rejected"]
        assert r["T_c"] == pytest.approx(r1["T_c"], rel=1e-4)
    # -3 diverges first; until then the two flows share every attempt
    assert rs[0]["T_c"] > rs[1]["T_c"]
    assert rs[1]["n_accepted"] >= rs[0]["n_accepted"]
    assert rs[0]["n_rhs"] == 1 + 6 * (rs[0]["n_accepted"] + rs[0]["n_rejected"])
