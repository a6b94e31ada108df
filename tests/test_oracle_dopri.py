"""Pins of the oracle's Dormand-Prince error estimate and step-size control.

The paper integrates its flow as an ordinary differential equation without naming the
scheme; the reading taken is Dormand-Prince 5(4) with the embedded error estimate
E = y5 - y4, the norm err = max_i |E_i| / (atol + rtol max(|V_i|, |V_i^new|)), acceptance at
err <= 1 and the step law h <- h min(5, max(0.2, 0.9 err^(-1/5))).  These tests fix that
reading against sources other than the oracle's own code:

* one attempt rebuilt in numpy from the published tableau (tests/golden/dopri5_tableau.txt)
  and the oracle's right-hand side, with the error weights formed from the published
  fifth- and fourth-order weights (not from the oracle's difference weights);
* the same attempt through scipy's Dormand-Prince stage routine and tableau
  (scipy.integrate RK45, after Hairer, Norsett and Wanner, Solving ODEs I, Sec. II.4), whose
  safety factor, smallest factor and error order give the step law;
* a whole one-patch flow against scipy's adaptive driver, whose accepted points coincide
  with the oracle's where neither driver's clamps act (scipy's RMS norm is the max norm on
  one component);
* properties no slip survives: the estimate scales as h^5 (a fourth-order embedded method),
  and a step proposed by the law meets err = 0.9^5 on a smooth problem (exponent -1/5);
* the rounding-order amplification of an adaptive flow, measured on the oracle alone by
  evaluating every right-hand side in the binned order: the step schedule moves by ~1e-9 in
  ln T and the final states differ by ~1e-10, while the same schedule replayed in both
  orders agrees to rounding.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from paper_2005_00827_amd import inputs

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def published_tableau():
    """Nodes, coupling, fifth-order weights and the error weights b - bh (formed exactly
    from the rationals, so that the estimate is not the difference of two rounded sums)."""
    c = np.zeros(7)
    a = np.zeros((7, 7))
    b = np.zeros(7)
    bf, bhf = {}, {}
    for line in open(os.path.join(GOLD, "dopri5_tableau.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        lhs, rhs = line.split("=")
        f = lhs.split()
        v = float(Fraction(rhs.strip()))
        if f[0] == "c":
            c[int(f[1])] = v
        elif f[0] == "a":
            a[int(f[1]), int(f[2])] = v
        elif f[0] == "b":
            b[int(f[1])] = v
            bf[int(f[1])] = Fraction(rhs.strip())
        elif f[0] == "bh":
            bhf[int(f[1])] = Fraction(rhs.strip())
    e = np.array([float(bf[i] - bhf[i]) for i in range(7)])
    return c, a, b, e


M4 = O.model(4, 16)
RTOL, ATOL = 1e-6, 1e-9


def f_of(m):
    """The oracle's right-hand side as f(s, y) with s = ln T and a flat state."""
    N = m.N

    def f(s, y):
        return O.rhs(m, math.exp(s), np.asarray(y, np.float64).reshape(N, N, N)).reshape(-1)
    return f


def numpy_attempt(m, s, h, V):
    """One attempt from the published tableau: stages, y5, and E = y5 - y4 from the
    difference of the fifth- and fourth-order weights."""
    c, a, b, e = published_tableau()
    f = f_of(m)
    y = V.reshape(-1)
    k = []
    for i in range(7):
        arg = y + h * sum(a[i, j] * k[j] for j in range(i))
        k.append(f(s + c[i] * h, arg))
    y5 = y + h * sum(b[i] * k[i] for i in range(7))
    E = h * sum(e[i] * k[i] for i in range(7))
    scale = ATOL + RTOL * np.maximum(np.abs(y), np.abs(y5))
    return y5, float(np.max(np.abs(E) / scale))


@pytest.mark.parametrize("h", [-0.05, -0.4, -1.2])
def test_one_attempt_from_the_published_tableau(h):
    """err, the accepted state and the proposed step of one oracle attempt, against an
    attempt assembled from the published coefficients (accepted at -0.05, rejected at
    -1.2)."""
    V = inputs.noisy_state(4, 2.0)
    s = math.log(0.3)
    y5, err = numpy_attempt(M4, s, h, V)
    cfg = O.flowcfg(U=1.0, integrator=1, rtol=RTOL, atol=ATOL)
    ls, hn, Vn, acc, oerr = O.step(M4, cfg, s, h, V)
    assert oerr == pytest.approx(err, rel=1e-9)
    assert acc == (err <= 1.0)
    want = h * min(5.0, max(0.2, 0.9 * err ** -0.2))
    assert hn == pytest.approx(want, rel=1e-9)
    if acc:
        assert np.abs(Vn.reshape(-1) - y5).max() <= 1e-13 * np.abs(y5).max()
        assert ls == s + h
    else:
        assert np.array_equal(Vn, V)
    if h == -0.05:
        assert acc
    if h == -1.2:
        assert not acc


@pytest.mark.parametrize("h", [-0.05, -0.4, -1.2])
def test_one_attempt_against_scipy(h):
    """The same attempt through scipy's Dormand-Prince stage routine and tableau; the step
    law with scipy's safety factor, smallest factor and error order (largest factor 5 is
    this reading's, scipy's driver uses 10)."""
    from scipy.integrate._ivp import rk
    V = inputs.noisy_state(4, 2.0)
    s = math.log(0.3)
    f = f_of(M4)
    y = V.reshape(-1).copy()
    K = np.empty((rk.RK45.n_stages + 1, y.size))
    y5, _ = rk.rk_step(f, s, y, f(s, y), h, rk.RK45.A, rk.RK45.B, rk.RK45.C, K)
    E = K.T @ rk.RK45.E * h
    scale = ATOL + RTOL * np.maximum(np.abs(y), np.abs(y5))
    err = float(np.max(np.abs(E) / scale))
    cfg = O.flowcfg(U=1.0, integrator=1, rtol=RTOL, atol=ATOL)
    ls, hn, Vn, acc, oerr = O.step(M4, cfg, s, h, V)
    assert oerr == pytest.approx(err, rel=1e-9)
    expo = -1.0 / (rk.RK45.error_estimator_order + 1)
    want = h * min(5.0, max(rk.MIN_FACTOR, rk.SAFETY * err ** expo))
    assert hn == pytest.approx(want, rel=1e-9)
    if acc:
        assert np.abs(Vn.reshape(-1) - y5).max() <= 1e-13 * np.abs(y5).max()


def test_whole_flow_against_scipy_driver():
    """One patch (a single component, where scipy's RMS norm is the max norm), T from 1 to
    0.3, tolerances chosen so that every factor stays inside (0.2, 5) and no attempt is
    rejected (scipy caps the factor after a rejection at 1, this reading does not): scipy's
    adaptive driver and the oracle's then take the same steps."""
    from scipy.integrate import solve_ivp
    m = O.model(1, 32)
    U, s0, s1 = 1.5, 0.0, math.log(0.3)
    rtol, atol, h0 = 1e-8, 1e-11, -0.05

    def f(s, y):
        return O.rhs(m, math.exp(s), np.array(y).reshape(1, 1, 1)).reshape(-1)

    sol = solve_ivp(f, (s0, s1), [U], method="RK45", rtol=rtol, atol=atol, first_step=abs(h0))
    assert sol.status == 0
    n_steps = len(sol.t) - 1
    assert sol.nfev == 1 + 6 * n_steps          # no rejected attempt
    hs = np.diff(sol.t)
    inner = hs[1:-1] / hs[:-2]                  # factors between full (unclamped) steps
    assert inner.min() > 0.2 and inner.max() < 5.0
    cfg = O.flowcfg(T0=1.0, T_end=0.3, U=U, integrator=1, rtol=rtol, atol=atol, h0=h0,
                    v_max=1e300)
    V, res, trace = O.flow(m, cfg, U)
    assert res["status"] == O.REACHED_TEND
    assert res["n_accepted"] == n_steps and res["n_rejected"] == 0
    # the estimate is a small difference of stage sums, so its rounding (summation order
    # differs between the two codes) moves each proposed step by ~1e-9 relative; a slip in
    # the norm or the law would move it by percent
    np.testing.assert_allclose(trace[:, 0], sol.t, rtol=0, atol=1e-7)
    np.testing.assert_allclose(trace[:, 1], np.abs(sol.y[0]), rtol=1e-9)
    assert V[0, 0, 0] == pytest.approx(sol.y[0, -1], rel=1e-12)


def test_error_estimate_is_fifth_order_and_the_law_targets_its_safety_factor():
    """A fourth-order embedded estimate scales as h^5: halving h divides err by 32.  The
    law's exponent -1/5 then proposes the step whose err is 0.9^5 = 0.59 (a slip to -1/4
    would give 0.59 err^-1/4, far from 0.59 for these err)."""
    V = inputs.noisy_state(4, 2.0)
    s = math.log(0.3)
    cfg = O.flowcfg(U=1.0, integrator=1, rtol=1e-10, atol=1e-13)
    errs = []
    for h in (-0.02, -0.01, -0.005):
        errs.append(O.step(M4, cfg, s, h, V)[4])
    for e1, e2 in zip(errs, errs[1:]):
        assert 28.0 < e1 / e2 < 36.0, errs
    for h in (-0.04, -0.08):        # one accepted, one rejected attempt, factors unclamped
        _, hn, _, acc, e0 = O.step(M4, cfg, s, h, V)
        assert 1.9e-4 < e0 < 1.9e3 and acc == (e0 <= 1.0)
        e1 = O.step(M4, cfg, s, hn, V)[4]
        assert e1 == pytest.approx(0.9 ** 5, rel=0.1), (h, e0, hn, e1)


def test_rounding_order_amplification_of_adaptive_flows():
    """The oracle alone, every right-hand side once in the direct and once in the binned
    order (equal to ~1e-15 per evaluation).  The error estimate of an accepted step is tiny,
    so its rounding moves the proposed step, the schedule shifts by up to ~1e-9 in ln T and
    the states at the divergence differ by up to ~1e-10 (measured: 1.05e-10 for U = 2 with a
    first step of -1, 6.8e-11 for U = 1.5 from T0 = 0.7).  The binned order is checked
    against the direct one per evaluation in tests/test_oracle_rhs.py.  Replaying one schedule in both
    orders agrees to rounding, and T_c is unaffected.  These numbers bound how closely two
    correct implementations of an adaptive flow can agree in the final state."""
    m = O.model(16, 32)
    worst = 0.0
    for kw in (dict(T0=0.7, U=1.5), dict(T0=1.0, U=2.0, h0=-1.0)):
        cfg_d = O.flowcfg(integrator=1, **kw)
        cfg_b = O.flowcfg(integrator=1, binned=True, **kw)
        Vd, rd, td = O.flow(m, cfg_d, kw["U"])
        Vb, rb, tb = O.flow(m, cfg_b, kw["U"])
        assert rd["status"] == rb["status"] == O.DIVERGED
        assert (rd["n_accepted"], rd["n_rejected"]) == (rb["n_accepted"], rb["n_rejected"])
        assert abs(rb["T_c"] / rd["T_c"] - 1.0) < 1e-11
        shift = np.abs(td[:, 0] - tb[:, 0]).max()
        d = np.abs(Vd - Vb).max() / np.abs(Vd).max()
        worst = max(worst, d)
        assert 1e-12 < shift < 1e-8, shift
        assert d < 5e-10, d
        # the direct flow's schedule replayed in the binned order
        V = np.full((16, 16, 16), kw["U"])
        Vr = V.copy()
        for i in range(len(td) - 1):
            s, h = td[i, 0], td[i + 1, 0] - td[i, 0]
            _, _, V, acc_d, _ = O.step(m, O.flowcfg(integrator=1, rtol=1e30, **kw), s, h, V)
            _, _, Vr, acc_b, _ = O.step(m, O.flowcfg(integrator=1, rtol=1e30, binned=True, **kw),
                                        s, h, Vr)
            assert acc_d and acc_b
        assert np.abs(V - Vr).max() / np.abs(V).max() < 1e-13
        assert np.abs(V - Vd).max() / np.abs(Vd).max() < 1e-13
    assert worst > 1e-11


def test_rounding_order_amplification_of_interaction_flows():
    """The same measurement for the interaction flow (U = 3 at T = 0.1, which diverges): the
    two summation orders end 1.6e-10 apart in V, with g* equal to rounding."""
    m = O.model(16, 32)
    kw = dict(T0=0.1, U=3.0, integrator=1, gflow=True)
    Vd, rd, _ = O.flow(m, O.flowcfg(**kw), 3.0)
    Vb, rb, _ = O.flow(m, O.flowcfg(binned=True, **kw), 3.0)
    assert rd["status"] == rb["status"] == O.DIVERGED
    assert (rd["n_accepted"], rd["n_rejected"]) == (rb["n_accepted"], rb["n_rejected"])
    assert abs(rb["g_c"] / rd["g_c"] - 1.0) < 1e-12
    d = np.abs(Vd - Vb).max() / np.abs(Vd).max()
    assert 1e-12 < d < 5e-10, d
