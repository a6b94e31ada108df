"""Pins of the oracle's right-hand side and geometry against things it does not compute.

* spin reduction: a generic antisymmetric spin-resolved one-loop flow with exact momenta
  (``oracle/spinflow.py``) must give dG(up,down;up,down) = dV and
  dG(up,up;up,up) = dV(k1,k2,k3) - dV(k2,k1,k3), at random exchange-symmetric V and along a
  flow;
* a literal pure-Python brute force at N = 4 (``oracle/brute.py``);
* channel closures: the crossed term alone sums the RPA series for V = v(k3-k2), the
  particle-particle term alone the ladder for V = v(k1+k2);
* exact symmetries with exact momenta (identity patching): exchange, the swap of in- and
  out-going pairs, the eight lattice point-group operations and the shift of every
  momentum by Q = (pi, pi) at half filling; in patch mode the point-group relabelling and
  xi -> -xi;
* the binned regrouping equals the direct sum;
* geometry: the patch table is point-group symmetric, has no boundary ties, Fermi points of
  the half-filled diamond are snapped exactly, xi(k + Q) = -xi(k).
"""
import math

import numpy as np
import pytest

from oracle import brute, oracle as O, spinflow
from paper_2005_00827_amd import inputs


def _k4(L, a, b, c):
    return ((a % L + b % L - c % L) % L) + L * ((a // L + b // L - c // L) % L)


def _exchange_sym(V, L):
    N = L * L
    a, b, c = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    return 0.5 * (V + V[b, a, _k4(L, a, b, c)])


# --------------------------------------------------------------------------------------
# spin-resolved generic flow
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("T", [0.5, 0.07])
def test_spin_reduction_rhs(T):
    L = 4
    sf = spinflow.SpinFlow(L)
    V = _exchange_sym(inputs.random_state(L * L, seed=11), L)
    G = sf.gamma_from_v(V)
    assert np.abs(G + G.transpose(1, 0, 2, 3)).max() == 0.0
    dG = sf.rhs(G, T)
    dV = O.rhs(O.model(L * L, L, identity=True), T, V)
    scale = np.abs(dV).max()
    assert np.abs(sf.v_from_gamma(dG, (0, 1)) - dV).max() <= 1e-12 * scale
    assert np.abs(sf.v_from_gamma(dG, (1, 0)) - dV).max() <= 1e-12 * scale
    assert np.abs(sf.v_from_gamma(dG, (0, 0)) - (dV - dV.transpose(1, 0, 2))).max() <= 1e-12 * scale
    assert np.abs(sf.v_from_gamma(dG, (1, 1)) - (dV - dV.transpose(1, 0, 2))).max() <= 1e-12 * scale


def test_spin_reduction_along_flow():
    L, U = 4, 1.5
    sf = spinflow.SpinFlow(L)
    G = sf.gamma_from_v(np.full((16, 16, 16), U))
    G = sf.rk4_flow(G, 1.0, 0.2, 40)
    m = O.model(16, L, identity=True)
    cfg = O.flowcfg(T0=1.0, T_end=0.2, n_steps=40, v_max=1e300, U=U)
    V, res, _ = O.flow(m, cfg, U)
    assert res["status"] == O.REACHED_TEND
    assert np.abs(V - U).max() > 0.5  # the flow went somewhere
    assert np.abs(sf.v_from_gamma(G, (0, 1)) - V).max() <= 1e-11 * np.abs(V).max()
    assert np.abs(sf.v_from_gamma(G, (0, 0)) - (V - V.transpose(1, 0, 2))).max() <= 1e-11 * np.abs(V).max()


# --------------------------------------------------------------------------------------
# literal brute force
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("L,T", [(8, 0.3), (16, 0.1)])
def test_brute_force_n4(L, T):
    N = 4
    V = inputs.noisy_state(N, 2.0, seed=5, rel=0.3)
    Z = np.array([0.9, 0.8, 0.85, 0.95])
    ref = brute.rhs(V.tolist(), N, L, T, Z=Z.tolist())
    got = O.rhs(O.model(N, L), T, V, Z=Z)
    r = np.array([ref[(a, b, c)] for a in range(N) for b in range(N) for c in range(N)])
    assert np.abs(got.ravel() - r).max() <= 1e-11 * np.abs(r).max()


def test_brute_force_t_prime():
    """Away from half filling and with t' (the method is stated for general t', mu)."""
    N, L, T = 4, 8, 0.2
    V = inputs.noisy_state(N, 1.5, seed=6, rel=0.3)
    ref = brute.rhs(V.tolist(), N, L, T, t=1.0, tp=-0.3, mu=-0.4)
    got = O.rhs(O.model(N, L, t=1.0, tp=-0.3, mu=-0.4), T, V)
    r = np.array([ref[(a, b, c)] for a in range(N) for b in range(N) for c in range(N)])
    assert np.abs(got.ravel() - r).max() <= 1e-11 * np.abs(r).max()


# --------------------------------------------------------------------------------------
# channel closures (identity patching, exact momenta)
# --------------------------------------------------------------------------------------
def _fermi(x, T):
    return 0.5 * (1.0 - np.tanh(x / (2 * T)))


def _chi(x, y, T):
    """-(f(x)-f(y))/(x-y) with the -f' limit; numpy, from the Fermi function."""
    d = x - y
    same = np.abs(d) < 1e-12
    num = -(_fermi(x, T) - _fermi(y, T))
    fp = _fermi(x, T) * (1 - _fermi(x, T)) / T
    return np.where(same, fp, num / np.where(same, 1.0, d))


def _xi_grid(L, t=1.0):
    k = -math.pi + 2 * math.pi * (np.arange(L) + 0.5) / L
    return -2 * t * (np.cos(k)[None, :] + np.cos(k)[:, None])  # [jy, jx]


def loop_sum(L, m, T, pp):
    """(1/L^2) sum_j chi_X(xi_j, xi_j') for transfer index m = (mx, my)."""
    xi = _xi_grid(L)
    jy, jx = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    if pp:
        px, py = (m[0] - jx - 1) % L, (m[1] - jy - 1) % L
        return np.mean(_chi(xi, -xi[py, px], T))
    px, py = (jx + m[0]) % L, (jy + m[1]) % L
    return np.mean(_chi(xi, xi[py, px], T))


@pytest.mark.parametrize("channel", ["cr", "pp"])
def test_channel_closures(channel):
    L, U, T0, T1 = 4, 1.2 if channel == "cr" else -1.2, 1.0, 0.15
    N = L * L
    ch = O.CH_CR if channel == "cr" else O.CH_PP
    m = O.model(N, L, identity=True, channels=ch)
    cfg = O.flowcfg(T0=T0, T_end=T1, integrator=1, rtol=1e-12, atol=1e-14, v_max=1e300, U=U)
    V, res, _ = O.flow(m, cfg, U)
    assert res["status"] == O.REACHED_TEND
    worst = 0.0
    for a in range(N):
        for b in range(N):
            for c in range(N):
                if channel == "cr":
                    q = ((c % L - b % L) % L, (c // L - b // L) % L)
                    inv = 1 / U - (loop_sum(L, q, T1, False) - loop_sum(L, q, T0, False))
                else:
                    q = ((a % L + b % L + 1) % L, (a // L + b // L + 1) % L)
                    inv = 1 / U + (loop_sum(L, q, T1, True) - loop_sum(L, q, T0, True))
                worst = max(worst, abs(V[a, b, c] - 1 / inv))
    assert worst <= 1e-9 * np.abs(V).max()


# --------------------------------------------------------------------------------------
# exact symmetries
# --------------------------------------------------------------------------------------
def _c4v_point_maps(L):
    """The 8 point-group operations as permutations of loop-point indices (j = jx + L jy)."""
    j = np.arange(L * L)
    jx, jy = j % L, j // L
    rx = lambda x: L - 1 - x       # k -> -k on the half-shifted grid
    ops = []
    for swap in (False, True):
        for sx in (False, True):
            for sy in (False, True):
                x, y = (jy, jx) if swap else (jx, jy)
                x = rx(x) if sx else x
                y = rx(y) if sy else y
                ops.append(x + L * y)
    return ops


@pytest.fixture(scope="module")
def identity_flow():
    L, U = 6, 2.0
    N = L * L
    m = O.model(N, L, identity=True)
    cfg = O.flowcfg(T0=1.0, T_end=0.2, n_steps=30, v_max=1e300, U=U)
    V, res, _ = O.flow(m, cfg, U)
    return L, V


def test_identity_exchange_and_pair_swap(identity_flow):
    L, V = identity_flow
    N = L * L
    a, b, c = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    d = _k4(L, a, b, c)
    tol = 1e-12 * np.abs(V).max()
    assert np.abs(V - V[b, a, d]).max() <= tol              # exchange
    assert np.abs(V - V[c, d, a]).max() <= tol              # (k1 k2) <-> (k3 k4)
    assert np.abs(V - 2.0).max() > 0.1


def test_identity_point_group_and_nesting_shift(identity_flow):
    L, V = identity_flow
    tol = 1e-12 * np.abs(V).max()
    for g in _c4v_point_maps(L):
        assert np.abs(V - V[np.ix_(g, g, g)]).max() <= tol
    j = np.arange(L * L)
    sq = ((j % L + L // 2) % L) + L * ((j // L + L // 2) % L)   # k -> k + Q
    assert np.abs(V - V[np.ix_(sq, sq, sq)]).max() <= tol


def _patch_ops(N):
    """Point-group action on angular patch labels (theta_off = 0): theta -> theta + pi/2 and
    theta -> -theta generate the group."""
    a = np.arange(N)
    rot = (a + N // 4) % N
    ref = (-a) % N
    ops, frontier = {tuple(a)}, [a]
    while frontier:
        g = frontier.pop()
        for h in (rot, ref):
            gh = tuple(h[np.array(g)])
            if gh not in ops:
                ops.add(gh)
                frontier.append(np.array(gh))
    assert len(ops) == 8
    return [np.array(o) for o in ops]


def test_patch_mode_symmetries():
    N, L, U = 16, 32, 2.0
    cfg = O.flowcfg(T0=1.0, T_end=0.1, n_steps=40, v_max=1e300, U=U)
    V, _, _ = O.flow(O.model(N, L), cfg, U)
    tol = 1e-12 * np.abs(V).max()
    for g in _patch_ops(N):
        assert np.abs(V - V[np.ix_(g, g, g)]).max() <= tol
    # particle-hole symmetry of the half-filled band: (t, t', mu) -> (-t, -t', -mu)
    V2, _, _ = O.flow(O.model(N, L, t=-1.0), cfg, U)
    assert np.array_equal(V, V2)


def test_geometry_symmetric_and_tie_free():
    for N, L in [(16, 32), (48, 128), (96, 256), (4, 16), (8, 8)]:
        xi, patch, anchor, margin = O.geometry(O.model(N, L))
        assert margin > 1e-6
        P = patch.reshape(L, L)                     # [jy, jx]
        for g, pg in zip(_c4v_point_maps(L), _patch_perm_for_points(N)):
            assert np.array_equal(patch[g], pg[patch]), (N, L)
        # nesting: xi(k + Q) = -xi(k) on the half-shifted grid
        X = xi.reshape(L, L)
        assert np.allclose(np.roll(np.roll(X, L // 2, 0), L // 2, 1), -X, atol=1e-14)
        del P


def _patch_perm_for_points(N):
    """Patch relabelling matching each point map of _c4v_point_maps (same order)."""
    a = np.arange(N)
    off = 0.0 if N % 8 == 0 else math.pi / N
    th = off + 2 * math.pi * a / N
    out = []
    for swap in (False, True):
        for sx in (False, True):
            for sy in (False, True):
                c, s = np.cos(th), np.sin(th)
                # point map: (x, y) -> (y, x) if swap, then x -> -x if sx, y -> -y if sy
                x, y = (s, c) if swap else (c, s)
                x = -x if sx else x
                y = -y if sy else y
                t2 = np.arctan2(y, x)
                out.append(np.round((t2 - off) * N / (2 * math.pi)).astype(int) % N)
    return out


def test_half_filling_fermi_points_snapped():
    N, L = 16, 32
    _, _, anchor, _ = O.geometry(O.model(N, L))
    # antinode (pi, 0) and node (pi/2, pi/2) of the diamond |kx| + |ky| = pi
    assert tuple(anchor[0]) == (L // 2, 0)
    assert tuple(anchor[N // 8]) == (L // 4, L // 4)
    # every snapped point lies on (or next to) the diamond
    k = anchor.astype(float)
    k = np.where(k > L // 2, k - L, k) * 2 * math.pi / L
    assert np.all(np.abs(np.abs(k[:, 0]) + np.abs(k[:, 1]) - math.pi) <= 2 * 2 * math.pi / L)


def test_transfer_counts():
    # |{k_F(a) + k_F(b)}| = |{k_F(a) - k_F(b)}| since -k_F(b) = k_F(b + N/2)
    for (N, L), n in {(16, 32): 48, (48, 128): 424, (96, 256): 1520}.items():
        assert O.transfer_counts(O.model(N, L)) == (n, n)


# --------------------------------------------------------------------------------------
# binned regrouping
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("N,L,identity", [(16, 32, False), (8, 16, False), (16, 4, True)])
def test_direct_equals_binned(N, L, identity):
    V = inputs.noisy_state(N, 2.0, seed=7, rel=0.5)
    Z = 0.7 + 0.3 * np.random.default_rng(8).random(N)
    m = O.model(N, L, identity=identity)
    d1 = O.rhs(m, 0.13, V, Z=Z)
    d2 = O.rhs(m, 0.13, V, Z=Z, binned=True)
    assert np.abs(d1 - d2).max() <= 1e-13 * np.abs(d1).max()


def test_points_equal_full():
    N, L = 16, 32
    V = inputs.noisy_state(N, 2.0, seed=9)
    m = O.model(N, L)
    full = O.rhs(m, 0.2, V)
    abc = inputs.sample_indices(N, 40)
    pts = O.rhs_points(m, 0.2, V, abc)
    assert np.array_equal(pts, full[abc[:, 0], abc[:, 1], abc[:, 2]])


def test_constant_V_direct_channel_cancels():
    """For V = U the direct-channel bracket is (-2 + 1 + 1) U^2 = 0."""
    N, L = 16, 32
    d = O.rhs(O.model(N, L, channels=O.CH_D), 0.3, np.full((N, N, N), 2.0))
    assert np.abs(d).max() <= 1e-15
