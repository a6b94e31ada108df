"""Literal pure-Python brute force of the flow right-hand side for tiny sizes.

TEST INFRASTRUCTURE, independent of both the C oracle and the HIP path: no lookup tables,
every momentum, energy (cos per point), patch (atan2 per point) and Fermi point is
recomputed where it is used (with energy shells, the shell of each point's energy too), and
the bubble weight is taken from the Fermi function itself:

    chi_ph(x, y) = -(f(x) - f(y)) / (x - y),   T d/dT f(x) = (x/T) f(x) (1 - f(x)),
    T d/dT chi_ph(x, y) = -(g(x) - g(y)) / (x - y),   g = T d/dT f,
    chi_pp(x, y) = chi_ph(x, -y),

with the coincident-argument limit -g'(x).  Meant for N = 4 and L <= 16 (a few seconds).
Sums follow the explicit one-loop formula (particle-particle, crossed and direct
particle-hole terms) that the C oracle states; Sec. 2.1 Eq. free_dispersion_xi for the
dispersion.
"""
from __future__ import annotations

import math


def _fermi(x, T):
    return 0.5 * (1.0 - math.tanh(x / (2.0 * T)))


def _g(x, T):
    f = _fermi(x, T)
    return (x / T) * f * (1.0 - f)


def _gprime(x, T):
    f = _fermi(x, T)
    ff = f * (1.0 - f)
    return ff / T - (x / (T * T)) * ff * (1.0 - 2.0 * f)


def chidot_ph(x, y, T):
    if abs(x - y) <= 1e-9 * T:
        return -_gprime(0.5 * (x + y), T)
    return -(_g(x, T) - _g(y, T)) / (x - y)


def chidot_pp(x, y, T):
    return chidot_ph(x, -y, T)


def chi_ph(x, y, T):
    """Static bubble -(f(x) - f(y))/(x - y), -f'(x) = f(1 - f)/T on the diagonal."""
    if abs(x - y) <= 1e-9 * T:
        f = _fermi(0.5 * (x + y), T)
        return f * (1.0 - f) / T
    return -(_fermi(x, T) - _fermi(y, T)) / (x - y)


def chi_pp(x, y, T):
    return chi_ph(x, -y, T)


def _disp(kx, ky, t, tp, mu):
    return -2.0 * t * (math.cos(kx) + math.cos(ky)) - 4.0 * tp * math.cos(kx) * math.cos(ky) - mu


def _k(j, L):
    return -math.pi + 2.0 * math.pi * (j + 0.5) / L


def _off(N):
    return 0.0 if (N == 1 or N % 8 == 0) else math.pi / N


def _edges(S, t, edges):
    """The |xi| at which S (odd) energy shells meet: given, or 2|t| (2^k - 1)/(2^m - 1)."""
    m = (S - 1) // 2
    if edges is not None:
        return list(edges)
    return [2.0 * abs(t) * (2.0 ** k - 1.0) / (2.0 ** m - 1.0) for k in range(1, m + 1)]


def _shell(x, E):
    k = sum(1 for e in E if abs(x) > e)
    m = len(E)
    return m - k if x < 0 else m + k


def _level(e, E):
    """Representative energy of shell e: 0 at the Fermi surface, the middle of an inner
    shell, the outermost shell's edge plus half the width of the shell inside it."""
    m = len(E)
    k = abs(e - m)
    if k == 0:
        return 0.0
    lo = E[k - 1]
    mag = 0.5 * (lo + E[k]) if k < m else lo + 0.5 * (lo - (E[k - 2] if k > 1 else 0.0))
    return -mag if e < m else mag


def _patch_of(jx, jy, L, N, t=1.0, tp=0.0, mu=0.0, S=1, E=()):
    """Angular sector of the point (atan2) and, with S > 1 energy shells, the shell of its
    energy: patch = shell * (N / S) + sector."""
    ns = N // S
    th = math.atan2(_k(jy, L), _k(jx, L))
    sec = int(round((th - _off(ns)) * ns / (2.0 * math.pi))) % ns
    if S == 1:
        return sec
    return _shell(_disp(_k(jx, L), _k(jy, L), t, tp, mu), E) * ns + sec


def _fermi_index(a, N, L, t, tp, mu, S=1, E=()):
    """Snapped point of patch a's sector centre ray where xi reaches its shell's energy."""
    ns = N // S
    level = _level(a // ns, E) if S > 1 else 0.0
    th = _off(ns) + 2.0 * math.pi * (a % ns) / ns
    c, s = math.cos(th), math.sin(th)
    rmax = math.pi / max(abs(c), abs(s))
    ns = 4096
    prev = _disp(0.0, 0.0, t, tp, mu) - level
    rp = 0.0
    best, rb = abs(prev), 0.0
    r_root = None
    for i in range(1, ns + 1):
        r = rmax * i / ns
        f = _disp(r * c, r * s, t, tp, mu) - level
        if (prev < 0 <= f) or (prev > 0 >= f):
            lo, hi = rp, r
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                if mid <= lo or mid >= hi:
                    break
                fm = _disp(mid * c, mid * s, t, tp, mu) - level
                if (prev < 0 and fm < 0) or (prev > 0 and fm > 0):
                    lo = mid
                else:
                    hi = mid
            r_root = hi
            break
        if abs(f) < best:
            best, rb = abs(f), r
        rp, prev = r, f
    r = rb if r_root is None else r_root
    kx, ky = r * c, r * s
    # half-way cases round away from zero, as C's lround does
    rnd = lambda v: int(math.floor(v + 0.5)) if v >= 0 else -int(math.floor(-v + 0.5))
    return rnd(kx * L / (2.0 * math.pi)) % L, rnd(ky * L / (2.0 * math.pi)) % L


def rhs(V, N, L, T, t=1.0, tp=0.0, mu=0.0, channels=7, Z=None, n_shells=1, shell_edges=None,
        g=None, K=None):
    """V: nested list or array indexable as V[a][b][c]; returns a dict (a,b,c) -> dV/dlnT.
    n_shells > 1: energy-shell patches (N = n_shells x angular sectors).
    g: the interaction flow's dV/dg at scale g instead, each line pair (j, j') weighted by
    g Z_j Z_j' (K_j Z_j + K_j' Z_j') times the static bubble (K: Katanin factors, default 1)."""
    out = {}
    z = (lambda a: 1.0) if Z is None else (lambda a: Z[a])
    kat = (lambda a: 1.0) if K is None else (lambda a: K[a])

    def weight(pj, pu, x, y, pp):
        if g is None:
            return z(pj) * z(pu) * (chidot_pp(x, y, T) if pp else chidot_ph(x, y, T))
        b = chi_pp(x, y, T) if pp else chi_ph(x, y, T)
        return g * z(pj) * z(pu) * (kat(pj) * z(pj) + kat(pu) * z(pu)) * b
    n = L * L
    S = n_shells if n_shells > 1 else 1
    E = _edges(S, t, shell_edges) if S > 1 else []

    def _patch(jx, jy, L, N):
        return _patch_of(jx, jy, L, N, t, tp, mu, S, E)
    for a in range(N):
        fa = _fermi_index(a, N, L, t, tp, mu, S, E)
        for b in range(N):
            fb = _fermi_index(b, N, L, t, tp, mu, S, E)
            for c in range(N):
                fc = _fermi_index(c, N, L, t, tp, mu, S, E)
                qpp = ((fa[0] + fb[0]) % L, (fa[1] + fb[1]) % L)
                qcr = ((fc[0] - fb[0]) % L, (fc[1] - fb[1]) % L)
                qd = ((fa[0] - fc[0]) % L, (fa[1] - fc[1]) % L)
                s = 0.0
                for jy in range(L):
                    for jx in range(L):
                        x = _disp(_k(jx, L), _k(jy, L), t, tp, mu)
                        pj = _patch(jx, jy, L, N)
                        if channels & 1:
                            ux, uy = (qpp[0] - jx - 1) % L, (qpp[1] - jy - 1) % L
                            y = _disp(_k(ux, L), _k(uy, L), t, tp, mu)
                            pu = _patch(ux, uy, L, N)
                            w = weight(pj, pu, x, y, True)
                            s -= w * V[a][b][pj] * V[pj][pu][c]
                        if channels & 2:
                            ux, uy = (jx + qcr[0]) % L, (jy + qcr[1]) % L
                            y = _disp(_k(ux, L), _k(uy, L), t, tp, mu)
                            pu = _patch(ux, uy, L, N)
                            w = weight(pj, pu, x, y, False)
                            s += w * V[a][pj][pu] * V[pu][b][c]
                        if channels & 4:
                            ux, uy = (jx + qd[0]) % L, (jy + qd[1]) % L
                            y = _disp(_k(ux, L), _k(uy, L), t, tp, mu)
                            pu = _patch(ux, uy, L, N)
                            w = weight(pj, pu, x, y, False)
                            s += w * (-2.0 * V[a][pj][c] * V[pu][b][pj]
                                      + V[pj][a][c] * V[pu][b][pj]
                                      + V[a][pj][c] * V[b][pu][pj])
                out[(a, b, c)] = s / n
    return out
