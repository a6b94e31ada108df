"""Literal pure-Python brute force of the flow right-hand side for tiny sizes.

TEST INFRASTRUCTURE, independent of both the C oracle and the HIP path: no lookup tables,
every momentum, energy (cos per point), patch (atan2 per point) and Fermi point is
recomputed where it is used, and the bubble weight is taken from the Fermi function itself:

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


def _disp(kx, ky, t, tp, mu):
    return -2.0 * t * (math.cos(kx) + math.cos(ky)) - 4.0 * tp * math.cos(kx) * math.cos(ky) - mu


def _k(j, L):
    return -math.pi + 2.0 * math.pi * (j + 0.5) / L


def _off(N):
    return 0.0 if (N == 1 or N % 8 == 0) else math.pi / N


def _patch(jx, jy, L, N):
    th = math.atan2(_k(jy, L), _k(jx, L))
    return int(round((th - _off(N)) * N / (2.0 * math.pi))) % N


def _fermi_index(a, N, L, t, tp, mu):
    th = _off(N) + 2.0 * math.pi * a / N
    c, s = math.cos(th), math.sin(th)
    rmax = math.pi / max(abs(c), abs(s))
    ns = 4096
    prev = _disp(0.0, 0.0, t, tp, mu)
    rp = 0.0
    best, rb = abs(prev), 0.0
    r_root = None
    for i in range(1, ns + 1):
        r = rmax * i / ns
        f = _disp(r * c, r * s, t, tp, mu)
        if (prev < 0 <= f) or (prev > 0 >= f):
            lo, hi = rp, r
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                if mid <= lo or mid >= hi:
                    break
                fm = _disp(mid * c, mid * s, t, tp, mu)
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


def rhs(V, N, L, T, t=1.0, tp=0.0, mu=0.0, channels=7, Z=None):
    """V: nested list or array indexable as V[a][b][c]; returns a dict (a,b,c) -> dV/dlnT."""
    out = {}
    z = (lambda a: 1.0) if Z is None else (lambda a: Z[a])
    n = L * L
    for a in range(N):
        fa = _fermi_index(a, N, L, t, tp, mu)
        for b in range(N):
            fb = _fermi_index(b, N, L, t, tp, mu)
            for c in range(N):
                fc = _fermi_index(c, N, L, t, tp, mu)
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
                            w = z(pj) * z(pu) * chidot_pp(x, y, T)
                            s -= w * V[a][b][pj] * V[pj][pu][c]
                        if channels & 2:
                            ux, uy = (jx + qcr[0]) % L, (jy + qcr[1]) % L
                            y = _disp(_k(ux, L), _k(uy, L), t, tp, mu)
                            pu = _patch(ux, uy, L, N)
                            w = z(pj) * z(pu) * chidot_ph(x, y, T)
                            s += w * V[a][pj][pu] * V[pu][b][c]
                        if channels & 4:
                            ux, uy = (jx + qd[0]) % L, (jy + qd[1]) % L
                            y = _disp(_k(ux, L), _k(uy, L), t, tp, mu)
                            pu = _patch(ux, uy, L, N)
                            w = z(pj) * z(pu) * chidot_ph(x, y, T)
                            s += w * (-2.0 * V[a][pj][c] * V[pu][b][pj]
                                      + V[pj][a][c] * V[pu][b][pj]
                                      + V[a][pj][c] * V[b][pu][pj])
                out[(a, b, c)] = s / n
    return out
