"""Generic spin-resolved one-loop flow of an antisymmetric static four-point vertex.

TEST INFRASTRUCTURE. An independent check of the spin-summed channel formula used by the C
oracle: here nothing is reduced by spin symmetry.  Single-particle states are (k, sigma)
with k on the half-shifted L x L grid (exact momenta, no patches).  The vertex
G[o1, o2, i1, i2] is antisymmetric in (o1, o2) and in (i1, i2) and conserves momentum.

Flow in s = ln T at one loop, static vertex (App. A, Eq. vertex_flow_general with bare
internal lines):

    dG/ds [o1 o2; i1 i2] = -1/2 sum_{m1 m2} G[o1 o2; m1 m2] Wpp(m1, m2) G[m1 m2; i1 i2]
                           - sum_{m1 m2} ( G[o1 m2; i1 m1] Wph(m1, m2) G[m1 o2; m2 i2]
                                           - (o1 <-> o2) )

with Wpp = T d/dT chi_pp(xi_m1, xi_m2) / L^2 and Wph = T d/dT chi_ph(xi_m1, xi_m2) / L^2.
The two overall signs are fixed by second-order perturbation theory of the Hubbard model
(opposite-spin vertex U - U^2 chi_pp(k1+k2) + U^2 chi_ph(k1-k4)); nothing else is chosen.

Spin-rotation-invariant vertices are built from a coupling function V as
    G[(k3 s3)(k4 s4); (k1 s1)(k2 s2)] = V(k1,k2,k3) d(s1,s3) d(s2,s4) - V(k2,k1,k3) d(s1,s4) d(s2,s3).
"""
from __future__ import annotations

import math

import numpy as np

from . import brute


def _k(j, L):
    return -math.pi + 2.0 * math.pi * (j + 0.5) / L


class SpinFlow:
    def __init__(self, L, t=1.0, tp=0.0, mu=0.0):
        self.L = L
        self.nk = L * L
        self.ns = 2 * self.nk
        kx = np.array([_k(j % L, L) for j in range(self.nk)])
        ky = np.array([_k(j // L, L) for j in range(self.nk)])
        self.xi = -2 * t * (np.cos(kx) + np.cos(ky)) - 4 * tp * np.cos(kx) * np.cos(ky) - mu
        st = np.arange(self.ns)
        self.kof = st // 2
        self.sof = st % 2
        jx, jy = self.kof % L, self.kof // L
        # momentum conservation k_o1 + k_o2 = k_i1 + k_i2 on the half-shifted grid
        ox = (jx[:, None, None, None] + jx[None, :, None, None]
              - jx[None, None, :, None] - jx[None, None, None, :]) % L
        oy = (jy[:, None, None, None] + jy[None, :, None, None]
              - jy[None, None, :, None] - jy[None, None, None, :]) % L
        self.cons = (ox == 0) & (oy == 0)

    def weights(self, T):
        x = self.xi[self.kof]
        n = self.ns
        wpp = np.empty((n, n))
        wph = np.empty((n, n))
        for i in range(n):
            for j in range(n):
                wpp[i, j] = brute.chidot_pp(x[i], x[j], T)
                wph[i, j] = brute.chidot_ph(x[i], x[j], T)
        return wpp / self.nk, wph / self.nk

    def gamma_from_v(self, V):
        """V[a, b, c] with a, b, c loop-point indices (k = jx + L jy); k4 implied."""
        L, n = self.L, self.ns
        k, s = self.kof, self.sof
        o1, o2, i1, i2 = np.ix_(range(n), range(n), range(n), range(n))
        G = (V[k[i1], k[i2], k[o1]] * ((s[i1] == s[o1]) & (s[i2] == s[o2]))
             - V[k[i2], k[i1], k[o1]] * ((s[i1] == s[o2]) & (s[i2] == s[o1])))
        return np.where(self.cons, G, 0.0)

    def v_from_gamma(self, G, s_in=(0, 1)):
        """Component G[(k3 s1)(k4 s2); (k1 s1)(k2 s2)] as V-shaped array [k1, k2, k3]."""
        L, nk = self.L, self.nk
        s1, s2 = s_in
        out = np.zeros((nk, nk, nk))
        for a in range(nk):
            for b in range(nk):
                for c in range(nk):
                    dx = ((a % L) + (b % L) - (c % L)) % L
                    dy = ((a // L) + (b // L) - (c // L)) % L
                    d = dx + L * dy
                    out[a, b, c] = G[2 * c + s1, 2 * d + s2, 2 * a + s1, 2 * b + s2]
        return out

    def rhs(self, G, T, weights=None):
        wpp, wph = self.weights(T) if weights is None else weights
        n = self.ns
        n2 = n * n
        Gm = G.reshape(n2, n2)
        pp = (Gm @ (wpp.reshape(n2)[:, None] * Gm)).reshape(n, n, n, n)
        X = G.transpose(0, 2, 3, 1).reshape(n2, n2)          # X[o1 i1, m1 m2] = G[o1 m2 i1 m1]
        Y = G.transpose(0, 2, 1, 3).reshape(n2, n2)          # Y[m1 m2, o2 i2] = G[m1 o2 m2 i2]
        D = (X @ (wph.reshape(n2)[:, None] * Y)).reshape(n, n, n, n)  # D[o1 i1 o2 i2]
        ph = D.transpose(0, 2, 1, 3) - D.transpose(2, 0, 1, 3)
        return -0.5 * pp - ph

    def rk4_flow(self, G, T0, T1, n_steps):
        s0, s1 = math.log(T0), math.log(T1)
        h = (s1 - s0) / n_steps
        for st in range(n_steps):
            s = s0 + st * h
            k1 = self.rhs(G, math.exp(s))
            k2 = self.rhs(G + 0.5 * h * k1, math.exp(s + 0.5 * h))
            k3 = self.rhs(G + 0.5 * h * k2, math.exp(s + 0.5 * h))
            k4 = self.rhs(G + h * k3, math.exp(s + h))
            G = G + h / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
        return G
