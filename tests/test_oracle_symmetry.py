"""Pins of the premise of the symmetric-state mode, on the oracle alone: the point group of the
square lattice maps the model onto itself, so

* the right-hand side of a point-group-invariant state is invariant (the flow keeps the
  symmetry: V(pi a, pi b, pi c) = V(a, b, c) for every operation, given Z_{pi a} = Z_a);
* the right-hand side is equivariant for any state: rhs(V o pi)(a, b, c) = rhs(V)(pi a, pi b, pi c);
* the synthetic Z table of the workloads is invariant (it depends on cos 4 theta).

The permutations pi come from the oracle's geometry: each loop point (jx, jy) mapped by the
operation (swap for o & 4, mirror x for o & 2, mirror y for o & 1, on the half-shifted grid
where j -> L - 1 - j is k -> -k) and the patch of its image read off.  A wrong equivariance
(a patch permutation that is not the lattice's, a channel whose transfer does not transform
with its pair) fails the second check at rounding level.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2005_00827_amd import inputs


def group_perms(m):
    _, patch, _, _ = O.geometry(m)
    L, N = m.L, m.N
    P = np.asarray(patch).reshape(L, L)
    jy, jx = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    out = []
    for o in range(8):
        x, y = (jy, jx) if o & 4 else (jx, jy)
        if o & 2:
            x = L - 1 - x
        if o & 1:
            y = L - 1 - y
        p = -np.ones(N, np.int64)
        p[P.ravel()] = P[y, x].ravel()
        assert (p >= 0).all() and len(set(p.tolist())) == N    # a permutation of the patches
        out.append(p)
    return out


def permute(V, p):
    return V[np.ix_(p, p, p)]


@pytest.mark.parametrize("N,L,tp,mu", [(8, 16, 0.0, 0.0), (16, 32, 0.0, 0.0), (16, 32, -0.3, -0.4)])
def test_rhs_is_equivariant_and_keeps_the_symmetry(N, L, tp, mu):
    m = O.model(N, L, tp=tp, mu=mu)
    perms = group_perms(m)
    T = 0.15
    lnT, tab = inputs.synthetic_z_table(N, 2.5, 1.0, 0.01)
    Z = np.array([np.interp(math.log(T), lnT, tab[:, a]) for a in range(N)])
    for p in perms:                                        # the table is invariant
        assert np.abs(tab[:, p] - tab).max() <= 1e-14
    V = inputs.random_state(N, seed=11)
    d = O.rhs(m, T, V, Z=Z)
    scale = np.abs(d).max()
    for o, p in enumerate(perms):
        dp = O.rhs(m, T, permute(V, p), Z=Z)
        assert np.abs(dp - permute(d, p)).max() <= 1e-12 * scale, o
    Vs = sum(permute(V, p) for p in perms) / len(perms)
    ds = O.rhs(m, T, Vs, Z=Z)
    for o, p in enumerate(perms):
        assert np.abs(permute(ds, p) - ds).max() <= 1e-12 * np.abs(ds).max(), o
    # a permutation that is not the lattice's breaks the equivariance
    q = np.roll(np.arange(N), 1)
    dq = O.rhs(m, T, permute(V, q), Z=Z)
    assert np.abs(dq - permute(d, q)).max() > 1e-3 * scale
