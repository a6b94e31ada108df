"""Energy-shell patching (Sec. 3.2: the angular patches subdivided in energy, 7 shells x 32
sectors = 224 patches), pinned on the oracle:

* patch assignment and representative points against the literal pure-Python brute force
  (atan2 and the shell of each point's energy, a ray scan per patch);
* one shell is the angular geometry, bit for bit, in the geometry and the right-hand side;
* the right-hand side at N = 3 x 4, L = 8 against the brute-force loop sums;
* the binned regrouping equals the direct sums with shells;
* rotating every sector by a quarter turn within its shell leaves the right-hand side of a
  constant V unchanged (the shells are invariant under the point group);
* the library's host geometry equals the oracle's bit for bit (tests/test_abi.py).
"""
import math

import numpy as np
import pytest

from oracle import brute
from oracle import oracle as O
from paper_2005_00827_amd import inputs


@pytest.mark.parametrize("N,L,S,edges", [(24, 32, 3, None), (40, 32, 5, [0.3, 1.1]),
                                         (56, 64, 7, None), (12, 8, 3, None)])
def test_shell_patches_and_points_against_brute_force(N, L, S, edges):
    m = O.model(N, L, n_shells=S, shell_edges=edges)
    _, patch, anchor, _ = O.geometry(m)
    E = brute._edges(S, 1.0, edges)
    for jy in range(L):
        for jx in range(L):
            assert patch[jx + L * jy] == brute._patch_of(jx, jy, L, N, 1.0, 0.0, 0.0, S, E)
    for a in range(N):
        assert tuple(anchor[a]) == brute._fermi_index(a, N, L, 1.0, 0.0, 0.0, S, E), a
    # every shell holds points, the Fermi-surface shell the most per unit energy
    counts = np.bincount(patch // (N // S), minlength=S)
    assert counts.min() > 0


def test_one_shell_is_the_angular_geometry():
    for N, L in ((16, 32), (48, 128)):
        ga = O.geometry(O.model(N, L))
        gs = O.geometry(O.model(N, L, n_shells=1))
        for x, y in zip(ga[:3], gs[:3]):
            assert np.array_equal(x, y)
    V = inputs.noisy_state(16, 2.0)
    a = O.rhs(O.model(16, 32), 0.1, V)
    b = O.rhs(O.model(16, 32, n_shells=1), 0.1, V)
    assert np.array_equal(a, b)


def test_shell_rhs_against_brute_force():
    N, L, S, T = 12, 8, 3, 0.3
    V = inputs.noisy_state(N, 2.0, seed=5)
    ref = brute.rhs(V.tolist(), N, L, T, n_shells=S)
    got = O.rhs(O.model(N, L, n_shells=S), T, V)
    want = np.array([[[ref[(a, b, c)] for c in range(N)] for b in range(N)] for a in range(N)])
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_shell_direct_equals_binned():
    N, L = 24, 32
    V = inputs.noisy_state(N, 2.0, seed=3)
    m = O.model(N, L, n_shells=3)
    d = O.rhs(m, 0.07, V)
    b = O.rhs(m, 0.07, V, binned=True)
    assert np.abs(d - b).max() <= 1e-13 * np.abs(d).max()


def test_shell_quarter_turn_invariance():
    N, L, S = 24, 32, 3
    ns = N // S
    d = O.rhs(O.model(N, L, n_shells=S), 0.1, inputs.constant_state(N, 2.5))
    a = np.arange(N)
    r = (a // ns) * ns + (a % ns + ns // 4) % ns
    assert np.abs(d[np.ix_(r, r, r)] - d).max() <= 1e-13 * np.abs(d).max()
    assert np.abs(d).max() > 1e-3
