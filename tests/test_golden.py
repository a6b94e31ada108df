"""Pins against published values kept as small text fixtures under tests/golden/.

* dopri5_tableau.txt: the Dormand-Prince RK5(4)7M coefficients as printed by Dormand and
  Prince (1980); the oracle's tableau must equal them exactly (to double rounding), and the
  oracle's error weights must be the fifth- minus fourth-order weights.
* angular_patches.txt: the paper's angular resolution (Sec. 3.2), 48 patches with seven
  centres from the antinodal to the nodal direction inclusive; the oracle's patch centres,
  read off the Fermi points it assigns, must have that count.
"""
import math
import os
from fractions import Fraction

import numpy as np

from oracle import oracle as O

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            yield line


def test_dopri_tableau_matches_the_published_coefficients():
    c, a, e = O.dopri_tableau()
    b, bh = {}, {}
    for line in _rows("dopri5_tableau.txt"):
        lhs, rhs = line.split("=")
        v = float(Fraction(rhs.strip()))
        f = lhs.split()
        if f[0] == "c":
            assert c[int(f[1])] == v, line
        elif f[0] == "a":
            assert a[int(f[1]), int(f[2])] == v, line
        elif f[0] == "b":
            b[int(f[1])] = Fraction(rhs.strip())
        elif f[0] == "bh":
            bh[int(f[1])] = Fraction(rhs.strip())
    assert len(b) == len(bh) == 7
    for i in range(7):
        assert e[i] == float(b[i] - bh[i]), i


def test_angular_patch_centres_from_antinode_to_node():
    """Each patch's centre is the circular mean angle of the loop points the oracle assigns
    to it; the patches centred from the antinodal to the nodal direction are counted."""
    for line in _rows("angular_patches.txt"):
        N, want = (int(x) for x in line.split())
        L = 128
        _, patch, _, _ = O.geometry(O.model(N, L))
        k = -math.pi + 2.0 * math.pi * (np.arange(L) + 0.5) / L
        ky, kx = np.meshgrid(k, k, indexing="ij")
        ang = np.arctan2(ky, kx).reshape(-1)
        cs = np.bincount(patch, weights=np.cos(ang), minlength=N)
        sn = np.bincount(patch, weights=np.sin(ang), minlength=N)
        centre = np.arctan2(sn, cs)
        n = int(np.sum((centre > -1e-6) & (centre < math.pi / 4 + 1e-6)))
        assert n == want, (N, n, np.degrees(np.sort(centre)))
