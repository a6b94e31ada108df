"""Pins of the oracle's Katanin correction of the interaction flow (App. A, Step 3): the
single-scale line S_g = Z^2 G0 becomes dG_g/dg = K Z^2 G0, so a line pair carries
g Z_a Z_b (K_a Z_a + K_b Z_b) chi (Eq. vertex_flow_feedback_Z_with_Katanin), and the tables
K_g = 1 + g^2 d_w Re(d Sigma_g / dg) (Eq. K_definition), A_g = -(2/g)(1 - Z_g K_g)
(Eq. A_g_simple).

* K = 1 is the Z-only flow bit for bit; a constant K = k multiplies the right-hand side by k
  and a flow with constant Z = z and K = k equals the plain flow of k z^3 U, rescaled.
* Per-patch K against the literal brute force (K on the line that carries Z^2, each patch
  its own factor).
* Second order: V(1) - U = U^2 int_0^1 g Z_a Z_b (K_a Z_a + K_b Z_b) chi dg + O(U^3) with
  g- and patch-dependent tables, by quadrature of numpy bubble sums.
* The tables: for Z_g from the slope s_g = c g^4 (second-order perturbation theory at
  coupling g^2 U, g Sigma_g = Sigma^(2)[g^2 U]) K = 1 + 3 s and A = 8 s / (g (1 - s)), reached
  at second order in the node spacing; Z from the oracle's own self-energy at g^2 U has
  exactly that g^4 law, so its K equals the one of the closed form.
"""
import numpy as np
import pytest

from oracle import brute
from oracle import oracle as O


def gcfg(T, U, **kw):
    kw.setdefault("v_rel", 1e300)
    return O.flowcfg(T0=T, U=U, gflow=True, **kw)


def _fermi(x, T):
    return 0.5 * (1.0 - np.tanh(x / (2 * T)))


def _chi(x, y, T):
    d = x - y
    same = np.abs(d) < 1e-12
    num = -(_fermi(x, T) - _fermi(y, T))
    fp = _fermi(x, T) * (1 - _fermi(x, T)) / T
    return np.where(same, fp, num / np.where(same, 1.0, d))


def _partner(L, m, pp):
    jy, jx = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    if pp:
        return (m[0] - jx - 1) % L, (m[1] - jy - 1) % L
    return (jx + m[0]) % L, (jy + m[1]) % L


def test_k_one_is_bitwise_z_only():
    N, L, T, U = 8, 16, 0.2, 2.0
    gs = np.linspace(0.0, 1.0, 5)
    ztab = np.array([[1.0 - 0.2 * g * (1 + 0.1 * (a % 3)) for a in range(N)] for g in gs])
    V0, _, _ = O.flow(O.model(N, L), gcfg(T, U, n_steps=30, z_lnT=gs, z_tab=ztab), U)
    V1, _, _ = O.flow(O.model(N, L), gcfg(T, U, n_steps=30, z_lnT=gs, z_tab=ztab,
                                          k_tab=np.ones((5, N))), U)
    assert np.abs(V0 - U).max() > 0.1
    assert np.array_equal(V0, V1)


def test_constant_k_scaling():
    N, L, T, g = 8, 16, 0.25, 0.6
    V = np.random.default_rng(5).standard_normal((N, N, N))
    Z = np.linspace(0.7, 0.95, N)
    d1 = O.rhs_g(O.model(N, L), T, g, V, Z=Z)
    dk = O.rhs_g(O.model(N, L), T, g, V, Z=Z, K=np.full(N, -0.35))
    assert np.abs(dk + 0.35 * d1).max() <= 1e-14 * np.abs(d1).max()
    # constant z and k: the flow of U equals the plain flow of k z^3 U, divided by k z^3
    U, z, k = 1.5, 0.8, 0.7
    gs = np.linspace(0.0, 1.0, 3)
    Vk, _, _ = O.flow(O.model(N, L), gcfg(0.15, U, n_steps=40, z_lnT=gs,
                                          z_tab=np.full((3, N), z), k_tab=np.full((3, N), k)), U)
    c = k * z ** 3
    V1, _, _ = O.flow(O.model(N, L), gcfg(0.15, c * U, n_steps=40), c * U)
    assert np.abs(Vk - U).max() > 0.05
    assert np.abs(Vk - V1 / c).max() <= 1e-12 * np.abs(Vk).max()


@pytest.mark.parametrize("channels", [7, 1, 2, 4])
def test_per_patch_k_against_brute_force(channels):
    N, L, T, g = 4, 8, 0.3, 0.7
    rng = np.random.default_rng(3)
    V = rng.standard_normal((N, N, N))
    Z = rng.uniform(0.6, 1.0, N)
    K = rng.uniform(-0.5, 1.5, N)
    d = brute.rhs(V, N, L, T, Z=Z, g=g, K=K, channels=channels)
    ref = np.array([[[d[(a, b, c)] for c in range(N)] for b in range(N)] for a in range(N)])
    got = O.rhs_g(O.model(N, L, channels=channels), T, g, V, Z=Z, K=K)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_tabulated_z_and_k_second_order():
    N, L, T, U = 8, 16, 0.25, 1e-6
    gs = np.linspace(0.0, 1.0, 6)
    ztab = np.array([[1.0 - 0.3 * g * (1.0 + 0.25 * (a % 3)) for a in range(N)] for g in gs])
    ktab = np.array([[1.0 - 1.2 * g * g * (1.0 + 0.2 * (a % 4)) for a in range(N)] for g in gs])
    V, _, _ = O.flow(O.model(N, L), gcfg(T, U, n_steps=60, z_lnT=gs, z_tab=ztab, k_tab=ktab),
                     U)
    xi, patch, anchor, _ = O.geometry(O.model(N, L))
    P, X = patch.reshape(L, L), xi.reshape(L, L)

    def integrand(g, m, pp):
        Z = np.array([np.interp(g, gs, ztab[:, a]) for a in range(N)])
        K = np.array([np.interp(g, gs, ktab[:, a]) for a in range(N)])
        px, py = _partner(L, m, pp)
        za, zb = Z[P], Z[P[py, px]]
        ka, kb = K[P], K[P[py, px]]
        y = -X[py, px] if pp else X[py, px]
        return np.mean(g * za * zb * (ka * za + kb * zb) * _chi(X, y, T))

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


def _k_closed(g, c):
    s = c * g ** 4
    return 1.0 + 3.0 * s, 8.0 * s / np.where(g > 0, g, 1.0) / (1.0 - s) * (g > 0)


def test_katanin_table_of_the_g4_law():
    """s_g = c g^4 (Z = 1/(1 - s)): K = 1 - s + g s' = 1 + 3 s and A = 2 s'/(1 - s)
    = 8 s/(g (1 - s)); the three-point derivative converges at second order."""
    c = np.array([0.05, 0.2, -0.1])
    errs = []
    for n in (11, 21, 41):
        g = np.linspace(0.0, 1.0, n)
        z = 1.0 / (1.0 - np.outer(g ** 4, c))
        K, A = O.katanin(g, z)
        eK = eA = 0.0
        for j, cj in enumerate(c):
            k_ref, a_ref = _k_closed(g, cj)
            eK = max(eK, np.abs(K[:, j] - k_ref).max())
            eA = max(eA, np.abs(A[:, j] - a_ref).max())    # A = 0 at g = 0
        errs.append((eK, eA))
    for (k0, a0), (k1, a1) in zip(errs, errs[1:]):
        assert 3.3 < k0 / k1 < 4.7 and 3.3 < a0 / a1 < 4.7, errs
    assert errs[-1][0] < 2e-3
    # non-uniform nodes: exact for a quadratic s
    g = np.array([0.0, 0.1, 0.35, 0.4, 0.8, 1.0])
    s = 0.1 + 0.3 * g - 0.25 * g * g
    K, A = O.katanin(g, (1.0 / (1.0 - s))[:, None])
    ds = 0.3 - 0.5 * g
    assert np.abs(K[:, 0] - (1.0 - s + g * ds)).max() <= 1e-14
    assert np.abs(A[1:, 0] - 2.0 * ds[1:] / (1.0 - s[1:])).max() <= 1e-13
    # the two forms of A agree: -(2/g)(1 - Z K) = 2 (dZ/dg)/Z
    Z = 1.0 / (1.0 - s)
    assert np.abs(A[1:, 0] + (2.0 / g[1:]) * (1.0 - Z[1:] * K[1:, 0])).max() <= 1e-13


def test_katanin_from_the_second_order_self_energy():
    """Z_g of second-order perturbation theory at scale g: g Sigma_g = Sigma^(2)[g^2 U], whose
    Re Sigma is U_eff^2 times a fixed function, so s_g = g^4 s_1 exactly and K, A are those of
    the g^4 law with the oracle's own s_1."""
    N, L, T, U = 8, 16, 0.3, 2.0
    g = np.linspace(0.25, 1.0, 7)
    z = np.stack([O.sigma2(O.model(N, L), T, gi * gi * U, n_w=512)[3] for gi in g])
    s1 = 1.0 - 1.0 / O.sigma2(O.model(N, L), T, U, n_w=512)[3]
    zlaw = 1.0 / (1.0 - np.outer(g ** 4, s1))
    assert np.abs(z - zlaw).max() <= 1e-12
    K, A = O.katanin(g, z)
    Kl, Al = O.katanin(g, zlaw)
    assert np.abs(K - Kl).max() <= 1e-10 and np.abs(A - Al).max() <= 1e-9
    assert (K < 1.0).all() and (K > 0.0).all()      # s < 0 near the Fermi level: K < 1


def test_katanin_needs_the_interaction_flow():
    N, L = 4, 8
    gs = np.linspace(0.0, 1.0, 3)
    cfg = O.flowcfg(T0=1.0, T_end=0.1, U=1.0, z_lnT=np.log([0.1, 0.3, 1.0]),
                    z_tab=np.ones((3, N)), k_tab=np.ones((3, N)))
    with pytest.raises(ValueError):
        O.flow(O.model(N, L), cfg, 1.0)
    cfg = gcfg(0.2, 1.0, k_tab=np.ones((3, N)))       # no Z table: no nodes for K
    with pytest.raises(ValueError):
        O.flow(O.model(N, L), cfg, 1.0)
    with pytest.raises(ValueError):
        O.katanin(gs[:2], np.ones((2, N)))
