"""Host-side checks of the C-ABI library that need no GPU: it loads, exports every entry
point of include/fm_flow.h, validates configurations, and its host geometry (written
independently of the oracle) agrees with the oracle's."""
import re
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2005_00827_amd import fm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    lib = fm.load()
    hdr = open(os.path.join(ROOT, "include", "fm_flow.h")).read()
    declared = set(re.findall(r"\b(fm_[a-z_]+)\s*\(", hdr))
    assert declared == set(fm.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("N,L,identity,tp,mu", [(16, 32, False, 0, 0), (48, 128, False, 0, 0),
                                                (96, 256, False, 0, 0), (4, 16, False, 0, 0),
                                                (8, 16, False, -0.3, -0.4), (1, 32, False, 0, 0),
                                                (16, 4, True, 0, 0), (36, 6, True, 0, 0)])
def test_geometry_matches_oracle(N, L, identity, tp, mu):
    cfg = fm.make_config(N, L, tp=tp, mu=mu, geometry="identity" if identity else "angular")
    xi, patch, anchor, npp, nph, margin = fm.geometry_query(cfg)
    oxi, opatch, oanchor, omargin = O.geometry(O.model(N, L, tp=tp, mu=mu, identity=identity))
    assert np.array_equal(patch, opatch)
    assert np.array_equal(anchor, oanchor)
    assert np.abs(xi - oxi).max() <= 1e-15
    assert (npp, nph) == O.transfer_counts(O.model(N, L, tp=tp, mu=mu, identity=identity))
    if not identity:
        assert margin == pytest.approx(omargin, rel=1e-9)


@pytest.mark.parametrize("N,L,S,edges,tp,mu", [(24, 32, 3, None, 0, 0), (40, 32, 5, [0.3, 1.1], 0, 0),
                                               (224, 128, 7, None, 0, 0),
                                               (24, 32, 3, None, -0.3, -0.4)])
def test_shell_geometry_matches_oracle(N, L, S, edges, tp, mu):
    """Energy shells: the library's host geometry (written independently) equals the
    oracle's bit for bit; the point group still reduces the transfers (empty patches of a
    sector the band does not reach permute with their sector)."""
    cfg = fm.make_config(N, L, tp=tp, mu=mu, geometry="shells", n_shells=S, shell_edges=edges)
    xi, patch, anchor, npp, nph, margin = fm.geometry_query(cfg)
    m = O.model(N, L, tp=tp, mu=mu, n_shells=S, shell_edges=edges)
    oxi, opatch, oanchor, omargin = O.geometry(m)
    assert np.array_equal(patch, opatch)
    assert np.array_equal(anchor, oanchor)
    assert np.abs(xi - oxi).max() <= 1e-15
    assert (npp, nph) == O.transfer_counts(m)
    nrp, nrd = fm.representative_counts(cfg)
    if tp == 0 and mu == 0:
        assert nrp < npp / 4 and nrd < nph / 4


def test_transfer_counts_of_the_workloads():
    for (N, L), n in {(16, 32): 48, (48, 128): 424, (96, 256): 1520, (128, 512): 2856}.items():
        _, _, _, npp, nph, _ = fm.geometry_query(fm.make_config(N, L))
        assert npp == nph == n


def _orbit_count(ms, L):
    """Orbits of transfer indices (mx, my) mod L under the square's point group: sign flips
    of either axis and the axis swap act on the unshifted transfer grid as m -> -m and
    (mx, my) -> (my, mx), for particle-particle and particle-hole transfers alike."""
    def canon(m):
        mx, my = m
        return min(((sx * a) % L, (sy * b) % L) for a, b in ((mx, my), (my, mx))
                   for sx in (1, -1) for sy in (1, -1))
    return len({canon(m) for m in ms})


@pytest.mark.parametrize("N,L,tp,mu", [(16, 32, 0, 0), (48, 128, 0, 0), (8, 16, -0.3, -0.4),
                                       (96, 256, 0, 0)])
def test_representative_counts_are_point_group_orbits(N, L, tp, mu):
    _, _, anchor, _ = O.geometry(O.model(N, L, tp=tp, mu=mu))
    a = np.asarray(anchor).reshape(N, 2)
    qpp = {((a[x, 0] + a[y, 0]) % L, (a[x, 1] + a[y, 1]) % L) for x in range(N) for y in range(N)}
    qph = {((a[y, 0] - a[x, 0]) % L, (a[y, 1] - a[x, 1]) % L) for x in range(N) for y in range(N)}
    nrp, nrd = fm.representative_counts(fm.make_config(N, L, tp=tp, mu=mu))
    assert (nrp, nrd) == (_orbit_count(qpp, L), _orbit_count(qph, L))


@pytest.mark.parametrize("kw,msg", [
    (dict(N=12, L=32), "N %"),                 # N % 8 == 4 is fine; 12 % 8 == 4 -> ok, so use 10
    (dict(N=10, L=32), "angular geometry"),
    (dict(N=16, L=30), "L % 4"),
    (dict(N=16, L=32, T0=0.01, T_end=1.0), "T0 > T_end"),
    (dict(N=16, L=32, integrator="rk4", n_steps=0), "n_steps"),
    (dict(N=16, L=32, max_batch=0), "max_batch"),
    (dict(N=17, L=4, geometry="identity"), "identity"),
    (dict(N=16, L=32, channels=9), "channel"),
    (dict(N=16, L=32, tile_rows=-1), "tile_rows"),
    (dict(N=16, L=32, flow=2), "bad flow"),
    (dict(N=16, L=32, y_kernel=5), "y_kernel"),
    (dict(N=16, L=32, phase1_variant=5), "phase1_variant"),
    (dict(N=16, L=32, y_kernel=4), "fused phase 2"),          # needs bf16 products
    (dict(N=136, L=128, precision="bf16x3", y_kernel=4), "N <= 128"),
    (dict(N=16, L=32, flow="interaction", T0=0.0), "T0 > 0"),
    (dict(N=16, L=32, flow="interaction", T0=0.2, g_end=-1.0), "g_end"),
    (dict(N=136, L=128, precision="bf16"), "N <= 128"),
    (dict(N=24, L=32, geometry="shells", n_shells=2), "odd n_shells"),
    (dict(N=24, L=32, geometry="shells", n_shells=5), "odd n_shells"),
    (dict(N=24, L=32, geometry="shells", n_shells=3, shell_edges=[-0.5]), "shell edges"),
    (dict(N=136, L=128, precision="bf16x3"), "N <= 128"),
    (dict(N=16, L=32, sym_state=2), "sym_state must be 0 or 1"),
    (dict(N=16, L=32, precision="fp64_direct", sym_state=1), "product buffers"),
    (dict(N=16, L=32, precision="fp32", y_kernel=1, sym_state=1), "product buffers"),
    (dict(N=16, L=32, precision="fp32", z_lnT=[0.0, 1.0],
          z_table=[[1.0 - 0.01 * a for a in range(16)]] * 2, sym_state=1), "invariant"),
])
def test_invalid_configs_rejected(kw, msg):
    cfg = fm.make_config(**kw)
    if kw.get("N") == 12:
        assert fm.workspace_bytes(cfg) > 0
        return
    with pytest.raises(fm.FmError) as e:
        fm.workspace_bytes(cfg)
    assert e.value.code == fm.FM_EINVAL
    assert msg in str(e.value)


def test_workspace_scales_with_batch():
    a = fm.workspace_bytes(fm.make_config(48, 128, precision="fp32", max_batch=1))
    b = fm.workspace_bytes(fm.make_config(48, 128, precision="fp32", max_batch=4))
    assert 3.5 * a < b < 4.5 * a


def test_interaction_flow_config_and_workspace():
    """The interaction flow ignores T_end and bins one temperature per flow (one bin set),
    the temperature flow's Dormand-Prince steps five stage nodes."""
    g = fm.make_config(48, 128, precision="fp32", flow="interaction", T0=0.1, T_end=0.0,
                       integrator="rk45")
    t = fm.make_config(48, 128, precision="fp32", integrator="rk45")
    nRp, nRd = fm.representative_counts(t)
    bin_set = (nRp + 2 * nRd) * 48 * 48 * 4
    assert fm.workspace_bytes(t) - fm.workspace_bytes(g) >= 4 * bin_set


def test_katanin_table_matches_the_oracle():
    """fm_katanin_table is host code: K, A_g and the per-node bounds of A against the
    oracle's table on non-uniform nodes (App. A, Eqs. K_definition and A_g_simple)."""
    rng = np.random.default_rng(8)
    g = np.array([0.0, 0.07, 0.2, 0.33, 0.5, 0.61, 0.8, 1.0])
    z = rng.uniform(0.5, 1.3, (g.size, 12))
    K, A, mm = fm.katanin_table(g, z)
    oK, oA = O.katanin(g, z)
    assert np.abs(K - oK).max() <= 1e-13 * np.abs(oK).max()
    assert np.abs(A - oA).max() <= 1e-12 * np.abs(oA).max()
    assert np.array_equal(mm[:, 0], A.min(axis=1)) and np.array_equal(mm[:, 1], A.max(axis=1))
    for bad in (dict(g=g[:2], z=z[:2]), dict(g=g[::-1], z=z),
                dict(g=g, z=np.where(np.arange(12) == 3, 0.0, z))):
        with pytest.raises(fm.FmError):
            fm.katanin_table(bad["g"], bad["z"])


def test_katanin_table_needs_the_interaction_flow():
    gs = np.linspace(0.0, 1.0, 4)
    z = np.full((4, 8), 0.9)
    ok = fm.make_config(8, 16, flow="interaction", T0=0.2, z_lnT=gs, z_table=z,
                        k_table=np.full((4, 8), 0.7))
    assert fm.workspace_bytes(ok) > 0
    for cfg in (fm.make_config(8, 16, z_lnT=np.log([0.01, 0.1, 0.5, 1.0]), z_table=z,
                               k_table=np.full((4, 8), 0.7)),
                fm.make_config(8, 16, flow="interaction", T0=0.2, z_lnT=gs, z_table=z,
                               k_table=np.full((4, 8), np.inf))):
        with pytest.raises(fm.FmError):
            fm.workspace_bytes(cfg)


def test_fused_phase2_workspace_holds_no_products():
    """y_kernel 4 runs phase 2 as one fused kernel: the workspace drops the product buffers,
    (nP + 3 nD) N^2 values per flow, stored as bf16 for bf16 products and f32 otherwise."""
    for prec, ys in (("bf16", 2), ("bf16x3", 4)):
        two = fm.make_config(48, 64, precision=prec, y_kernel=3, max_batch=2)
        one = fm.make_config(48, 64, precision=prec, y_kernel=4, max_batch=2)
        _, _, _, nP, nD, _ = fm.geometry_query(two)
        saved = fm.workspace_bytes(two) - fm.workspace_bytes(one)
        want = 2 * (nP + 3 * nD) * 48 * 48 * ys
        assert want <= saved <= want + 4 * 256
