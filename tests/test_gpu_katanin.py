"""GPU parity of the Katanin correction of the interaction flow (App. A, Step 3) through the C
ABI against the oracle: dV/dg with Z and Katanin tables (the single-scale line K Z^2 G0,
Eq. vertex_flow_feedback_Z_with_Katanin) in every precision, a whole RK4 flow in double
precision, and the chain Z of second-order perturbation theory at scale g (fm_flow_z at the
coupling g^2 U) -> K and A_g (fm_katanin_table, Eqs. K_definition and A_g_simple) -> the
flow, each side from its own tables.  Tolerances as for the interaction flow: 1e-10 double
precision, 1e-4 single precision and split bf16, 1e-2 bf16."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2005_00827_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp64_direct": 1e-10, "fp32": 1e-4, "bf16": 1e-2, "bf16x3": 1e-4}


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    return torch, torch.device("cuda:0")


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def tables(N, n=6):
    """Z falling with g, K falling through zero for some patches (K may change sign)."""
    gs = np.linspace(0.0, 1.0, n)
    z = np.array([[1.0 - 0.3 * g * (1.0 + 0.25 * (a % 3)) for a in range(N)] for g in gs])
    k = np.array([[1.0 - 1.4 * g * g * (1.0 + 0.2 * (a % 4)) for a in range(N)] for g in gs])
    return gs, z, k


def interp(g, gs, tab):
    return np.array([np.interp(g, gs, tab[:, a]) for a in range(tab.shape[1])])


@pytest.mark.parametrize("prec,y_kernel", [("fp64", 0), ("fp64_direct", 0), ("fp32", 0),
                                           ("bf16", 3), ("bf16x3", 3), ("bf16", 4), ("bf16x3", 4)])
def test_rhs_g_with_katanin_table(torch_dev, prec, y_kernel):
    """y_kernel 3: phase 2 on the orbit kernel and phase 2b; 4: the fused phase 2."""
    from paper_2005_00827_amd import fm
    torch, dev = torch_dev
    N, L, U = 16, 32, 2.5
    gs, z, k = tables(N)
    V = np.stack([inputs.noisy_state(N, U, seed=1), inputs.noisy_state(N, U, seed=2)])
    T, g = [0.3, 0.05], [0.35, 0.9]
    f = fm.Flow(N=N, L=L, precision=prec, flow="interaction", T0=0.3, max_batch=2,
                z_lnT=gs, z_table=z, k_table=k, y_kernel=y_kernel, device=dev)
    try:
        got = f.rhs_g(T, g, torch.from_numpy(V).to(dev)).cpu().numpy()
    finally:
        f.close()
    for i in range(2):
        ref = O.rhs_g(O.model(N, L), T[i], g[i], V[i], Z=interp(g[i], gs, z),
                      K=interp(g[i], gs, k))
        assert rel(got[i], ref) <= TOL[prec], (i, rel(got[i], ref))
        plain = O.rhs_g(O.model(N, L), T[i], g[i], V[i], Z=interp(g[i], gs, z))
        assert rel(plain, ref) > 3 * TOL[prec]        # the factors matter at this tolerance


def test_katanin_rk4_flow_fp64(torch_dev):
    from paper_2005_00827_amd import fm
    torch, dev = torch_dev
    N, L, U, T = 16, 32, 2.5, 0.1
    gs, z, k = tables(N)
    f = fm.Flow(N=N, L=L, U=U, T0=T, precision="fp64", integrator="rk4", n_steps=60,
                flow="interaction", z_lnT=gs, z_table=z, k_table=k, device=dev)
    try:
        res, Vg = f.run_batch([U], [T], return_V=True)
        with pytest.raises(fm.FmError):        # per-flow Z tables cannot carry K
            f.run_batch([U], [T], z_lnT=gs[None], z_tables=z[None])
    finally:
        f.close()
    cfg = O.flowcfg(T0=T, U=U, n_steps=60, gflow=True, z_lnT=gs, z_tab=z, k_tab=k)
    Vo, ores, _ = O.flow(O.model(N, L), cfg, U)
    r = res[0]
    assert r["status"] == ores["status"] and r["n_accepted"] == ores["n_accepted"]
    if ores["status"] == O.DIVERGED:
        assert abs(r["g_c"] / ores["g_c"] - 1) <= 1e-9
    assert rel(Vg.cpu().numpy()[0], Vo) <= 1e-10


def test_katanin_chain_from_second_order_self_energy(torch_dev):
    """Z_g at the nodes g from fm_flow_z at the coupling g^2 U (g Sigma_g = Sigma^(2)[g^2 U]),
    K and A from fm_katanin_table, then a Dormand-Prince interaction flow with both tables;
    the oracle does the same with O.sigma2, O.katanin and O.flow.  Tables agree to 1e-9
    (Re Sigma to 1e-10, then differences of neighbouring nodes), the outcome and max|V| at the
    end to 1e-8.  Here K < 1 slows the flow enough that it reaches g = 1 (max|V| about 22 U/3)
    where the same flow without K diverges near g = 0.94: the saturation the correction can
    bring about."""
    from paper_2005_00827_amd import fm
    torch, dev = torch_dev
    N, L, U, T = 16, 32, 3.0, 0.15
    gs = np.linspace(0.2, 1.0, 9)
    h = fm.Flow(N=N, L=L, device=dev)
    try:
        z = np.stack([h.z(T, g * g * U) for g in gs])
    finally:
        h.close()
    oz = np.stack([O.sigma2(O.model(N, L), T, g * g * U, n_w=fm.SIGMA_NW)[3] for g in gs])
    assert np.abs(z - oz).max() <= 1e-10
    K, A, mm = fm.katanin_table(gs, z)
    oK, oA = O.katanin(gs, oz)
    assert np.abs(K - oK).max() <= 1e-9 and np.abs(A - oA).max() <= 1e-8
    assert np.array_equal(mm[:, 0], A.min(axis=1)) and np.array_equal(mm[:, 1], A.max(axis=1))
    assert (K < 1.0).all()
    f = fm.Flow(N=N, L=L, U=U, T0=T, precision="fp64", integrator="rk45", flow="interaction",
                v_rel=20.0, z_lnT=gs, z_table=z, k_table=K, device=dev)
    try:
        res = f.run_batch([U], [T])[0]
    finally:
        f.close()
    cfg = O.flowcfg(T0=T, U=U, integrator=1, gflow=True, v_rel=20.0, z_lnT=gs, z_tab=oz,
                    k_tab=oK)
    _, ores, _ = O.flow(O.model(N, L), cfg, U)
    assert res["status"] == ores["status"]
    if ores["status"] == O.DIVERGED:
        assert abs(res["g_c"] / ores["g_c"] - 1.0) <= 1e-8
    assert res["max_abs_V"] == pytest.approx(ores["max_abs_V"], rel=1e-8)
    # without K the same flow diverges, and earlier
    cfg0 = O.flowcfg(T0=T, U=U, integrator=1, gflow=True, v_rel=20.0, z_lnT=gs, z_tab=oz)
    _, o0, _ = O.flow(O.model(N, L), cfg0, U)
    assert o0["status"] == O.DIVERGED
    assert ores["status"] != O.DIVERGED or o0["g_c"] < ores["g_c"]
