"""GPU parity: the HIP path through the C ABI against the double-precision CPU oracle.

Tolerances (relative to max|reference|): 1e-10 for the double-precision paths, 1e-4 for
single precision and for split-bf16 products, 1e-2 for bf16 products; T_c to 1e-3 relative.  Inputs are seeded and synthetic
(paper_2005_00827_amd.inputs); expected values come only from the oracle.
"""
import math

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


def _fm():
    from paper_2005_00827_amd import fm
    return fm


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def gpu_rhs(torch_dev, N, L, T, V, prec, **kw):
    torch, dev = torch_dev
    fm = _fm()
    V = np.asarray(V, np.float64).reshape(-1, N, N, N)
    f = fm.Flow(N=N, L=L, precision=prec, max_batch=V.shape[0], device=dev, **kw)
    try:
        out = f.rhs(np.atleast_1d(T), torch.from_numpy(V).to(dev))
        torch.cuda.synchronize()
        return out.cpu().numpy()
    finally:
        f.close()


def oracle_model(N, L, **kw):
    return O.model(N, L, t=kw.get("t", 1.0), tp=kw.get("tp", 0.0), mu=kw.get("mu", 0.0),
                   identity=kw.get("geometry") == "identity",
                   channels=kw.get("channels", O.CH_ALL))


RHS_CASES = [
    # N, L, T, state, extra
    (16, 32, 1.0, "s0", {}),
    (16, 32, 0.2, "s1", {}),
    (16, 32, 0.01, "s1", {}),
    (16, 32, 0.05, "rand", {"channels": 1}),
    (16, 32, 0.05, "rand", {"channels": 2}),
    (16, 32, 0.05, "rand", {"channels": 4}),
    (4, 16, 0.1, "s1", {}),
    (1, 32, 0.3, "s1", {}),
    (8, 16, 0.2, "rand", {"tp": -0.3, "mu": -0.4}),
    (16, 4, 0.3, "rand", {"geometry": "identity"}),
    (36, 6, 0.1, "rand", {"geometry": "identity"}),
    (24, 20, 0.07, "s1", {}),      # ragged: N not a tile multiple, L not a power of two
]


def make_state(kind, N, U=2.0, seed=inputs.SEED):
    if kind == "s0":
        return inputs.constant_state(N, U)
    if kind == "s1":
        return inputs.noisy_state(N, U, seed=seed)
    return inputs.random_state(N, seed=seed)


@pytest.mark.parametrize("prec", ["fp64", "fp64_direct", "fp32", "bf16", "bf16x3"])
@pytest.mark.parametrize("N,L,T,state,kw", RHS_CASES)
def test_rhs_small(torch_dev, prec, N, L, T, state, kw):
    V = make_state(state, N)
    ref = O.rhs(oracle_model(N, L, **kw), T, V)
    got = gpu_rhs(torch_dev, N, L, T, V, prec, **kw)[0]
    if np.abs(ref).max() < 1e-13:   # the direct channel alone vanishes for constant V
        assert np.abs(got).max() < 1e-12
        return
    assert rel(got, ref) <= TOL[prec], (prec, N, L, T, state, kw, rel(got, ref))


@pytest.mark.parametrize("prec", ["fp32", "bf16", "bf16x3"])
@pytest.mark.parametrize("N,L,T,state,kw", RHS_CASES)
def test_rhs_small_orbit_kernel(torch_dev, prec, N, L, T, state, kw):
    """The orbit phase-2a kernel forced on every small case: N = 1 (stores one value at a
    time), identity geometries (every operation set trivial), channel subsets, ragged N."""
    V = make_state(state, N)
    ref = O.rhs(oracle_model(N, L, **kw), T, V)
    got = gpu_rhs(torch_dev, N, L, T, V, prec, y_kernel=3, **kw)[0]
    if np.abs(ref).max() < 1e-13:
        assert np.abs(got).max() < 1e-12
        return
    assert rel(got, ref) <= TOL[prec], (prec, N, L, T, state, kw, rel(got, ref))


@pytest.mark.parametrize("y_kernel", [1, 2, 3])
@pytest.mark.parametrize("tile_rows", [1, 2, 3, 100])
@pytest.mark.parametrize("prec", ["fp32", "bf16", "bf16x3"])
@pytest.mark.parametrize("N,L", [(32, 64), (48, 64), (20, 16)])
def test_rhs_every_phase2a_tile_choice(torch_dev, prec, tile_rows, y_kernel, N, L):
    """The three matrix-core kernels (per-row gathers; operation classes; orbits) at every
    row-tile count per wavefront, up to all of a group's or class's tiles (100 is clamped),
    give the oracle's RHS: 12 and more transfer tiles, so runs of 2 and 3 tiles end ragged,
    classes of uneven size, representatives with fewer than eight operations, and N = 20
    (not a multiple of 8) for the rows read past their end."""
    V = inputs.noisy_state(N, 2.5)
    ref = O.rhs(O.model(N, L), 0.09, V)
    got = gpu_rhs(torch_dev, N, L, 0.09, V, prec, tile_rows=tile_rows, y_kernel=y_kernel)[0]
    assert rel(got, ref) <= TOL[prec]


@pytest.mark.parametrize("prec", ["bf16", "bf16x3"])
@pytest.mark.parametrize("N,L,channels", [(16, 32, 7), (20, 16, 7), (32, 64, 7), (48, 64, 7),
                                          (64, 64, 7), (96, 32, 7), (32, 64, 1), (32, 64, 2),
                                          (32, 64, 4), (32, 64, 6)])
def test_rhs_fused_phase2(torch_dev, prec, N, L, channels):
    """Phase 2 as one fused launch (products and contraction, no product buffers), forced
    with y_kernel 4: every N from one 16-column tile to 96 (every column-tile and k-step
    count of the kernel), every channel alone and together (channels switched off write
    zeros), two states at two temperatures with a Z table."""
    lnT, tab = inputs.synthetic_z_table(N, 2.5, 1.0, 0.01)
    V = np.stack([inputs.noisy_state(N, 2.5, seed=5), inputs.noisy_state(N, 2.0, seed=6)])
    T = [0.3, 0.06]
    got = gpu_rhs(torch_dev, N, L, T, V, prec, y_kernel=4, channels=channels, z_lnT=lnT,
                  z_table=tab)
    for i in range(2):
        Z = np.array([np.interp(math.log(T[i]), lnT, tab[:, a]) for a in range(N)])
        ref = O.rhs(O.model(N, L, channels=channels), T[i], V[i], Z=Z)
        assert rel(got[i], ref) <= TOL[prec], (i, rel(got[i], ref))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_rhs_with_z_table_and_batch(torch_dev, prec):
    """Two states at two temperatures in one batch, Z interpolated from a table."""
    N, L, U = 16, 32, 3.0
    lnT, tab = inputs.synthetic_z_table(N, U, 1.0, 0.01)
    V = np.stack([inputs.noisy_state(N, U, seed=1), inputs.noisy_state(N, U, seed=2)])
    T = [0.5, 0.037]
    got = gpu_rhs(torch_dev, N, L, T, V, prec, z_lnT=lnT, z_table=tab)
    for i in range(2):
        Z = np.array([np.interp(math.log(T[i]), lnT, tab[:, a]) for a in range(N)])
        ref = O.rhs(O.model(N, L), T[i], V[i], Z=Z)
        assert rel(got[i], ref) <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16", "bf16x3"])
def test_rhs_c2_full(torch_dev, prec):
    """N = 48, L = 128 (the quasi-particle workload's size): every output element."""
    N, L, U = 48, 128, 3.0
    lnT, tab = inputs.synthetic_z_table(N, U, 1.0, 0.01)
    T = 0.11
    Z = np.array([np.interp(math.log(T), lnT, tab[:, a]) for a in range(N)])
    V = inputs.noisy_state(N, U)
    ref = O.rhs(O.model(N, L), T, V, Z=Z)
    got = gpu_rhs(torch_dev, N, L, T, V, prec, z_lnT=lnT, z_table=tab)[0]
    assert rel(got, ref) <= TOL[prec]


@pytest.mark.parametrize("N,L", [(96, 256), (128, 512)])
@pytest.mark.parametrize("prec,y_kernel", [("fp64", 0), ("fp32", 1), ("fp32", 2), ("fp32", 3),
                                           ("bf16", 1), ("bf16", 2), ("bf16", 3), ("bf16", 4),
                                           ("bf16x3", 1), ("bf16x3", 2), ("bf16x3", 3),
                                           ("bf16x3", 4)])
def test_rhs_large_sampled(torch_dev, N, L, prec, y_kernel):
    """Full-size grids: sampled outputs against the oracle's per-element sums, with each
    matrix-core phase-2a kernel."""
    V = inputs.noisy_state(N, 3.0)
    T = 0.08
    abc = inputs.sample_indices(N, 48)
    ref = O.rhs_points(O.model(N, L), T, V, abc)
    got = gpu_rhs(torch_dev, N, L, T, V, prec, y_kernel=y_kernel)[0]
    g = got[abc[:, 0], abc[:, 1], abc[:, 2]]
    # relative to the largest sampled reference value
    assert rel(g, ref) <= TOL[prec]
    # property at every element: C4v relabelling a -> a + N/4 leaves the RHS of a
    # C4v-symmetric state invariant (checked on the constant state)
    if prec == "fp64" and N == 96:
        V0 = inputs.constant_state(N, 3.0)
        d = gpu_rhs(torch_dev, N, L, T, V0, prec)[0]
        r = (np.arange(N) + N // 4) % N
        assert rel(d[np.ix_(r, r, r)], d) <= 1e-12


@pytest.mark.parametrize("N,L,prec", [(136, 128, "fp64"), (136, 128, "fp32"),
                                      (264, 64, "fp64_direct")])
def test_rhs_above_128_patches_sampled(torch_dev, N, L, prec):
    """More than 128 patches: phase 2b gathers its pair vectors in several rounds, FP32
    phase 2a runs on the vector units, and the direct kernel loops its threads over the
    outgoing patch (264 > 256 threads per block).  Sampled outputs against the oracle; bf16
    modes reject this size."""
    fm = _fm()
    V = inputs.noisy_state(N, 3.0)
    T = 0.08
    abc = inputs.sample_indices(N, 48)
    ref = O.rhs_points(O.model(N, L), T, V, abc)
    got = gpu_rhs(torch_dev, N, L, T, V, prec)[0]
    assert rel(got[abc[:, 0], abc[:, 1], abc[:, 2]], ref) <= TOL[prec]
    with pytest.raises(fm.FmError):
        fm.Flow(N=N, L=L, precision="bf16", device=torch_dev[1])


@pytest.mark.parametrize("integrator", ["rk4", "rk45"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_step_matches_oracle(torch_dev, integrator, prec):
    torch, dev = torch_dev
    fm = _fm()
    N, L, U = 16, 32, 2.0
    V = inputs.noisy_state(N, U)
    f = fm.Flow(N=N, L=L, U=U, precision=prec, integrator=integrator, device=dev)
    cfg = O.flowcfg(U=U, integrator=1 if integrator == "rk45" else 0)
    try:
        lnT, h = math.log(0.3), -0.05
        Vd = torch.from_numpy(V.reshape(1, N, N, N).copy()).to(dev)
        lnT2, h2, acc = f.step([lnT], [h], Vd)
        ol, oh, oV, oacc, oerr = O.step(O.model(N, L), cfg, lnT, h, V)
        assert bool(acc[0]) == oacc
        assert lnT2[0] == pytest.approx(ol, abs=1e-14)
        if integrator == "rk45" and prec == "fp64":
            assert h2[0] == pytest.approx(oh, rel=1e-9)
        elif integrator == "rk45":
            # the embedded error estimate of a single-precision RHS is set by its rounding,
            # so only the step-size rule's bounds are comparable
            assert 0.2 * abs(h) - 1e-15 <= abs(h2[0]) <= 5 * abs(h) + 1e-15
        assert rel(Vd.cpu().numpy()[0], oV) <= TOL[prec]
    finally:
        f.close()


@pytest.mark.parametrize("prec,integ,check", [("fp64", "rk45", "all"), ("fp32", "rk45", "ends"),
                                              ("fp64", "rk4", "ends")])
def test_stage_wide_tiles_ragged_batch(torch_dev, prec, integ, check):
    """Eight flows at N = 36 have 216 stage tiles of 16 x 16 x 16 between them, so the later
    stages of a step form the stage argument and its transposed layouts in 16-wide tiles, with
    ragged edges (36 = 2 * 16 + 4) in all three directions; the k slots' crossed and direct
    parts reach V order through the same tiles in the stage, RK4 update and error-norm
    kernels.  Each checked flow's step must match the oracle's (FP64: 1e-10, FP32: 1e-4);
    "ends" checks the first and last flow of the batch."""
    torch, dev = torch_dev
    fm = _fm()
    N, L = 36, 32
    Us = [1.0 + 0.25 * i for i in range(8)]
    V = np.stack([inputs.noisy_state(N, u, seed=31 + i) for i, u in enumerate(Us)])
    lnT, h = math.log(0.2), -0.02
    f = fm.Flow(N=N, L=L, U=Us[0], precision=prec, integrator=integ, max_batch=len(Us),
                device=dev)
    m = O.model(N, L)
    try:
        Vb = torch.from_numpy(V.copy()).to(dev)
        lb, hb, ab = f.step([lnT] * len(Us), [h] * len(Us), Vb)
        got = Vb.cpu().numpy()
        for i in (range(len(Us)) if check == "all" else (0, len(Us) - 1)):
            cfg = O.flowcfg(U=Us[i], integrator=1 if integ == "rk45" else 0)
            ol, oh, oV, oacc, _ = O.step(m, cfg, lnT, h, V[i])
            assert bool(ab[i]) == bool(oacc)
            if prec == "fp64":
                assert hb[i] == pytest.approx(oh, rel=1e-9)
            assert rel(got[i], oV) <= TOL[prec], (i, rel(got[i], oV))
    finally:
        f.close()


def test_rk45_rejects_a_too_large_step(torch_dev):
    torch, dev = torch_dev
    fm = _fm()
    N, L, U = 16, 32, 2.0
    V = inputs.noisy_state(N, U)
    f = fm.Flow(N=N, L=L, U=U, precision="fp64", integrator="rk45", device=dev)
    cfg = O.flowcfg(U=U, integrator=1)
    try:
        Vd = torch.from_numpy(V.reshape(1, N, N, N).copy()).to(dev)
        lnT2, h2, acc = f.step([math.log(0.1)], [-1.5], Vd)
        ol, oh, oV, oacc, oerr = O.step(O.model(N, L), cfg, math.log(0.1), -1.5, V)
        assert not oacc and not acc[0]
        assert h2[0] == pytest.approx(oh, rel=1e-9)
        assert np.array_equal(Vd.cpu().numpy()[0], V)   # rejected: state untouched
    finally:
        f.close()


def test_c1_flow_fp64(torch_dev):
    """The plain workload: N = 16, L = 32, U = 2, RK4 with 200 steps from T = 1 to 0.01."""
    fm = _fm()
    torch, dev = torch_dev
    N, L, U = 16, 32, 2.0
    f = fm.Flow(N=N, L=L, U=U, precision="fp64", integrator="rk4", n_steps=200, device=dev)
    try:
        res, Vg = f.run_batch([U], [1.0], return_V=True)
    finally:
        f.close()
    Vo, ores, _ = O.flow(O.model(N, L), O.flowcfg(U=U), U)
    r = res[0]
    assert r["status"] == ores["status"] == fm.DIVERGED
    assert (r["n_accepted"], r["n_rhs"]) == (ores["n_accepted"], ores["n_rhs"])
    assert r["T_c"] == pytest.approx(ores["T_c"], rel=1e-3)
    assert abs(r["T_c"] / ores["T_c"] - 1) <= 1e-9
    assert rel(Vg.cpu().numpy()[0], Vo) <= 1e-10


# Final states of independently adaptive FP64 flows.  Two correct implementations that sum
# the right-hand side in different orders (about 1e-15 apart per evaluation) move the
# proposed steps through the tiny error estimate, so the schedules drift apart by ~1e-9 in
# ln T and the states at the divergence by up to 1.05e-10: measured on the oracle alone,
# direct against binned summation (tests/test_oracle_dopri.py,
# test_rounding_order_amplification_of_adaptive_flows).  The final state is held to ten times
# that; the per-step comparison on one replayed schedule (test_rk45_schedule_replay_fp64)
# holds the FP64 path to 1e-10.
ADAPTIVE_FINAL_FP64 = 1e-9


@pytest.mark.parametrize("prec,tol", [("fp64", ADAPTIVE_FINAL_FP64), ("fp32", 1e-3),
                                      ("bf16", None), ("bf16x3", None)])
def test_rk45_batch_ragged(torch_dev, prec, tol):
    """Three flows in one launch: diverging at different temperatures and one reaching T_end."""
    fm = _fm()
    torch, dev = torch_dev
    N, L = 16, 32
    U = [2.5, 1.5, 0.4]
    T0 = [1.0, 0.7, 1.0]
    f = fm.Flow(N=N, L=L, U=2.0, precision=prec, integrator="rk45", max_batch=4, device=dev)
    try:
        res, Vg = f.run_batch(U, T0, return_V=True)
    finally:
        f.close()
    Vg = Vg.cpu().numpy()
    for i in range(3):
        cfg = O.flowcfg(T0=T0[i], U=U[i], integrator=1)
        Vo, ores, _ = O.flow(O.model(N, L), cfg, U[i])
        assert res[i]["status"] == ores["status"], (i, res[i], ores)
        if ores["status"] == O.DIVERGED:
            assert res[i]["T_c"] == pytest.approx(ores["T_c"], rel=1e-3)
        if prec == "fp64":
            assert (res[i]["n_accepted"], res[i]["n_rejected"]) == (ores["n_accepted"], ores["n_rejected"])
            assert rel(Vg[i], Vo) <= tol
    assert res[2]["status"] == O.REACHED_TEND


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rk45_rejections_in_a_batch(torch_dev, prec):
    """A first step of -1 in ln T makes the Dormand-Prince control reject many attempts (16
    for U = 2 in the oracle).  A rejected attempt keeps the step's first k slot (first same
    as last) and its retry forms that slot's sum again; two flows in one batch must follow
    the oracle's accept/reject sequence exactly in FP64 and reach its T_c.  The final state
    is held to ADAPTIVE_FINAL_FP64 (the oracle alone moves by 1.05e-10 here when it sums in
    another order)."""
    fm = _fm()
    torch, dev = torch_dev
    N, L, h0 = 16, 32, -1.0
    U = [2.0, 1.5]
    f = fm.Flow(N=N, L=L, U=2.0, precision=prec, integrator="rk45", h0=h0, max_batch=2,
                device=dev)
    try:
        res, Vg = f.run_batch(U, [1.0, 1.0], return_V=True)
    finally:
        f.close()
    Vg = Vg.cpu().numpy()
    for i in range(2):
        cfg = O.flowcfg(T0=1.0, U=U[i], integrator=1, h0=h0)
        Vo, ores, _ = O.flow(O.model(N, L), cfg, U[i])
        assert ores["n_rejected"] > 0
        assert res[i]["status"] == ores["status"], (i, res[i], ores)
        if ores["status"] == O.DIVERGED:
            assert res[i]["T_c"] == pytest.approx(ores["T_c"], rel=1e-3)
        if prec == "fp64":
            assert (res[i]["n_accepted"], res[i]["n_rejected"]) == \
                (ores["n_accepted"], ores["n_rejected"])
            assert rel(Vg[i], Vo) <= ADAPTIVE_FINAL_FP64


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("bf16", 1e-2), ("bf16x3", 1e-4)])
def test_mixed_precision_along_the_fp64_schedule(torch_dev, prec, tol):
    """N = 96, L = 256, U = 3 (the mixed-precision workload's size): the FP64 GPU path (its
    RHS matches the oracle to 1e-10 above; the oracle itself takes minutes per RHS here)
    sets the Dormand-Prince schedule; the mixed-precision path replays the same steps
    (every step accepted) and its state is compared after each accepted step, up to the
    divergence.  Then its own adaptive flow's T_c."""
    fm = _fm()
    torch, dev = torch_dev
    N, L, U = 96, 256, 3.0
    f64 = fm.Flow(N=N, L=L, U=U, precision="fp64", integrator="rk45", device=dev)
    V = torch.full((1, N, N, N), U, dtype=torch.float64, device=dev)
    lnT, h, lnTe = 0.0, math.log(0.01) / 200, math.log(0.01)
    sched, states = [], []
    try:
        for _ in range(200):
            l1, h1, acc = f64.step([lnT], [h], V)
            if acc[0]:
                sched.append((lnT, h))
                states.append(V.clone())
                lnT = l1[0]
                if V.abs().max().item() > 20.0 or lnT <= lnTe:
                    break
            h = max(h1[0], lnTe - lnT)
        r64 = f64.run_batch([U], [1.0])[0]
    finally:
        f64.close()
    assert states[-1].abs().max().item() > 20.0 and len(sched) >= 5
    fm_ = fm.Flow(N=N, L=L, U=U, precision=prec, integrator="rk45", rtol=1e30, device=dev)
    Vm = torch.full((1, N, N, N), U, dtype=torch.float64, device=dev)
    try:
        for (l0, h0), Vr in zip(sched, states):
            _, _, acc = fm_.step([l0], [h0], Vm)
            assert acc[0]
            err = ((Vm - Vr).abs().max() / Vr.abs().max()).item()
            assert err <= tol, (l0, err)
    finally:
        fm_.close()
    fa = fm.Flow(N=N, L=L, U=U, precision=prec, integrator="rk45", device=dev)
    try:
        r = fa.run_batch([U], [1.0])[0]
    finally:
        fa.close()
    assert r["status"] == r64["status"] == fm.DIVERGED
    assert r["T_c"] == pytest.approx(r64["T_c"], rel=1e-3)


def test_flow_with_z_feedback_fp64(torch_dev):
    fm = _fm()
    torch, dev = torch_dev
    N, L, U = 16, 32, 3.0
    lnT, tab = inputs.synthetic_z_table(N, U, 1.0, 0.01)
    f = fm.Flow(N=N, L=L, U=U, precision="fp64", integrator="rk45", z_lnT=lnT, z_table=tab,
                device=dev)
    try:
        res, Vg = f.run_batch([U], [1.0], return_V=True)
    finally:
        f.close()
    Vo, ores, _ = O.flow(O.model(N, L), O.flowcfg(U=U, integrator=1, z_lnT=lnT, z_tab=tab), U)
    assert res[0]["status"] == ores["status"]
    assert res[0]["T_c"] == pytest.approx(ores["T_c"], rel=1e-6)
    assert rel(Vg.cpu().numpy()[0], Vo) <= ADAPTIVE_FINAL_FP64


def test_run_batch_per_flow_z_tables(torch_dev):
    """Three flows in one batch, each with its own Z table (the synthetic table of its own
    U, one of them with fewer nodes' worth of variation), against the oracle's flows with the
    same tables; then a table that is not ascending, or has a Z that is not positive and
    finite, is refused."""
    fm = _fm()
    torch, dev = torch_dev
    N, L = 16, 32
    U = [3.0, 2.5, 3.5]
    tabs = [inputs.synthetic_z_table(N, u, 1.0, 0.01) for u in U]
    zl = np.stack([t[0] for t in tabs])
    zt = np.stack([t[1] for t in tabs])
    zt[1] = np.sqrt(zt[1])          # a different table shape for the second flow
    f = fm.Flow(N=N, L=L, U=U[0], precision="fp64", integrator="rk45", z_lnT=zl[0],
                z_table=zt[0], max_batch=3, device=dev)
    try:
        res, Vg = f.run_batch(U, [1.0] * 3, z_lnT=zl, z_tables=zt, return_V=True)
        Vg = Vg.cpu().numpy()
        for i in range(3):
            Vo, ores, _ = O.flow(O.model(N, L), O.flowcfg(U=U[i], integrator=1, z_lnT=zl[i],
                                                         z_tab=zt[i]), U[i])
            assert res[i]["status"] == ores["status"] == O.DIVERGED
            assert res[i]["T_c"] == pytest.approx(ores["T_c"], rel=1e-6)
            assert rel(Vg[i], Vo) <= ADAPTIVE_FINAL_FP64
        bad = zl.copy()
        bad[2, 5] = bad[2, 4]
        with pytest.raises(fm.FmError):
            f.run_batch(U, [1.0] * 3, z_lnT=bad, z_tables=zt)
        for z in (0.0, -0.2, np.inf, np.nan):
            bad = zt.copy()
            bad[0, 3, 7] = z
            with pytest.raises(fm.FmError):
                f.run_batch(U, [1.0] * 3, z_lnT=zl, z_tables=bad)
        with pytest.raises(ValueError):
            f.run_batch(U, [1.0] * 3, z_lnT=zl[:, :-1], z_tables=zt)
    finally:
        f.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("flow", ["temperature", "interaction"])
def test_sync_batch_against_oracle(torch_dev, prec, flow):
    """sync_batch: flows with equal T0 (for the interaction flow: equal temperature) step on
    one schedule, and each group's bins are computed once, by its first running flow (the
    one diverging first hands that over).  Six flows in two interleaved groups against the
    oracle's shared-schedule flows of each group: FP64 with the oracle's exact accept/reject
    counts, T_c (g*) to 1e-9 and V to ADAPTIVE_FINAL_FP64; FP32 status and T_c (g*) to
    1e-3."""
    fm = _fm()
    torch, dev = torch_dev
    N, L = 16, 32
    gf = flow == "interaction"
    U = [2.5, 2.2, 2.0, 1.5, 1.8, 0.4] if not gf else [3.0, 2.6, 2.5, 0.5, 3.5, 4.0]
    T0 = [1.0, 0.7, 1.0, 1.0, 0.7, 1.0] if not gf else [0.1, 0.05, 0.1, 0.1, 0.05, 0.1]
    f = fm.Flow(N=N, L=L, U=U[0], T0=T0[0], precision=prec, integrator="rk45",
                flow=flow, max_batch=6, sync_batch=True, device=dev)
    try:
        res, Vg = f.run_batch(U, T0, return_V=True)
    finally:
        f.close()
    Vg = Vg.cpu().numpy()
    m = O.model(N, L)
    key = "g_c" if gf else "T_c"
    for t0 in sorted(set(T0)):
        idx = [i for i in range(6) if T0[i] == t0]
        Vo, ro = O.flow_sync(m, O.flowcfg(T0=t0, integrator=1, atol=0.0, gflow=gf),
                             [U[i] for i in idx])
        assert any(r["status"] == O.DIVERGED for r in ro)
        for j, i in enumerate(idx):
            assert res[i]["status"] == ro[j]["status"], (i, res[i], ro[j])
            if ro[j]["status"] == O.DIVERGED:
                tol = 1e-9 if prec == "fp64" else 1e-3
                assert abs(res[i][key] / ro[j][key] - 1.0) <= tol, (i, res[i][key], ro[j][key])
            if prec == "fp64":
                assert (res[i]["n_accepted"], res[i]["n_rejected"], res[i]["n_rhs"]) == \
                    (ro[j]["n_accepted"], ro[j]["n_rejected"], ro[j]["n_rhs"]), (i, res[i], ro[j])
                assert rel(Vg[i], Vo[j]) <= ADAPTIVE_FINAL_FP64, (i, rel(Vg[i], Vo[j]))


@pytest.mark.parametrize("case", ["U2.5", "U2_h0-1", "U3_Z"])
def test_rk45_schedule_replay_fp64(torch_dev, case):
    """The FP64 path at 1e-10 after every accepted step of an adaptive flow: the oracle's own
    flow fixes the schedule (its accepted points), and the GPU and the oracle each integrate
    their own state along it (every attempt accepted), so rounding cannot move the steps.
    Cases: a flow from T0 = 1 to its divergence; one whose first step of -1 the control
    rejects many times (only the accepted steps are replayed); one with the Z table."""
    fm = _fm()
    torch, dev = torch_dev
    N, L = 16, 32
    kw = {"U2.5": dict(U=2.5), "U2_h0-1": dict(U=2.0, h0=-1.0),
          "U3_Z": dict(U=3.0)}[case]
    zkw = {}
    if case == "U3_Z":
        lnTz, tab = inputs.synthetic_z_table(N, 3.0, 1.0, 0.01)
        zkw = dict(z_lnT=lnTz, z_tab=tab)
    m = O.model(N, L)
    _, ores, trace = O.flow(m, O.flowcfg(T0=1.0, integrator=1, **kw, **zkw), kw["U"])
    assert ores["status"] == O.DIVERGED and len(trace) > 10
    replay = O.flowcfg(T0=1.0, integrator=1, rtol=1e30, **kw, **zkw)
    gkw = dict(z_lnT=zkw["z_lnT"], z_table=zkw["z_tab"]) if zkw else {}
    f = fm.Flow(N=N, L=L, U=kw["U"], precision="fp64", integrator="rk45", rtol=1e30,
                device=dev, **gkw)
    try:
        Vo = inputs.constant_state(N, kw["U"])
        Vd = torch.from_numpy(Vo.reshape(1, N, N, N).copy()).to(dev)
        worst = 0.0
        for i in range(len(trace) - 1):
            s, h = trace[i, 0], trace[i + 1, 0] - trace[i, 0]
            _, _, acc = f.step([s], [h], Vd)
            _, _, Vo, oacc, _ = O.step(m, replay, s, h, Vo)
            assert acc[0] and oacc
            e = rel(Vd.cpu().numpy()[0], Vo)
            worst = max(worst, e)
            assert e <= 1e-10, (i, s, e)
        assert np.abs(Vo).max() > 20.0
    finally:
        f.close()


def test_kernel_time_replay_leaves_the_flow_state(torch_dev):
    """The kernel replay measurement times each group and restores the flows: the next run
    agrees with the one before it (to the rounding of phase 1's atomic bin sums, whose order
    varies from run to run)."""
    fm = _fm()
    torch, dev = torch_dev
    f = fm.Flow(N=16, L=32, U=2.5, precision="fp64", integrator="rk45", max_batch=2, device=dev)
    try:
        r1 = f.run_batch([2.5, 2.0], [1.0, 0.8])
        for g in (0, 1, 2, 3):
            assert f.kernel_time(g, batch=2, reps=3) > 0.0
        r2 = f.run_batch([2.5, 2.0], [1.0, 0.8])
        with pytest.raises(fm.FmError):
            f.kernel_time(4, batch=1, reps=1)
    finally:
        f.close()
    for x, y in zip(r1, r2):
        assert x["status"] == y["status"] == fm.DIVERGED
        assert abs(x["T_c"] / y["T_c"] - 1.0) < 1e-10


def test_stop_at_start(torch_dev):
    fm = _fm()
    f = fm.Flow(N=16, L=32, U=30.0, precision="fp32", integrator="rk45", device=torch_dev[1])
    try:
        res = f.run_batch([30.0], [1.0])
    finally:
        f.close()
    assert res[0]["status"] == fm.DIVERGED and res[0]["T_c"] == pytest.approx(1.0)
    assert res[0]["n_rhs"] == 0
