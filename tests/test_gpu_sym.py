"""GPU parity of the symmetric-state mode (sym_state = 1) through the C ABI against the oracle.

For a state invariant under the square lattice's point group (V(pi a, pi b, pi c) = V(a, b, c)
for the patch permutation pi of each of the 8 operations, Z likewise) the products of a
transfer q = o(r) are those of its orbit representative r read through the permutation, so
phase 2 computes the representatives' products only.  Inputs: seeded states symmetrised over
the group with permutations taken from the oracle's own geometry (each loop point mapped by
the operation, k -> (+-kx, +-ky) and the swap), Z from the synthetic table (it depends on
cos 4 theta).  Expected values come only from the oracle; tolerances as in the other parity
tests: 1e-10 double, 1e-4 single and split bf16, 1e-2 bf16.
"""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2005_00827_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-4, "bf16": 1e-2, "bf16x3": 1e-4}
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    return torch, torch.device("cuda:0")


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def group_perms(m):
    """The 8 patch permutations of the oracle geometry: pi_o(patch(j)) = patch(o j), o j the
    loop point (jx, jy) swapped (o & 4) and mirrored (o & 2: x, o & 1: y) on the half-shifted
    grid (j -> L - 1 - j is k -> -k)."""
    _, patch, _, _ = O.geometry(m)
    L, N = m.L, m.N
    P = np.asarray(patch).reshape(L, L)            # [jy][jx]
    jy, jx = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    perms = []
    for o in range(8):
        x, y = (jy, jx) if o & 4 else (jx, jy)
        if o & 2:
            x = L - 1 - x
        if o & 1:
            y = L - 1 - y
        p = -np.ones(N, np.int64)
        p[P.ravel()] = P[y, x].ravel()
        assert (p >= 0).all() and len(set(p.tolist())) == N
        perms.append(p)
    return perms


def symmetrise(V, perms):
    return sum(V[np.ix_(p, p, p)] for p in perms) / len(perms)


def sym_z(N, U, T):
    lnT, tab = inputs.synthetic_z_table(N, U, 1.0, 0.01)
    Z = np.array([np.interp(math.log(T), lnT, tab[:, a]) for a in range(N)])
    return lnT, tab, Z


def lib_rhs(torch_dev, N, L, T, V, prec, **kw):
    from paper_2005_00827_amd import fm
    torch, dev = torch_dev
    V = np.asarray(V, np.float64).reshape(-1, N, N, N)
    f = fm.Flow(N=N, L=L, precision=prec, max_batch=V.shape[0], device=dev, **kw)
    try:
        out = f.rhs(np.atleast_1d(T), torch.from_numpy(V).to(dev))
        torch.cuda.synchronize()
        return out.cpu().numpy()
    finally:
        f.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16", "bf16x3"])
@pytest.mark.parametrize("N,L,T,kw", [(16, 32, 0.2, {}), (24, 20, 0.07, {}), (48, 64, 0.1, {}),
                                      (4, 16, 0.1, {}), (16, 32, 0.05, {"channels": 1}),
                                      (16, 32, 0.05, {"channels": 2}),
                                      (16, 32, 0.05, {"channels": 4}),
                                      (8, 16, 0.2, {"tp": -0.3, "mu": -0.4})])
def test_rhs_sym_small(torch_dev, prec, N, L, T, kw):
    m = O.model(N, L, tp=kw.get("tp", 0.0), mu=kw.get("mu", 0.0),
                channels=kw.get("channels", O.CH_ALL))
    perms = group_perms(m)
    # a channel alone on a nearly constant state cancels (the direct channel vanishes for
    # constant V), so channel subsets take a random state, as in the full mode's tests
    V0 = inputs.random_state(N, seed=7) if "channels" in kw else inputs.noisy_state(N, 2.5, seed=7)
    V = symmetrise(V0, perms)
    lnT, tab, Z = sym_z(N, 2.5, T)
    ref = O.rhs(m, T, V, Z=Z)
    got = lib_rhs(torch_dev, N, L, T, V, prec, sym_state=1, z_lnT=lnT, z_table=tab, **kw)[0]
    assert rel(got, ref) <= TOL[prec], rel(got, ref)
    # a state without the symmetry: the mode's results differ (the assumption matters)
    Va = inputs.random_state(N, seed=8)
    if N >= 8 and kw.get("channels", 7) == 7:
        bad = lib_rhs(torch_dev, N, L, T, Va, prec, sym_state=1, z_lnT=lnT, z_table=tab, **kw)[0]
        assert rel(bad, O.rhs(m, T, Va, Z=Z)) > 10 * TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "bf16", "bf16x3"])
@pytest.mark.parametrize("tile_rows", [1, 2, 4])
@pytest.mark.parametrize("y_kernel", [2, 3])
def test_rhs_sym_every_tile_choice(torch_dev, prec, tile_rows, y_kernel):
    """Phase 2a on the class kernel (class 0) or the orbit kernel (operation 0), every tile
    count; two flows per batch."""
    N, L, T = 32, 64, 0.09
    m = O.model(N, L)
    perms = group_perms(m)
    V = np.stack([symmetrise(inputs.noisy_state(N, 2.5, seed=s), perms) for s in (3, 4)])
    got = lib_rhs(torch_dev, N, L, [T, T], V, prec, sym_state=1, y_kernel=y_kernel,
                  tile_rows=tile_rows)
    for i in range(2):
        assert rel(got[i], O.rhs(m, T, V[i])) <= TOL[prec], i


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16", "bf16x3"])
def test_rhs_sym_full_size_sampled(torch_dev, prec):
    """N = 128, L = 512 (the batch workload's size): sampled outputs against the oracle, for
    two flows in one batch (the second reads its products at the batch's per-flow stride)."""
    N, L, T = 128, 512, 0.08
    m = O.model(N, L)
    perms = group_perms(m)
    V = np.stack([symmetrise(inputs.noisy_state(N, 3.0, seed=s), perms) for s in (1, 2)])
    lnT, tab, Z = sym_z(N, 3.0, T)
    abc = inputs.sample_indices(N, 48)
    got = lib_rhs(torch_dev, N, L, [T, T], V, prec, sym_state=1, z_lnT=lnT, z_table=tab)
    for i in range(2):
        ref = O.rhs_points(m, T, V[i], abc, Z=Z)
        assert rel(got[i][abc[:, 0], abc[:, 1], abc[:, 2]], ref) <= TOL[prec], (i, prec)


def c2_golden():
    out = {}
    for ln in open(os.path.join(GOLD, "c2_flow.txt")):
        if ln.startswith("#") or not ln.strip():
            continue
        k, *v = ln.split()
        if k == "T_c":
            out[k] = float(v[0])
        elif k != "trace":
            out[k] = int(v[0])
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_sym_c2_flow_against_oracle_golden(torch_dev, prec):
    """The quasi-particle flow (N = 48, L = 128, U = 3, Z table, from V = U) in the symmetric
    mode against the oracle's flow in tests/golden/c2_flow.txt: FP64 with the same steps and
    T_c to 1e-9, single precision to 1e-3."""
    from paper_2005_00827_amd import fm
    gold = c2_golden()
    w = inputs.workload("C2")
    N, L, U = w["N"], w["L"], w["U"][0]
    zl, zt = inputs.synthetic_z_table(N, U, 1.0, w["T_end"])
    f = fm.Flow(N=N, L=L, U=U, T0=1.0, T_end=w["T_end"], integrator="rk45", precision=prec,
                z_lnT=zl, z_table=zt, sym_state=1, device=torch_dev[1])
    try:
        res = f.run_batch([U], [1.0])[0]
    finally:
        f.close()
    assert res["status"] == gold["status"] == fm.DIVERGED
    if prec == "fp64":
        assert (res["n_accepted"], res["n_rejected"], res["n_rhs"]) == \
            (gold["n_accepted"], gold["n_rejected"], gold["n_rhs"])
        assert abs(res["T_c"] / gold["T_c"] - 1.0) <= 1e-9
    else:
        assert abs(res["T_c"] / gold["T_c"] - 1.0) <= 1e-3


def test_sym_c5_batch_against_converged_fp64(torch_dev):
    """The 16-flow batch (N = 128, L = 512, U = 1..4, Z per flow) in the symmetric mode: T_c
    of the bf16, split-bf16, FP32 and FP64 right-hand sides against a converged FP64 run of
    the full mode (rtol 1e-8) to 1e-3 (bf16 to its unit roundoff 2^-9: its products are
    rounded to 8 bits and its trajectory varies with the order of the bins' float atomics),
    and the same statuses."""
    from paper_2005_00827_amd import fm
    w = inputs.workload("C5")
    N, L, U, T0 = w["N"], w["L"], w["U"], w["T0"]
    tabs = [inputs.synthetic_z_table(N, u, 1.0, w["T_end"]) for u in U]
    zl = np.stack([t[0] for t in tabs])
    zt = np.stack([t[1] for t in tabs])

    def run(prec, sym, rtol=0.0):
        f = fm.Flow(N=N, L=L, U=U[0], T0=1.0, T_end=w["T_end"], integrator="rk45",
                    precision=prec, rtol=rtol, z_lnT=zl[0], z_table=zt[0], max_batch=len(U),
                    sym_state=sym, sync_batch=2 if sym else 0, device=torch_dev[1])
        try:
            return f.run_batch(U, T0, z_lnT=zl, z_tables=zt)
        finally:
            f.close()

    ref = run("fp64", 0, 1e-8)
    assert sum(r["status"] == fm.DIVERGED for r in ref) >= 12
    for prec in ("bf16", "bf16x3", "fp32", "fp64"):
        res = run(prec, 1)
        for i, (r, q) in enumerate(zip(res, ref)):
            assert r["status"] == q["status"], (prec, i, r, q)
            if q["status"] == fm.DIVERGED:
                tol = 2.0 ** -9 if prec == "bf16" else 1e-3
                assert abs(r["T_c"] / q["T_c"] - 1.0) <= tol, (prec, i, r["T_c"], q["T_c"])


def test_sym_rejects_asymmetric_per_flow_tables(torch_dev):
    from paper_2005_00827_amd import fm
    N, L = 16, 32
    lnT, tab = inputs.synthetic_z_table(N, 2.5, 1.0, 0.01)
    f = fm.Flow(N=N, L=L, T0=1.0, T_end=0.01, integrator="rk45", precision="fp32",
                z_lnT=lnT, z_table=tab, max_batch=1, sym_state=1, device=torch_dev[1])
    try:
        bad = tab.copy()
        bad[:, 3] *= 1.01
        with pytest.raises(fm.FmError):
            f.run_batch([2.5], [1.0], z_lnT=lnT[None], z_tables=bad[None])
    finally:
        f.close()


_ORACLE_FLOWS = {}


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_sym_step_sharing_group_against_oracle(torch_dev, prec):
    """A step-sharing group of five flows (one T0, U = 2.5 ... 1.5, one Z table) in the
    symmetric mode on the orbit kernel: the running flows that read one group's bins are
    served two per phase-2a block (pairs, and a lone flow when their number is odd, which
    changes as flows diverge).  Against the oracle's shared-schedule flows: the same
    statuses, and T_c to 1e-3 in FP32 and 1e-2 in bf16 (its products carry 8 bits; a pair
    that mixed up its flows' operands or outputs would move T_c by several per cent, since
    the couplings differ by 0.25 U)."""
    from paper_2005_00827_amd import fm
    N, L = 16, 32
    U = [2.5, 2.25, 2.0, 1.75, 1.5]
    zl, zt = inputs.synthetic_z_table(N, 2.0, 1.0, 0.01)
    f = fm.Flow(N=N, L=L, U=U[0], T0=1.0, precision=prec, integrator="rk45", z_lnT=zl,
                z_table=zt, sym_state=1, y_kernel=3, max_batch=len(U), sync_batch=True,
                device=torch_dev[1])
    try:
        res = f.run_batch(U, [1.0] * len(U))
    finally:
        f.close()
    if "group5" not in _ORACLE_FLOWS:   # the same oracle flows serve both precisions
        _ORACLE_FLOWS["group5"] = O.flow_sync(
            O.model(N, L), O.flowcfg(T0=1.0, integrator=1, atol=0.0, z_lnT=zl, z_tab=zt), U)[1]
    ro = _ORACLE_FLOWS["group5"]
    assert sum(r["status"] == O.DIVERGED for r in ro) >= 3
    tol = 1e-2 if prec == "bf16" else 1e-3
    for i, (r, q) in enumerate(zip(res, ro)):
        assert r["status"] == q["status"], (i, r, q)
        if q["status"] == O.DIVERGED:
            assert abs(r["T_c"] / q["T_c"] - 1.0) <= tol, (i, r["T_c"], q["T_c"])
