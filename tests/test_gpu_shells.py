"""GPU parity of energy-shell patching (Sec. 3.2: angular patches subdivided in energy; the
paper's 224 = 7 shells x 32 sectors), through the C ABI against the oracle:

* the right-hand side at small sizes (3 and 5 shells, the latter with given edges, t' and mu
  away from half filling), every precision and each matrix-core phase-2a kernel, every
  element;
* the paper's 224 patches on a 128 x 128 grid, sampled outputs (FP64, FP32 on the vector
  units, the direct FP64 kernel);
* a Dormand-Prince flow with three shells to its divergence, FP64 and FP32.

Tolerances as for angular patches: FP64 1e-10, FP32 and split bf16 1e-4, bf16 1e-2, T_c 1e-3
(FP64 1e-9).
"""
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


def gpu_rhs(torch_dev, T, V, **kw):
    torch, dev = torch_dev
    from paper_2005_00827_amd import fm
    N = kw["N"]
    V = np.asarray(V, np.float64).reshape(-1, N, N, N)
    f = fm.Flow(max_batch=V.shape[0], device=dev, **kw)
    try:
        out = f.rhs(np.atleast_1d(T), torch.from_numpy(V).to(dev))
        torch.cuda.synchronize()
        return out.cpu().numpy()
    finally:
        f.close()


CASES = [(24, 32, 3, None, 0.0, 0.0), (40, 32, 5, [0.3, 1.1], -0.3, -0.4)]


@pytest.mark.parametrize("prec,y_kernel", [("fp64", 0), ("fp64_direct", 0), ("fp32", 1),
                                           ("fp32", 3), ("bf16", 1), ("bf16", 2), ("bf16", 3),
                                           ("bf16x3", 3)])
@pytest.mark.parametrize("N,L,S,edges,tp,mu", CASES)
def test_shell_rhs_small(torch_dev, prec, y_kernel, N, L, S, edges, tp, mu):
    V = inputs.noisy_state(N, 2.0, seed=9)
    T = 0.08
    ref = O.rhs(O.model(N, L, tp=tp, mu=mu, n_shells=S, shell_edges=edges), T, V)
    got = gpu_rhs(torch_dev, T, V, N=N, L=L, tp=tp, mu=mu, geometry="shells", n_shells=S,
                  shell_edges=edges, precision=prec, y_kernel=y_kernel)[0]
    assert rel(got, ref) <= TOL[prec], (prec, rel(got, ref))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp64_direct"])
def test_shell_rhs_224_patches_sampled(torch_dev, prec):
    N, L, S = 224, 128, 7
    V = inputs.noisy_state(N, 3.0)
    T = 0.1
    abc = inputs.sample_indices(N, 48)
    ref = O.rhs_points(O.model(N, L, n_shells=S), T, V, abc)
    got = gpu_rhs(torch_dev, T, V, N=N, L=L, geometry="shells", n_shells=S, precision=prec)[0]
    assert rel(got[abc[:, 0], abc[:, 1], abc[:, 2]], ref) <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_shell_flow_against_oracle(torch_dev, prec):
    torch, dev = torch_dev
    from paper_2005_00827_amd import fm
    N, L, S, U = 24, 32, 3, 2.5
    f = fm.Flow(N=N, L=L, U=U, geometry="shells", n_shells=S, precision=prec,
                integrator="rk45", device=dev)
    try:
        res, Vg = f.run_batch([U], [1.0], return_V=True)
    finally:
        f.close()
    Vo, ores, _ = O.flow(O.model(N, L, n_shells=S), O.flowcfg(U=U, integrator=1), U)
    assert res[0]["status"] == ores["status"] == fm.DIVERGED
    tol = 1e-9 if prec == "fp64" else 1e-3
    assert abs(res[0]["T_c"] / ores["T_c"] - 1.0) <= tol
    if prec == "fp64":
        assert (res[0]["n_accepted"], res[0]["n_rejected"]) == (ores["n_accepted"], ores["n_rejected"])
        # independently adaptive FP64 flows: see ADAPTIVE_FINAL_FP64 in test_gpu_parity.py
        assert rel(Vg.cpu().numpy()[0], Vo) <= 1e-9
