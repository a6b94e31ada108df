"""fm_flow_rhs_static, the right-hand side for callers that cannot allocate device memory,
against fm_flow_rhs on a caller-allocated workspace: the same kernels on the library's static
device array.  Two calls in a row, the second with a smaller input (fewer patches, a
smaller grid, one state instead of two), so the second reuses the array the first left
behind; then a configuration beyond the array's size is refused."""
import math

import numpy as np
import pytest

from paper_2005_00827_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-4}


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_static_rhs_matches_workspace_rhs(prec):
    import torch
    from paper_2005_00827_amd import fm
    dev = torch.device("cuda:0")
    for N, L, T in ((16, 32, [0.3, 0.05]), (8, 16, [0.2])):
        U = 2.5
        zl, zt = inputs.synthetic_z_table(N, U, 1.0, 0.01)
        V = np.stack([inputs.noisy_state(N, U, seed=7 + i) for i in range(len(T))])
        Vd = torch.from_numpy(V).to(dev)
        kw = dict(N=N, L=L, precision=prec, max_batch=len(T), z_lnT=zl, z_table=zt)
        f = fm.Flow(device=dev, **kw)
        try:
            ref = f.rhs(T, Vd).cpu().numpy()
        finally:
            f.close()
        got = fm.rhs_static(T, Vd, device=dev, **kw).cpu().numpy()
        torch.cuda.synchronize()
        assert rel(got, ref) <= TOL[prec], (N, L, prec, rel(got, ref))
        # the same call again reuses the handle built on the static array
        again = fm.rhs_static(T, Vd, device=dev, **kw).cpu().numpy()
        assert rel(again, ref) <= TOL[prec]
    V = torch.zeros((1, 96, 96, 96), dtype=torch.float64, device=dev)
    with pytest.raises(fm.FmError) as e:
        fm.rhs_static([0.1], V, device=dev, N=96, L=256, precision=prec)
    assert "static array" in str(e.value)
