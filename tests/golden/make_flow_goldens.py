"""Writes the oracle flow fixtures used by the GPU tests of whole flows at N = 48, L = 128.

Calls only the oracle (oracle/oracle.py) and the seeded input module; run from the repository
root with `python tests/golden/make_flow_goldens.py` (about 80 minutes on 8 host threads).

  c2_flow.txt   the quasi-particle workload: N = 48, L = 128, U = 3, T 1 -> 0.01, Dormand-Prince
                (rtol 1e-6), synthetic Z table, FP64: outcome, counts, T_c and the trace of
                (ln T, max|V|) after every accepted step
  c4_flows.txt  three early-diverging flows of the 64-flow sweep (N = 48, L = 128, no Z,
                Dormand-Prince): (U, T0, status, T_c, accepted, rejected, RHS)
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O                 # noqa: E402
from paper_2005_00827_amd import inputs       # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
C4_FLOWS = [(4.5, 0.5), (4.0, 0.5 * 4.0 ** (1.0 / 7.0)), (3.5, 0.5)]


def c2():
    w = inputs.workload("C2")
    N, L, U = w["N"], w["L"], w["U"][0]
    zl, zt = inputs.synthetic_z_table(N, U, 1.0, w["T_end"])
    cfg = O.flowcfg(T0=1.0, T_end=w["T_end"], U=U, integrator=1, z_lnT=zl, z_tab=zt,
                    progress=True)
    _, res, trace = O.flow(O.model(N, L), cfg, U)
    with open(os.path.join(HERE, "c2_flow.txt"), "w") as fh:
        fh.write("# oracle flow, N=48 L=128 U=3 T 1 -> 0.01, Dormand-Prince rtol 1e-6, synthetic Z\n")
        fh.write("# written by tests/golden/make_flow_goldens.py (oracle only)\n")
        for k in ("status", "n_accepted", "n_rejected", "n_rhs"):
            fh.write("%s %d\n" % (k, res[k]))
        fh.write("T_c %.17g\n" % res["T_c"])
        for s, m in trace:
            fh.write("trace %.17g %.17g\n" % (s, m))


def c4():
    w = inputs.workload("C4")
    m = O.model(w["N"], w["L"])
    with open(os.path.join(HERE, "c4_flows.txt"), "w") as fh:
        fh.write("# oracle flows of the 64-flow sweep, N=48 L=128, no Z, Dormand-Prince rtol 1e-6\n")
        fh.write("# written by tests/golden/make_flow_goldens.py (oracle only)\n")
        fh.write("# U T0 status T_c n_accepted n_rejected n_rhs\n")
        for U, T0 in C4_FLOWS:
            cfg = O.flowcfg(T0=T0, T_end=w["T_end"], U=U, integrator=1, progress=True)
            _, res, _ = O.flow(m, cfg, U)
            fh.write("%.17g %.17g %d %.17g %d %d %d\n" % (U, T0, res["status"], res["T_c"],
                                                          res["n_accepted"], res["n_rejected"],
                                                          res["n_rhs"]))
            fh.flush()


if __name__ == "__main__":
    c4()
    c2()
