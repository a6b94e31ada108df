"""ctypes wrapper of the double-precision CPU oracle (``fm_oracle.c``).

TEST INFRASTRUCTURE. The oracle checks the HIP library; it is not part of it. Only the test
suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import this
module. It shares no code with ``paper_2005_00827_amd``; both sides only receive the same
seeded inputs from ``paper_2005_00827_amd.inputs``.

Functions mirror the definitions written out in ``fm_oracle.c``:

* geometry of the half-shifted loop grid, angular patches and snapped Fermi points
  (Sec. 2.1 Eq. free_dispersion_xi; Sec. 3.2 on angular patch resolutions);
* the bubble weights chi and T d/dT chi;
* the one-loop flow right-hand side dV/d ln T (App. A, Eqs. vertex_flow_general and
  vertex_flow_feedback_Z, written out per channel), direct and binned;
* RK4 / Dormand-Prince flows in ln T with the stop rule of Sec. 3.2 (largest |V| above a
  threshold);
* the interaction flow in g at fixed T (Sec. 2.2; App. A, Steps 1-2: lines G_g = g Z G0,
  S_g = Z^2 G0), with the crossover coupling U* = g*^2 U.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from ctypes import POINTER, c_double, c_int, c_uint

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CH_PP, CH_CR, CH_D, CH_ALL = 1, 2, 4, 7
RUNNING, DIVERGED, NONFINITE, REACHED_TEND, STEPFAIL = 0, 1, 2, 3, 4


class Model(ctypes.Structure):
    _fields_ = [("t", c_double), ("tp", c_double), ("mu", c_double), ("N", c_int),
                ("L", c_int), ("identity", c_int), ("channels", c_uint), ("n_shells", c_int),
                ("shell_edges", POINTER(c_double))]


class FlowCfg(ctypes.Structure):
    _fields_ = [("T0", c_double), ("T_end", c_double), ("integrator", c_int),
                ("n_steps", c_int), ("rtol", c_double), ("atol", c_double),
                ("h0", c_double), ("h_min", c_double), ("v_max", c_double),
                ("n_z", c_int), ("z_lnT", POINTER(c_double)), ("z_tab", POINTER(c_double)),
                ("gflow", c_int), ("g_end", c_double), ("v_rel", c_double),
                ("rhs_binned", c_int), ("progress", c_int), ("k_tab", POINTER(c_double))]


class Result(ctypes.Structure):
    _fields_ = [("T_c", c_double), ("T_final", c_double), ("max_abs_V", c_double),
                ("status", c_int), ("n_accepted", c_int), ("n_rejected", c_int),
                ("n_rhs", c_int), ("g_c", c_double), ("U_star", c_double),
                ("g_final", c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        d, i = c_double, c_int
        pd, pi = POINTER(c_double), POINTER(c_int)
        pm, pf, pr = POINTER(Model), POINTER(FlowCfg), POINTER(Result)
        sig = {
            "orc_phi_dd": (d, [d, d]),
            "orc_chi_ph": (d, [d, d, d]), "orc_chi_pp": (d, [d, d, d]),
            "orc_chidot_ph": (d, [d, d, d]), "orc_chidot_pp": (d, [d, d, d]),
            "orc_geometry": (i, [pm, pd, pi, pi, pd]),
            "orc_transfer_counts": (i, [pm, pi, pi]),
            "orc_rhs": (i, [pm, d, pd, pd, pd, i]),
            "orc_rhs_g": (i, [pm, d, d, pd, pd, pd, i]),
            "orc_rhs_gk": (i, [pm, d, d, pd, pd, pd, pd, i]),
            "orc_katanin": (i, [i, pd, i, pd, pd, pd]),
            "orc_rhs_points_g": (i, [pm, d, d, pd, pd, i, pi, pd, i]),
            "orc_rhs_binned": (i, [pm, d, pd, pd, pd, i]),
            "orc_rhs_points": (i, [pm, d, pd, pd, i, pi, pd, i]),
            "orc_flow": (i, [pm, pf, d, pd, pr, pd, i, pi, i]),
            "orc_step": (i, [pm, pf, pd, pd, pd, pi, pd, i]),
            "orc_flow_sync": (i, [pm, pf, i, pd, pd, pr, i]),
            "orc_sigma2": (i, [pm, d, d, pd, i, pd, pd, pd, pd, i]),
            "orc_kramers_kronig": (None, [i, d, d, pd, pd]),
            "orc_sigma_wmax": (d, [pm]),
            "orc_dopri_tableau": (i, [pd, pd, pd]),
            "orc_num_threads": (i, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype, fn.argtypes = res, args
        _lib = L
    return _lib


def _pd(a):
    return a.ctypes.data_as(POINTER(c_double)) if a is not None else None


def _pi(a):
    return a.ctypes.data_as(POINTER(c_int)) if a is not None else None


def model(N, L, t=1.0, tp=0.0, mu=0.0, identity=False, channels=CH_ALL, n_shells=0,
          shell_edges=None) -> Model:
    """n_shells > 1: energy-shell patching, N = n_shells x angular sectors; shell_edges:
    (n_shells - 1)/2 ascending |xi| edges, or None for the default."""
    m = Model(float(t), float(tp), float(mu), int(N), int(L), int(bool(identity)),
              int(channels), int(n_shells), None)
    if shell_edges is not None:
        se = np.ascontiguousarray(shell_edges, np.float64)
        m.shell_edges = _pd(se)
        m._keep = se
    return m


def n_threads() -> int:
    return int(lib().orc_num_threads())


# --------------------------------------------------------------------------------------
# weights
# --------------------------------------------------------------------------------------
def phi_dd(a, b):
    return lib().orc_phi_dd(float(a), float(b))


def chi_ph(x, y, T):
    return lib().orc_chi_ph(float(x), float(y), float(T))


def chi_pp(x, y, T):
    return lib().orc_chi_pp(float(x), float(y), float(T))


def chidot_ph(x, y, T):
    return lib().orc_chidot_ph(float(x), float(y), float(T))


def chidot_pp(x, y, T):
    return lib().orc_chidot_pp(float(x), float(y), float(T))


# --------------------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------------------
def geometry(m: Model):
    """Returns (xi[L*L], patch[L*L], anchor[N,2], min boundary margin in sectors)."""
    np_ = m.L * m.L
    xi = np.zeros(np_, np.float64)
    patch = np.zeros(np_, np.int32)
    anchor = np.zeros((m.N, 2), np.int32)
    margin = c_double(0.0)
    rc = lib().orc_geometry(ctypes.byref(m), _pd(xi), _pi(patch), _pi(anchor),
                            ctypes.byref(margin))
    if rc:
        raise ValueError("oracle geometry rejected N=%d L=%d" % (m.N, m.L))
    return xi, patch, anchor, margin.value


def transfer_counts(m: Model):
    a, b = c_int(0), c_int(0)
    if lib().orc_transfer_counts(ctypes.byref(m), ctypes.byref(a), ctypes.byref(b)):
        raise ValueError("bad model")
    return a.value, b.value


# --------------------------------------------------------------------------------------
# right-hand side
# --------------------------------------------------------------------------------------
def _zarg(Z, N):
    if Z is None:
        return None
    Z = np.ascontiguousarray(Z, np.float64)
    assert Z.shape == (N,)
    return Z


def rhs(m: Model, T, V, Z=None, nthreads=0, binned=False):
    N = m.N
    V = np.ascontiguousarray(V, np.float64).reshape(N * N * N)
    Z = _zarg(Z, N)
    out = np.zeros_like(V)
    fn = lib().orc_rhs_binned if binned else lib().orc_rhs
    if fn(ctypes.byref(m), float(T), _pd(Z), _pd(V), _pd(out), int(nthreads)):
        raise ValueError("oracle rhs rejected its arguments")
    return out.reshape(N, N, N)


def rhs_g(m: Model, T, g, V, Z=None, K=None, nthreads=0):
    """Interaction flow: dV/dg at temperature T and scale g (K: Katanin factors [N] on the
    single-scale line, App. A Step 3)."""
    N = m.N
    V = np.ascontiguousarray(V, np.float64).reshape(N * N * N)
    Z = _zarg(Z, N)
    out = np.zeros_like(V)
    if K is None:
        rc = lib().orc_rhs_g(ctypes.byref(m), float(T), float(g), _pd(Z), _pd(V), _pd(out),
                             int(nthreads))
    else:
        K = _zarg(K, N)
        rc = lib().orc_rhs_gk(ctypes.byref(m), float(T), float(g), _pd(Z), _pd(K), _pd(V),
                              _pd(out), int(nthreads))
    if rc:
        raise ValueError("oracle rhs_g rejected its arguments")
    return out.reshape(N, N, N)


def katanin(g, z_tab):
    """Katanin factors K and A_g on the nodes g of a Z table [n][N] (App. A, Eqs. K_definition
    and A_g_simple); returns (K [n][N], A [n][N])."""
    g = np.ascontiguousarray(g, np.float64)
    z = np.ascontiguousarray(z_tab, np.float64)
    n, N = z.shape
    K = np.zeros_like(z)
    A = np.zeros_like(z)
    if lib().orc_katanin(int(n), _pd(g), int(N), _pd(z), _pd(K), _pd(A)):
        raise ValueError("oracle katanin rejected its arguments")
    return K, A


def rhs_points_g(m: Model, T, g, V, abc, Z=None, nthreads=0):
    N = m.N
    V = np.ascontiguousarray(V, np.float64).reshape(N * N * N)
    Z = _zarg(Z, N)
    abc = np.ascontiguousarray(abc, np.int32).reshape(-1, 3)
    out = np.zeros(abc.shape[0], np.float64)
    if lib().orc_rhs_points_g(ctypes.byref(m), float(T), float(g), _pd(Z), _pd(V),
                              abc.shape[0], _pi(abc), _pd(out), int(nthreads)):
        raise ValueError("oracle rhs_points_g rejected its arguments")
    return out


def rhs_points(m: Model, T, V, abc, Z=None, nthreads=0):
    N = m.N
    V = np.ascontiguousarray(V, np.float64).reshape(N * N * N)
    Z = _zarg(Z, N)
    abc = np.ascontiguousarray(abc, np.int32).reshape(-1, 3)
    out = np.zeros(abc.shape[0], np.float64)
    if lib().orc_rhs_points(ctypes.byref(m), float(T), _pd(Z), _pd(V), abc.shape[0],
                            _pi(abc), _pd(out), int(nthreads)):
        raise ValueError("oracle rhs_points rejected its arguments")
    return out


# --------------------------------------------------------------------------------------
# flows
# --------------------------------------------------------------------------------------
def flowcfg(T0=1.0, T_end=0.01, integrator=0, n_steps=200, rtol=1e-6, atol=None, U=1.0,
            h0=0.0, h_min=0.0, v_max=20.0, z_lnT=None, z_tab=None, gflow=False, g_end=1.0,
            v_rel=100.0, binned=False, progress=False, k_tab=None):
    """Build a FlowCfg; keeps references to the Z arrays on the returned object.  gflow:
    interaction flow at the fixed temperature T0 from g = 0 to g_end (Z nodes in g), stopped
    when max|V| exceeds v_rel |U|.  binned: every right-hand side in the binned form (the
    same sums in another order).  progress: one line per Dormand-Prince step attempt on
    stderr.  k_tab: interaction flow only, Katanin factors [n_z][N] on the Z table's nodes."""
    if atol is None:
        atol = 1e-9 * max(1.0, abs(U))
    cfg = FlowCfg(float(T0), float(T_end), int(integrator), int(n_steps), float(rtol),
                  float(atol), float(h0), float(h_min), float(v_max), 0, None, None,
                  int(bool(gflow)), float(g_end), float(v_rel), int(bool(binned)),
                  int(bool(progress)), None)
    if z_tab is not None:
        z_lnT = np.ascontiguousarray(z_lnT, np.float64)
        z_tab = np.ascontiguousarray(z_tab, np.float64)
        assert z_tab.shape[0] == z_lnT.shape[0]
        cfg.n_z = z_lnT.shape[0]
        cfg.z_lnT = _pd(z_lnT)
        cfg.z_tab = _pd(z_tab)
        cfg._keep = (z_lnT, z_tab)
    if k_tab is not None:
        k_tab = np.ascontiguousarray(k_tab, np.float64)
        cfg.k_tab = _pd(k_tab)
        cfg._keep_k = k_tab
    return cfg


def flow(m: Model, cfg: FlowCfg, U, nthreads=0, max_trace=100000):
    N = m.N
    V = np.zeros(N * N * N, np.float64)
    res = Result()
    trace = np.zeros((max_trace, 2), np.float64)
    ntr = c_int(0)
    if lib().orc_flow(ctypes.byref(m), ctypes.byref(cfg), float(U), _pd(V), ctypes.byref(res),
                      _pd(trace), max_trace, ctypes.byref(ntr), int(nthreads)):
        raise ValueError("oracle flow rejected its arguments")
    return V.reshape(N, N, N), res.as_dict(), trace[: ntr.value].copy()


def flow_sync(m: Model, cfg: FlowCfg, U, nthreads=0):
    """Dormand-Prince flows from V = U[i] on one shared step schedule (an attempt is accepted
    only if every running flow accepts it; the next step follows from the largest error
    norm); cfg.atol <= 0 gives each flow 1e-9 max(1, |U_i|).  Returns (V [nf, N, N, N],
    [result dicts])."""
    N = m.N
    U = np.ascontiguousarray(np.atleast_1d(U), np.float64)
    nf = U.shape[0]
    V = np.zeros(nf * N ** 3, np.float64)
    res = (Result * nf)()
    if lib().orc_flow_sync(ctypes.byref(m), ctypes.byref(cfg), nf, _pd(U), _pd(V), res,
                           int(nthreads)):
        raise ValueError("oracle flow_sync rejected its arguments")
    return V.reshape(nf, N, N, N), [r.as_dict() for r in res]


def sigma2(m: Model, T, U, V=None, n_w=2048, nthreads=0):
    """Second-order self-energy on the real axis at each patch's representative point, bare
    (V None: U^2) or with the static vertex V; returns (w [n_w], Im [N, n_w], Re [N, n_w],
    Z [N])."""
    N = m.N
    w = np.zeros(n_w)
    im = np.zeros((N, n_w))
    re = np.zeros((N, n_w))
    Z = np.zeros(N)
    Vp = None
    if V is not None:
        Vp = np.ascontiguousarray(V, np.float64).reshape(N ** 3)
    if lib().orc_sigma2(ctypes.byref(m), float(T), float(U), _pd(Vp), int(n_w), _pd(w), _pd(im),
                        _pd(re), _pd(Z), int(nthreads)):
        raise ValueError("oracle sigma2 rejected its arguments")
    return w, im, re, Z


def kramers_kronig(w0, dw, im):
    im = np.ascontiguousarray(im, np.float64)
    re = np.zeros_like(im)
    lib().orc_kramers_kronig(im.shape[0], float(w0), float(dw), _pd(im), _pd(re))
    return re


def sigma_wmax(m: Model):
    return lib().orc_sigma_wmax(ctypes.byref(m))


def step(m: Model, cfg: FlowCfg, lnT, h, V, nthreads=0):
    """One step; returns (lnT, h_next, V, accepted, err)."""
    N = m.N
    V = np.ascontiguousarray(V, np.float64).reshape(N * N * N).copy()
    lt, hh, acc, err = c_double(lnT), c_double(h), c_int(0), c_double(0.0)
    if lib().orc_step(ctypes.byref(m), ctypes.byref(cfg), ctypes.byref(lt), ctypes.byref(hh),
                      _pd(V), ctypes.byref(acc), ctypes.byref(err), int(nthreads)):
        raise ValueError("oracle step rejected its arguments")
    return lt.value, hh.value, V.reshape(N, N, N), bool(acc.value), err.value


def dopri_tableau():
    c = np.zeros(7)
    a = np.zeros((7, 6))
    e = np.zeros(7)
    lib().orc_dopri_tableau(_pd(c), _pd(a), _pd(e))
    return c, a, e


def tc_interp(s_prev, m_prev, s_new, m_new, v_max):
    """The stop rule's crossing point, for tests: 1/max|V| linear in ln T."""
    return s_prev + (1.0 / m_prev - 1.0 / v_max) * (s_new - s_prev) / (
        1.0 / m_prev - 1.0 / m_new)


def gc_interp(g_prev, m_prev, g_new, m_new, v_max):
    """The interaction flow's crossing point, for tests: 1/max|V| linear in g^2."""
    u = g_prev ** 2 + (1.0 / m_prev - 1.0 / v_max) * (g_new ** 2 - g_prev ** 2) / (
        1.0 / m_prev - 1.0 / m_new)
    return math.sqrt(u)
