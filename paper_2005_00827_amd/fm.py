"""ctypes binding of libfmflow (include/fm_flow.h): argument marshalling only.

Every step of the flow runs in the library's HIP kernels; PyTorch supplies device memory
(the workspace and the state tensors) and the stream.  There is no fallback: when the
library is missing, :func:`load` raises.
"""
from __future__ import annotations

import ctypes
import math
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_size_t, c_uint, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfmflow.so")

FM_OK, FM_EINVAL, FM_ENOMEM, FM_EDEVICE, FM_ESTATE = 0, -1, -2, -3, -4
GEOM_ANGULAR, GEOM_IDENTITY, GEOM_SHELLS = 0, 1, 2
GEOMETRIES = {"angular": GEOM_ANGULAR, "identity": GEOM_IDENTITY, "shells": GEOM_SHELLS}
RK4_FIXED, RK45_DOPRI = 0, 1
FP64, FP32, FP32_BF16MFMA, FP64_DIRECT, FP32_BF16X3 = 0, 1, 2, 3, 4
CH_PP, CH_CR, CH_D, CH_ALL = 1, 2, 4, 7
RUNNING, DIVERGED, NONFINITE, REACHED_TEND, STEPFAIL = 0, 1, 2, 3, 4

PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": FP32_BF16MFMA, "fp64_direct": FP64_DIRECT,
              "bf16x3": FP32_BF16X3}
INTEGRATORS = {"rk4": RK4_FIXED, "rk45": RK45_DOPRI}

# every entry point declared in include/fm_flow.h
EXPORTS = ("fm_flow_workspace_bytes", "fm_flow_init", "fm_flow_rhs", "fm_flow_rhs_g",
           "fm_flow_step", "fm_flow_run_batch", "fm_flow_tstar", "fm_geometry_query",
           "fm_flow_set_timing", "fm_flow_timings", "fm_flow_kernel_time", "fm_flow_destroy",
           "fm_last_error", "fm_flow_rhs_static", "fm_flow_z", "fm_sigma_wmax",
           "fm_katanin_table")
SIGMA_NW = 2048
FLOWS = {"temperature": 0, "interaction": 1}


class Config(ctypes.Structure):
    _fields_ = [("t", c_double), ("tp", c_double), ("mu", c_double), ("U", c_double),
                ("geometry", c_int), ("N", c_int), ("L", c_int),
                ("T0", c_double), ("T_end", c_double),
                ("integrator", c_int), ("n_steps", c_int),
                ("rtol", c_double), ("atol", c_double), ("h0", c_double), ("h_min", c_double),
                ("v_max", c_double), ("channels", c_uint), ("precision", c_int),
                ("n_zT", c_int), ("z_lnT", POINTER(c_double)), ("z_table", POINTER(c_double)),
                ("stream", c_void_p), ("max_batch", c_int), ("tile_rows", c_int),
                ("flow", c_int), ("g_end", c_double), ("v_rel", c_double), ("y_kernel", c_int),
                ("sync_batch", c_int), ("n_shells", c_int), ("shell_edges", POINTER(c_double)),
                ("k_table", POINTER(c_double)), ("phase1_variant", c_int),
                ("sym_state", c_int)]


class Result(ctypes.Structure):
    _fields_ = [("T_c", c_double), ("T_final", c_double), ("max_abs_V", c_double),
                ("status", c_int), ("n_accepted", c_int), ("n_rejected", c_int),
                ("n_rhs", c_int), ("g_c", c_double), ("U_star", c_double),
                ("g_final", c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class FmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libfmflow error %d: %s" % (code, msg))
        self.code = code


_lib = None


def load():
    """Loads libfmflow.so from the package directory; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libfmflow.so is not built (run __graft_entry__.build() or "
                           "python paper_2005_00827_amd/build.py); no fallback exists")
    L = ctypes.CDLL(LIB_PATH)
    pc, pr = POINTER(Config), POINTER(Result)
    pd, pi = POINTER(c_double), POINTER(c_int)
    sig = {
        "fm_flow_workspace_bytes": (c_int, [pc, POINTER(c_size_t)]),
        "fm_flow_init": (c_int, [pc, c_void_p, c_size_t, POINTER(c_void_p)]),
        "fm_flow_rhs": (c_int, [c_void_p, c_int, pd, c_void_p, c_void_p]),
        "fm_flow_rhs_g": (c_int, [c_void_p, c_int, pd, pd, c_void_p, c_void_p]),
        "fm_flow_tstar": (c_int, [c_void_p, c_int, pd, c_double, c_double, c_double, pd, pi]),
        "fm_flow_step": (c_int, [c_void_p, c_int, pd, pd, c_void_p, pi]),
        "fm_flow_run_batch": (c_int, [c_void_p, c_int, pd, pd, pd, pd, c_void_p, pr]),
        "fm_geometry_query": (c_int, [pc, pd, pi, pi, pi, pi, pd, pi]),
        "fm_flow_set_timing": (c_int, [c_void_p, c_int]),
        "fm_flow_timings": (c_int, [c_void_p, POINTER(c_char_p), pd, pi, c_int]),
        "fm_flow_kernel_time": (c_int, [c_void_p, c_int, c_int, c_int, pd]),
        "fm_flow_rhs_static": (c_int, [pc, c_int, pd, c_void_p, c_void_p]),
        "fm_flow_z": (c_int, [c_void_p, c_double, c_double, c_void_p, pd, pd, pd]),
        "fm_sigma_wmax": (c_double, [pc]),
        "fm_katanin_table": (c_int, [c_int, pd, c_int, pd, pd, pd, pd]),
        "fm_flow_destroy": (None, [c_void_p]),
        "fm_last_error": (c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype, fn.argtypes = res, args
    _lib = L
    return L


def _check(rc):
    if rc != FM_OK:
        raise FmError(rc, load().fm_last_error().decode())


def _pd(a):
    return None if a is None else a.ctypes.data_as(POINTER(c_double))


def _pi(a):
    return None if a is None else a.ctypes.data_as(POINTER(c_int))


def make_config(N, L, U=1.0, t=1.0, tp=0.0, mu=0.0, geometry="angular", T0=1.0, T_end=0.01,
                integrator="rk4", n_steps=200, rtol=0.0, atol=0.0, h0=0.0, h_min=0.0,
                v_max=20.0, channels=CH_ALL, precision="fp64", z_lnT=None, z_table=None,
                stream=None, max_batch=1, tile_rows=0, flow="temperature", g_end=0.0,
                v_rel=0.0, y_kernel=0, sync_batch=False, n_shells=0, shell_edges=None,
                k_table=None, phase1_variant=0, sym_state=False):
    cfg = Config()
    cfg.t, cfg.tp, cfg.mu, cfg.U = float(t), float(tp), float(mu), float(U)
    cfg.geometry = GEOMETRIES[geometry] if isinstance(geometry, str) else int(geometry)
    cfg.N, cfg.L = int(N), int(L)
    cfg.T0, cfg.T_end = float(T0), float(T_end)
    cfg.integrator = INTEGRATORS[integrator] if isinstance(integrator, str) else int(integrator)
    cfg.n_steps = int(n_steps)
    cfg.rtol, cfg.atol, cfg.h0, cfg.h_min = float(rtol), float(atol), float(h0), float(h_min)
    cfg.v_max = float(v_max)
    cfg.channels = int(channels)
    cfg.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    keep = []
    if z_table is not None:
        zl = np.ascontiguousarray(z_lnT, np.float64)
        zt = np.ascontiguousarray(z_table, np.float64)
        if zt.shape != (zl.shape[0], int(N)):
            raise ValueError("z_table must be [n_zT, N]")
        cfg.n_zT = zl.shape[0]
        cfg.z_lnT, cfg.z_table = _pd(zl), _pd(zt)
        keep = [zl, zt]
    cfg.stream = stream
    cfg.max_batch = int(max_batch)
    cfg.tile_rows = int(tile_rows)
    cfg.flow = FLOWS[flow] if isinstance(flow, str) else int(flow)
    cfg.g_end = float(g_end)
    cfg.v_rel = float(v_rel)
    cfg.y_kernel = int(y_kernel)
    cfg.sync_batch = int(sync_batch)
    cfg.phase1_variant = int(phase1_variant)
    cfg.sym_state = int(sym_state)
    cfg.n_shells = int(n_shells)
    if shell_edges is not None:
        se = np.ascontiguousarray(shell_edges, np.float64)
        if se.shape != ((int(n_shells) - 1) // 2,):
            raise ValueError("shell_edges must hold (n_shells - 1) / 2 values")
        cfg.shell_edges = _pd(se)
        keep = keep + [se]
    if k_table is not None:
        kt = np.ascontiguousarray(k_table, np.float64)
        if z_table is None or kt.shape != (cfg.n_zT, int(N)):
            raise ValueError("k_table must be [n_zT, N], on the Z table's nodes")
        cfg.k_table = _pd(kt)
        keep = keep + [kt]
    cfg._keep = keep
    return cfg


def katanin_table(g, z_table):
    """fm_katanin_table: Katanin factors K, A_g and its per-node bounds from Z on the scales
    g (host-only); returns (K [n, N], A [n, N], A_minmax [n, 2])."""
    g = np.ascontiguousarray(g, np.float64)
    z = np.ascontiguousarray(z_table, np.float64)
    n, N = z.shape
    if g.shape != (n,):
        raise ValueError("g must hold one scale per table row")
    K, A, mm = np.zeros_like(z), np.zeros_like(z), np.zeros((n, 2))
    _check(load().fm_katanin_table(int(n), _pd(g), int(N), _pd(z), _pd(K), _pd(A), _pd(mm)))
    return K, A, mm


def geometry_query(cfg: Config):
    """Host-only: (xi[L*L], patch[L*L], anchor[N,2], n_pp, n_ph, margin)."""
    np_ = cfg.L * cfg.L
    xi = np.zeros(np_, np.float64)
    patch = np.zeros(np_, np.int32)
    anchor = np.zeros((cfg.N, 2), np.int32)
    npp, nph, mg = c_int(0), c_int(0), c_double(0)
    _check(load().fm_geometry_query(ctypes.byref(cfg), _pd(xi), _pi(patch), _pi(anchor),
                                    ctypes.byref(npp), ctypes.byref(nph), ctypes.byref(mg),
                                    None))
    return xi, patch, anchor, npp.value, nph.value, mg.value


def representative_counts(cfg: Config):
    """Host-only: numbers of particle-particle and particle-hole transfers binned by phase 1."""
    rep = np.zeros(2, np.int32)
    _check(load().fm_geometry_query(ctypes.byref(cfg), None, None, None, None, None, None,
                                    _pi(rep)))
    return int(rep[0]), int(rep[1])


def workspace_bytes(cfg: Config) -> int:
    n = c_size_t(0)
    _check(load().fm_flow_workspace_bytes(ctypes.byref(cfg), ctypes.byref(n)))
    return n.value


class Flow:
    """A library handle plus its torch-allocated workspace."""

    def __init__(self, device=None, **kw):
        import torch
        self.torch = torch
        self.device = torch.device(device or "cuda:0")
        if "stream" not in kw or kw["stream"] is None:
            kw["stream"] = torch.cuda.current_stream(self.device).cuda_stream
        self.cfg = make_config(**kw)
        self.N = self.cfg.N
        self.nbytes = workspace_bytes(self.cfg)
        self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        h = c_void_p(0)
        _check(load().fm_flow_init(ctypes.byref(self.cfg), c_void_p(self.workspace.data_ptr()),
                                   self.nbytes, ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            load().fm_flow_destroy(self.h)
            self.h = c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _state(self, V, batch=None):
        t = self.torch
        if not (isinstance(V, t.Tensor) and V.is_cuda and V.dtype == t.float64 and V.is_contiguous()):
            raise TypeError("V must be a contiguous float64 CUDA tensor")
        n3 = self.N ** 3
        if V.numel() % n3:
            raise ValueError("V must hold batch x N^3 values")
        return V.numel() // n3

    def rhs(self, T, V, out=None):
        """dV/d ln T at temperatures T[batch] for states V [batch, N, N, N] (float64 CUDA)."""
        b = self._state(V)
        T = np.ascontiguousarray(np.atleast_1d(T), np.float64)
        if T.shape[0] != b:
            raise ValueError("one temperature per state")
        if out is None:
            out = self.torch.empty_like(V)
        _check(load().fm_flow_rhs(self.h, b, _pd(T), c_void_p(V.data_ptr()),
                                  c_void_p(out.data_ptr())))
        return out

    def rhs_g(self, T, g, V, out=None):
        """Interaction flow: dV/dg at temperatures T[batch] and scales g[batch]."""
        b = self._state(V)
        T = np.ascontiguousarray(np.atleast_1d(T), np.float64)
        g = np.ascontiguousarray(np.atleast_1d(g), np.float64)
        if T.shape[0] != b or g.shape[0] != b:
            raise ValueError("one temperature and one g per state")
        if out is None:
            out = self.torch.empty_like(V)
        _check(load().fm_flow_rhs_g(self.h, b, _pd(T), _pd(g), c_void_p(V.data_ptr()),
                                    c_void_p(out.data_ptr())))
        return out

    def tstar(self, U, T_lo, T_hi, rtol=1e-4):
        """Interaction flow: T*(U) per coupling by bisection in ln T; returns (T*, status)."""
        U = np.ascontiguousarray(np.atleast_1d(U), np.float64)
        out = np.zeros(U.shape[0], np.float64)
        st = np.zeros(U.shape[0], np.int32)
        _check(load().fm_flow_tstar(self.h, U.shape[0], _pd(U), float(T_lo), float(T_hi),
                                    float(rtol), _pd(out), _pi(st)))
        return out, st

    def z(self, T, U, V=None, spectra=False):
        """Quasi-particle weights Z[N] from the second-order self-energy on the real axis at
        temperature T (bare U when V is None, else the static vertex V [N, N, N] float64 CUDA);
        with spectra, also (w [SIGMA_NW], Im Sigma [N, SIGMA_NW], Re Sigma [N, SIGMA_NW])."""
        N = self.N
        Z = np.zeros(N, np.float64)
        im = re = None
        if spectra:
            im = np.zeros((N, SIGMA_NW), np.float64)
            re = np.zeros((N, SIGMA_NW), np.float64)
        vp = None
        if V is not None:
            if self._state(V) != 1:
                raise ValueError("one vertex V")
            vp = c_void_p(V.data_ptr())
        _check(load().fm_flow_z(self.h, float(T), float(U), vp, _pd(Z), _pd(im), _pd(re)))
        if not spectra:
            return Z
        w0 = load().fm_sigma_wmax(ctypes.byref(self.cfg))
        w = -w0 + 2.0 * w0 * np.arange(SIGMA_NW) / (SIGMA_NW - 1)
        return Z, w, im, re

    def step(self, lnT, h, V):
        """One integrator step in place on V; returns (lnT, h, accepted) arrays (for the
        interaction flow: g, its step, accepted)."""
        b = self._state(V)
        lnT = np.ascontiguousarray(np.atleast_1d(lnT), np.float64).copy()
        hh = np.ascontiguousarray(np.atleast_1d(h), np.float64).copy()
        acc = np.zeros(b, np.int32)
        _check(load().fm_flow_step(self.h, b, _pd(lnT), _pd(hh), c_void_p(V.data_ptr()),
                                   _pi(acc)))
        return lnT, hh, acc.astype(bool)

    def run_batch(self, U, T0, z_lnT=None, z_tables=None, return_V=False):
        U = np.ascontiguousarray(np.atleast_1d(U), np.float64)
        T0 = np.ascontiguousarray(np.atleast_1d(T0), np.float64)
        n = U.shape[0]
        zl = None if z_lnT is None else np.ascontiguousarray(z_lnT, np.float64)
        zt = None if z_tables is None else np.ascontiguousarray(z_tables, np.float64)
        if (zl is None) != (zt is None):
            raise ValueError("give both per-flow Z arrays or neither")
        if zt is not None:
            nz = self.cfg.n_zT
            if zl.shape != (n, nz) or zt.shape != (n, nz, self.N):
                raise ValueError("per-flow Z arrays must be [n_flows, n_zT] and "
                                 "[n_flows, n_zT, N] with the configured n_zT = %d" % nz)
        res = (Result * n)()
        Vout = None
        if return_V:
            Vout = self.torch.empty((n, self.N, self.N, self.N), dtype=self.torch.float64,
                                    device=self.device)
        _check(load().fm_flow_run_batch(self.h, n, _pd(U), _pd(T0), _pd(zl), _pd(zt),
                                        c_void_p(Vout.data_ptr()) if Vout is not None else None,
                                        res))
        out = [r.as_dict() for r in res]
        return (out, Vout) if return_V else out

    def set_timing(self, on=True):
        _check(load().fm_flow_set_timing(self.h, int(bool(on))))

    def kernel_time(self, group, batch=1, reps=50):
        """Average launch duration (ms) of kernel group 0 (stage + phase 1 of a step's stage
        nodes), 1 (phase 2a), 2 (phase 2b) or 3 (stage alone), replayed back to back on the
        handle's current state."""
        out = c_double(0.0)
        _check(load().fm_flow_kernel_time(self.h, int(group), int(batch), int(reps),
                                          ctypes.byref(out)))
        return out.value

    def timings(self):
        names = (c_char_p * 16)()
        ms = np.zeros(16, np.float64)
        n = np.zeros(16, np.int32)
        k = load().fm_flow_timings(self.h, names, _pd(ms), _pi(n), 16)
        if k < 0:
            _check(k)
        return {names[i].decode(): (float(ms[i]), int(n[i])) for i in range(k)}


def rhs_static(T, V, out=None, device=None, **kw):
    """fm_flow_rhs_static: dV/d ln T like Flow.rhs, with the library's static device array as
    the workspace (no allocation; one flow of the N = 48, L = 128 workloads fits).  kw as
    make_config; the stream defaults to torch's current stream."""
    import torch
    dev = torch.device(device or "cuda:0")
    if kw.get("stream") is None:
        kw["stream"] = torch.cuda.current_stream(dev).cuda_stream
    cfg = make_config(**kw)
    if not (isinstance(V, torch.Tensor) and V.is_cuda and V.dtype == torch.float64
            and V.is_contiguous()):
        raise TypeError("V must be a contiguous float64 CUDA tensor")
    n3 = cfg.N ** 3
    if V.numel() % n3:
        raise ValueError("V must hold batch x N^3 values")
    b = V.numel() // n3
    T = np.ascontiguousarray(np.atleast_1d(T), np.float64)
    if T.shape[0] != b:
        raise ValueError("one temperature per state")
    if out is None:
        out = torch.empty_like(V)
    _check(load().fm_flow_rhs_static(ctypes.byref(cfg), b, _pd(T), c_void_p(V.data_ptr()),
                                     c_void_p(out.data_ptr())))
    return out


def hubbard_flow(N, L, **kw):
    return Flow(N=N, L=L, **kw)


def lnT_grid(T0, T_end, n):
    return [math.log(T0) + i * (math.log(T_end) - math.log(T0)) / n for i in range(n + 1)]
