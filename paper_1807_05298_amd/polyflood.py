"""Thin ctypes binding of the HIP library (C ABI in ``include/polyflood.h``).

Argument marshalling only: every step of the Newton iteration runs in the
library's HIP kernels.  PyTorch supplies the device workspace (one uint8
tensor) and the stream.  Importing this module fails loudly when the built
library is missing.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# PF_LIB may name another build of the same library (e.g. a variant built
# for a timing comparison); by default the in-tree build is loaded.
LIB_PATH = os.environ.get("PF_LIB") or os.path.join(_HERE, "libpolyflood.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"HIP library not built: {LIB_PATH} is missing "
                      "(run paper_1807_05298_amd/build_lib.py or __graft_entry__.build())")

# torch first: its bundled HIP runtime carries the same soname as the one the
# library links, so loading torch before the library makes both share one
# runtime (the other order loads a second runtime that sees no device).
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

PF_OK, PF_EINVAL, PF_ENOMEM, PF_ENONCONV, PF_ELINEAR, PF_EHIP, PF_EBUSY = range(7)
# kernels that pf_profile_begin can time (PF_K_* in the header)
(PF_K_ASSEMBLE, PF_K_SPMV, PF_K_ZLINE, PF_K_MDOT, PF_K_MUPDATE, PF_K_ILU, PF_K_STAGE_RESID, PF_K_RED_SPMV,
 PF_K_BLACK_SPMV) = range(1, 10)
PREC_FP64, PREC_MIXED = 0, 1
CPR_PF, CPR_FP = 0, 1
SMOOTH_BJAC, SMOOTH_RBILU0 = 0, 1
WELL_Z, WELL_X = 0, 1

_d = ctypes.c_double
_i = ctypes.c_int32
_pd = ctypes.POINTER(ctypes.c_double)


class Grid(ctypes.Structure):
    _fields_ = [("nx", _i), ("ny", _i), ("nz", _i), ("dx", _d), ("dy", _d), ("dz", _d), ("top_depth", _d)]


class Rock(ctypes.Structure):
    _fields_ = [("poro", _pd), ("kx", _pd), ("ky", _pd), ("kz", _pd), ("cr", _d), ("p_ref", _d)]


TABLE_MAX = 16
_tab = _d * TABLE_MAX


class Fluid(ctypes.Structure):
    _fields_ = [(k, _d) for k in ("rho_w0", "rho_o0", "c_w", "c_o", "mu_w", "mu_o", "swc", "sor",
                                   "n_w", "n_o", "krw0", "kro0", "gravity")] + \
               [("n_pc", _i), ("reserved", _i), ("pc_s", _tab), ("pc_v", _tab)]


class Polymer(ctypes.Structure):
    _fields_ = [(k, _d) for k in ("a1", "a2", "omega", "c_max", "ads_max", "ads_b", "rrf", "ipv")] + \
               [("mix_rule", _i), ("n_ads", _i), ("mu_p_ref", _d), ("n_visc", _i), ("reserved", _i),
                ("ads_c", _tab), ("ads_a", _tab), ("visc_c", _tab), ("visc_m", _tab),
                ("ads_res", _d), ("n_kperm", _i), ("reserved2", _i),
                ("kperm_k", _tab), ("kperm_rrf", _tab), ("kperm_admax", _tab)]


def _table(points):
    """(n, x[16], y[16]) of a table given as (x, y) points (None: empty)."""
    x, y = _tab(), _tab()
    pts = list(points or [])
    if len(pts) > TABLE_MAX:
        raise ValueError(f"at most {TABLE_MAX} table points")
    for k, (a, b) in enumerate(pts):
        x[k], y[k] = float(a), float(b)
    return len(pts), x, y


class WellC(ctypes.Structure):
    _fields_ = [("ix", _i), ("iy", _i), ("k_top", _i), ("k_bot", _i), ("is_injector", _i), ("control", _i),
                ("target", _d), ("c_inj", _d), ("rw", _d), ("skin", _d), ("bhp_limit", _d),
                ("direction", _i), ("ix_last", _i)]


class ModelDesc(ctypes.Structure):
    _fields_ = [("grid", Grid), ("rock", Rock), ("fluid", Fluid), ("polymer", Polymer),
                ("n_wells", _i), ("wells", ctypes.POINTER(WellC))]


class SolverOpts(ctypes.Structure):
    _fields_ = [("precision", _i), ("cpr_order", _i), ("smoother", _i), ("restart", _i),
                ("max_lin_it", _i), ("max_newton", _i), ("max_cuts", _i), ("inexact", _i),
                ("tol_res", _d), ("tol_upd", _d), ("lin_tol", _d), ("ds_max", _d),
                ("mg_pre", _i), ("mg_post", _i), ("mg_coarse", _i), ("reorth", _i),
                ("mg_cycles", _i), ("zline_len", _i), ("mg_pre_small", _i), ("mg_small_cells", _i),
                ("dt_init", _d)]


class StepStats(ctypes.Structure):
    _fields_ = [("newton_its", _i), ("lin_its", _i), ("cuts", _i), ("converged", _i),
                ("dt_taken", _d), ("res_norm", _d), ("upd_norm", _d), ("lin_rel", _d),
                ("t_assemble", _d), ("t_setup", _d), ("t_solve", _d), ("t_total", _d),
                ("well_switches", _i), ("reserved", _i)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp = ctypes.c_void_p
_lib.pf_default_opts.argtypes = [ctypes.POINTER(SolverOpts)]
_lib.pf_workspace_size.argtypes = [ctypes.POINTER(ModelDesc), ctypes.POINTER(SolverOpts), ctypes.POINTER(ctypes.c_size_t)]
_lib.pf_create.argtypes = [ctypes.POINTER(ModelDesc), ctypes.POINTER(SolverOpts), _vp, ctypes.c_size_t, _vp,
                           ctypes.POINTER(_vp)]
_lib.pf_create_static.argtypes = [ctypes.POINTER(ModelDesc), ctypes.POINTER(SolverOpts), _vp, ctypes.POINTER(_vp)]
_lib.pf_destroy.argtypes = [_vp]
_lib.pf_set_equilibrium_state.argtypes = [_vp, _d, _d, _d]
_lib.pf_set_opts.argtypes = [_vp, ctypes.POINTER(SolverOpts)]
_lib.pf_set_state.argtypes = [_vp, _vp, _vp, _vp, _vp]
_lib.pf_get_state.argtypes = [_vp, _vp, _vp, _vp, _vp]
_lib.pf_begin_step.argtypes = [_vp]
_lib.pf_newton_iteration.argtypes = [_vp, _d, ctypes.POINTER(StepStats)]
_lib.pf_step.argtypes = [_vp, _d, ctypes.POINTER(StepStats)]
_lib.pf_assemble.argtypes = [_vp, _d, _vp, _vp, _vp]
_lib.pf_spmv.argtypes = [_vp, _vp, _vp]
_lib.pf_linear_solve.argtypes = [_vp, _vp, _d, _vp, ctypes.POINTER(_i), ctypes.POINTER(_d)]
_lib.pf_get_static.argtypes = [_vp] + [_vp] * 8
_lib.pf_n_perf.restype = ctypes.c_int64
_lib.pf_n_perf.argtypes = [_vp]
_lib.pf_last_error.restype = ctypes.c_char_p
_lib.pf_profile_begin.argtypes = [_vp, _i, _i]
_lib.pf_server_create.argtypes = [_vp, ctypes.c_size_t, _i, _i, ctypes.POINTER(_vp)]
_lib.pf_fusion_create.argtypes = [_vp, ctypes.POINTER(_vp)]
_lib.pf_fusion_join.argtypes = [_vp, _vp]
_lib.pf_fusion_leave.argtypes = [_vp]
_lib.pf_fusion_step.argtypes = [_vp, _i, _vp, _vp, _vp]
_lib.pf_fusion_stats.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                 ctypes.POINTER(ctypes.c_int64)]
_lib.pf_fusion_destroy.argtypes = [_vp]
_lib.pf_server_submit.argtypes = [_vp, ctypes.POINTER(ModelDesc), ctypes.POINTER(SolverOpts), _vp, _vp, _vp, _vp, _i,
                                  _vp, ctypes.POINTER(ctypes.c_uint64)]
_lib.pf_server_poll.argtypes = [_vp, ctypes.c_uint64, ctypes.POINTER(_i), _vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.pf_server_wait.argtypes = [_vp, ctypes.c_uint64]
_lib.pf_server_release.argtypes = [_vp, ctypes.c_uint64]
_lib.pf_server_info.argtypes = [_vp, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i),
                                ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
_lib.pf_server_destroy.argtypes = [_vp]
_lib.pf_pressure_level.restype = _i
_lib.pf_pressure_level.argtypes = [_vp, _i, _vp, _vp]
_lib.pf_pressure_smooth.argtypes = [_vp, _i, _i, _i, _vp, _vp]
_lib.pf_pressure_vcycle.argtypes = [_vp, _vp, _vp]
_lib.pf_smoother_apply.argtypes = [_vp, _vp, _vp]
_lib.pf_precond_apply.argtypes = [_vp, _vp, _vp, _vp]
_lib.pf_profile_end.argtypes = [_vp, ctypes.POINTER(_i), ctypes.POINTER(_d)]
_lib.pf_well_status.argtypes = [_vp, _vp, _vp, _vp, _vp]
_lib.pf_set_well_operation.argtypes = [_vp, _i, _i, _d, _d, _d]

EXPORTED = ["pf_default_opts", "pf_workspace_size", "pf_create", "pf_destroy", "pf_set_opts", "pf_set_state",
            "pf_get_state", "pf_begin_step", "pf_newton_iteration", "pf_step", "pf_assemble", "pf_spmv",
            "pf_linear_solve", "pf_get_static", "pf_n_perf", "pf_last_error", "pf_profile_begin", "pf_profile_end",
            "pf_pressure_level", "pf_pressure_smooth", "pf_pressure_vcycle", "pf_smoother_apply",
            "pf_precond_apply", "pf_server_create", "pf_server_submit", "pf_server_poll",
            "pf_server_wait", "pf_server_release", "pf_server_info", "pf_server_destroy", "pf_well_status", "pf_set_well_operation",
            "pf_fusion_create", "pf_fusion_join", "pf_fusion_leave", "pf_fusion_step", "pf_fusion_stats",
            "pf_fusion_destroy"]


STATIC_WORKSPACE_BYTES = 64 << 20     # PF_STATIC_WORKSPACE_BYTES of polyflood.h


class PFError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"polyflood status {status}: {msg}")
        self.status = status


def _check(st: int):
    if st != PF_OK:
        raise PFError(st, _lib.pf_last_error().decode())


def default_opts(**kw) -> SolverOpts:
    o = SolverOpts()
    _lib.pf_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class _Desc:
    """A pf_model_desc for a ``inputs.Case`` plus the arrays it points to."""

    def __init__(self, case):
        self.keep = [_f64(case.poro), _f64(case.kx), _f64(case.ky), _f64(case.kz)]
        g = Grid(case.nx, case.ny, case.nz, case.dx, case.dy, case.dz, case.top)
        r = Rock(*(a.ctypes.data_as(_pd) for a in self.keep), case.cr, case.p_ref)
        f = case.fluid
        npc, pcs, pcv = _table(getattr(f, "pc_table", None))
        fl = Fluid(f.rho_w0, f.rho_o0, f.c_w, f.c_o, f.mu_w, f.mu_o, f.swc, f.sor, f.n_w, f.n_o,
                   f.krw0, f.kro0, f.gravity, npc, 0, pcs, pcv)
        p = case.polymer
        na, ac, aa = _table(getattr(p, "ads_table", None))
        nv, vc, vm = _table(getattr(p, "visc_table", None))
        kp = list(getattr(p, "kperm_table", None) or [])
        if len(kp) > TABLE_MAX:
            raise ValueError(f"at most {TABLE_MAX} table points")
        kk, kr, ka = _tab(), _tab(), _tab()
        for k, (a, b, c) in enumerate(kp):
            kk[k], kr[k], ka[k] = float(a), float(b), float(c)
        po = Polymer(p.a1, p.a2, p.omega, p.c_max, p.ads_max, p.ads_b, p.rrf, p.ipv,
                     int(getattr(p, "mix_rule", 0)), na, float(getattr(p, "mu_p_ref", 0.0)), nv, 0,
                     ac, aa, vc, vm, float(getattr(p, "ads_res", 0.0) or 0.0), len(kp), 0, kk, kr, ka)
        nw = len(case.wells)
        self.wells = (WellC * max(nw, 1))()
        for k, w in enumerate(case.wells):
            d = int(getattr(w, "direction", 0))
            self.wells[k] = WellC(w.ix, w.iy, w.k_top, w.k_bot, int(w.injector), w.control, w.target,
                                  w.c_inj, w.rw, w.skin, float(getattr(w, "bhp_limit", 0.0) or 0.0),
                                  d, int(w.ix_last) if d == WELL_X else int(w.ix))
        self.desc = ModelDesc(g, r, fl, po, nw, ctypes.cast(self.wells, ctypes.POINTER(WellC)))


def workspace_size(case, opts: Optional[SolverOpts] = None) -> int:
    d = _Desc(case)
    o = opts or default_opts()
    n = ctypes.c_size_t(0)
    _check(_lib.pf_workspace_size(ctypes.byref(d.desc), ctypes.byref(o), ctypes.byref(n)))
    return int(n.value)


class Simulator:
    """One reservoir model on one GPU.  State vectors in the library's plane
    layout: P, S, C (N each) and Pb (n_wells)."""

    def __init__(self, case, opts: Optional[SolverOpts] = None, device: str = "cuda:0", stream=None,
                 static_workspace: bool = False):
        """static_workspace: create through pf_create_static (the library's
        fixed per-GPU workspace; no device memory is allocated)."""
        import torch
        self.case = case
        self.n = case.n
        self.nw = len(case.wells)
        self.nv = 3 * self.n + self.nw
        self._ops = {}                   # well operations changed by schedule events
        self.opts = opts or default_opts()
        self._d = _Desc(case)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = _vp()
        if static_workspace:
            self.ws = None
            with torch.cuda.device(self.device):
                _check(_lib.pf_create_static(ctypes.byref(self._d.desc), ctypes.byref(self.opts),
                                             _vp(self.stream.cuda_stream), ctypes.byref(h)))
        else:
            nbytes = workspace_size(case, self.opts)
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            if self.ws.data_ptr() % 256:
                raise RuntimeError("workspace tensor is not 256-byte aligned")
            _check(_lib.pf_create(ctypes.byref(self._d.desc), ctypes.byref(self.opts), _vp(self.ws.data_ptr()),
                                  nbytes, _vp(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        self.n_perf = int(_lib.pf_n_perf(self.h))
        self.set_state(case.P0, case.S0, case.C0, case.Pb0)

    def close(self):
        if getattr(self, "h", None):
            _lib.pf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def workspace_bytes(self) -> int:
        return int(self.ws.numel()) if self.ws is not None else STATIC_WORKSPACE_BYTES

    def set_opts(self, opts: SolverOpts):
        _check(_lib.pf_set_opts(self.h, ctypes.byref(opts)))
        self.opts = opts

    def set_state(self, P, S, C, Pb):
        P, S, C = _f64(P), _f64(S), _f64(C)
        Pb = _f64(Pb if len(Pb) else np.zeros(1))
        _check(_lib.pf_set_state(self.h, P.ctypes.data, S.ctypes.data, C.ctypes.data, Pb.ctypes.data))

    def set_equilibrium_state(self, datum_depth: float, datum_pressure: float, fwl_depth: float):
        """Capillary-gravity equilibrium initial state computed by the library."""
        _check(_lib.pf_set_equilibrium_state(self.h, float(datum_depth), float(datum_pressure), float(fwl_depth)))

    def get_state(self):
        P, S, C = np.empty(self.n), np.empty(self.n), np.empty(self.n)
        Pb = np.empty(max(self.nw, 1))
        _check(_lib.pf_get_state(self.h, P.ctypes.data, S.ctypes.data, C.ctypes.data, Pb.ctypes.data))
        return P, S, C, Pb[:self.nw]

    def begin_step(self):
        _check(_lib.pf_begin_step(self.h))

    def set_well_operation(self, well: int, control: int, target: float, c_inj: float = 0.0,
                           bhp_limit: float = 0.0):
        """Change a well's operation between timesteps."""
        _check(_lib.pf_set_well_operation(self.h, int(well), int(control), float(target), float(c_inj),
                                          float(bhp_limit)))

    def apply_events(self, case, step: int):
        """Apply the case's well-operation changes scheduled before ``step``."""
        for k, w, ch in getattr(case, "events", []):
            if k == step:
                W = case.wells[w]
                op = dict(control=W.control, target=W.target, c_inj=W.c_inj, bhp_limit=W.bhp_limit)
                op.update(self._ops.get(w, {}))
                op.update(ch)
                self._ops[w] = op
                self.set_well_operation(w, **op)

    def well_status(self) -> dict:
        """Active control, its target and surface water/oil rates of every well
        at the last assembled state."""
        nw = max(self.nw, 1)
        ctrl = np.zeros(nw, dtype=np.int32)
        target, qw, qo = np.zeros(nw), np.zeros(nw), np.zeros(nw)
        _check(_lib.pf_well_status(self.h, ctrl.ctypes.data, target.ctypes.data, qw.ctypes.data, qo.ctypes.data))
        return dict(ctrl=ctrl[:self.nw], target=target[:self.nw], qw=qw[:self.nw], qo=qo[:self.nw])

    def newton_iteration(self, dt: float) -> dict:
        st = StepStats()
        _check(_lib.pf_newton_iteration(self.h, float(dt), ctypes.byref(st)))
        return st.as_dict()

    def step(self, dt: float) -> dict:
        st = StepStats()
        _check(_lib.pf_step(self.h, float(dt), ctypes.byref(st)))
        return st.as_dict()

    def assemble(self, dt: float, with_jacobian: bool = True, with_border: bool = True):
        R = np.empty(self.nv)
        J = np.empty(63 * self.n) if with_jacobian else None
        B = np.empty(7 * max(self.n_perf, 1)) if with_border else None
        _check(_lib.pf_assemble(self.h, float(dt), R.ctypes.data, J.ctypes.data if J is not None else None,
                                B.ctypes.data if B is not None else None))
        if B is not None:
            B = B[:7 * self.n_perf].reshape(-1, 7)
        return R, J, B

    def spmv(self, x) -> np.ndarray:
        x = _f64(x)
        y = np.empty(self.nv)
        _check(_lib.pf_spmv(self.h, x.ctypes.data, y.ctypes.data))
        return y

    def linear_solve(self, b, rtol: float):
        b = _f64(b)
        dx = np.empty(self.nv)
        its = _i(0)
        rel = _d(0.0)
        _check(_lib.pf_linear_solve(self.h, b.ctypes.data, float(rtol), dx.ctypes.data, ctypes.byref(its),
                                    ctypes.byref(rel)))
        return dx, int(its.value), float(rel.value)

    def pressure_levels(self):
        """[(dims, A planes (7, n_l))] of the pressure multigrid hierarchy."""
        nl = int(_lib.pf_pressure_level(self.h, -1, None, None))
        out = []
        for l in range(nl):
            dims = np.zeros(3, np.int32)
            _lib.pf_pressure_level(self.h, l, dims.ctypes.data, None)
            A = np.empty(7 * int(np.prod(dims)))
            if _lib.pf_pressure_level(self.h, l, dims.ctypes.data, A.ctypes.data) < 0:
                raise PFError(PF_EHIP, "level read-back failed")
            out.append((tuple(int(d) for d in dims), A.reshape(7, -1)))
        return out

    def pressure_smooth(self, level: int, colour: int, zero_init: bool, b, x):
        b = _f64(b)
        x = _f64(x).copy()
        _check(_lib.pf_pressure_smooth(self.h, level, colour, int(zero_init), b.ctypes.data, x.ctypes.data))
        return x

    def smoother_apply(self, f):
        """The second-stage smoother S^{-1} f (3N + n_wells, plane layout)."""
        f = _f64(f)
        z = np.empty(self.nv)
        _check(_lib.pf_smoother_apply(self.h, f.ctypes.data, z.ctypes.data))
        return z

    def precond_apply(self, v):
        """z = M^{-1} v (the two-stage CPR preconditioner) and w = J~ z as FGMRES forms them."""
        v = _f64(v)
        z = np.empty(self.nv)
        w = np.empty(self.nv)
        _check(_lib.pf_precond_apply(self.h, v.ctypes.data, z.ctypes.data, w.ctypes.data))
        return z, w

    def pressure_vcycle(self, b):
        """The pressure multigrid (mg_cycles V-cycles from 0) applied to b (N, natural order)."""
        b = _f64(b)
        x = np.empty(self.n)
        _check(_lib.pf_pressure_vcycle(self.h, b.ctypes.data, x.ctypes.data))
        return x

    def static(self) -> dict:
        n, npf = self.n, max(self.n_perf, 1)
        out = dict(row_scale=np.empty(self.nv), Tx=np.empty(n), Ty=np.empty(n), Tz=np.empty(n), PVr=np.empty(n),
                   perf_well=np.empty(npf, np.int32), perf_cell=np.empty(npf, np.int32), perf_wi=np.empty(npf))
        _check(_lib.pf_get_static(self.h, *(out[k].ctypes.data for k in
                                            ("row_scale", "Tx", "Ty", "Tz", "PVr", "perf_well", "perf_cell",
                                             "perf_wi"))))
        for k in ("perf_well", "perf_cell", "perf_wi"):
            out[k] = out[k][:self.n_perf]
        return out


class Fusion:
    """Fusion group (pf_fusion_*): simulators stepped together with their
    launches merged, on ``stream`` (default: the current stream)."""

    def __init__(self, device: str = "cuda:0", stream=None):
        import torch
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = _vp()
        with torch.cuda.device(self.device):
            _check(_lib.pf_fusion_create(_vp(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            _lib.pf_fusion_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, sims, dts) -> list:
        """One pf_step of every simulator (its own dt), fused; per-sim stats."""
        n = len(sims)
        hs = (_vp * n)(*[s.h for s in sims])
        d = _f64(dts)
        st = (StepStats * n)()
        _check(_lib.pf_fusion_step(self.h, n, ctypes.cast(hs, _vp), d.ctypes.data, ctypes.cast(st, _vp)))
        return [x.as_dict() for x in st]

    def stats(self) -> dict:
        a, b, c = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
        _check(_lib.pf_fusion_stats(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return dict(issues=a.value, ops=b.value, launches=c.value)


class Server:
    """Continuous-batching server over one device arena (a torch uint8
    tensor of ``arena_bytes``) with ``max_slots`` concurrent realisations;
    ``fused`` = G > 0: the slots form G fusion groups whose members' launches
    are merged."""

    def __init__(self, arena_bytes: int, max_slots: int = 8, device: str = "cuda:0", fused: int = 0):
        import torch
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
        h = _vp()
        _check(_lib.pf_server_create(_vp(self.arena.data_ptr()), int(arena_bytes), int(max_slots), int(fused),
                                     ctypes.byref(h)))
        self.h = h
        self._req = {}

    def close(self):
        if getattr(self, "h", None):
            _lib.pf_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, case, opts: Optional[SolverOpts] = None, n_steps: Optional[int] = None) -> int:
        d = _Desc(case)
        o = opts or default_opts()
        dts = _f64(case.dts if n_steps is None else case.dts[:n_steps])
        P0, S0, C0 = _f64(case.P0), _f64(case.S0), _f64(case.C0)
        Pb0 = _f64(case.Pb0 if len(case.Pb0) else np.zeros(1))
        t = ctypes.c_uint64(0)
        _check(_lib.pf_server_submit(self.h, ctypes.byref(d.desc), ctypes.byref(o), P0.ctypes.data, S0.ctypes.data,
                                     C0.ctypes.data, Pb0.ctypes.data, len(dts), dts.ctypes.data, ctypes.byref(t)))
        self._req[t.value] = (case.n, len(case.wells), len(dts))
        return int(t.value)

    def poll(self, ticket: int):
        """(state, result) with result a dict once state == 2 (done)."""
        n, nw, ns = self._req[ticket]
        st = _i(0)
        P, S, C = np.empty(n), np.empty(n), np.empty(n)
        Pb = np.empty(max(nw, 1))
        lat = np.empty(ns)
        its = np.empty(ns, np.int32)
        times = np.empty(3)
        r = _lib.pf_server_poll(self.h, ticket, ctypes.byref(st), P.ctypes.data, S.ctypes.data, C.ctypes.data,
                                Pb.ctypes.data, lat.ctypes.data, its.ctypes.data, times.ctypes.data)
        _check(r)
        if st.value == 3:
            raise PFError(PF_ENONCONV, _lib.pf_last_error().decode())
        if st.value != 2:
            return st.value, None
        return 2, dict(P=P, S=S, C=C, Pb=Pb[:nw], latency=lat, newton=its, t_submit=times[0],
                       t_start=times[1], t_end=times[2])

    def wait(self, ticket: int = 0):
        _check(_lib.pf_server_wait(self.h, ticket))

    def release(self, ticket: int):
        """Free a finished request's results (the ticket is unknown afterwards)."""
        _check(_lib.pf_server_release(self.h, ticket))
        self._req.pop(ticket, None)

    def info(self) -> dict:
        q, r, pr = _i(0), _i(0), _i(0)
        pb, fb = ctypes.c_size_t(0), ctypes.c_size_t(0)
        _check(_lib.pf_server_info(self.h, ctypes.byref(q), ctypes.byref(r), ctypes.byref(pr), ctypes.byref(pb),
                                   ctypes.byref(fb)))
        return dict(queued=q.value, running=r.value, peak_running=pr.value, peak_bytes=pb.value,
                    free_bytes=fb.value)
