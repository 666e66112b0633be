"""Plain FP64 CPU oracle: the reference the HIP library is checked against.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(``paper_1807_05298_amd``) never imports, links or runs it, and the two share
no code: the residual and its Jacobian come from ``polyflood_oracle.cpp``
(written from the paper, Jacobian by automatic differentiation), and the
nonlinear / timestep drivers below follow the paper's Algorithm 1 (inexact
Newton, here run as standard Newton with an exact linear solve) and its
timestep rules (Sec. 3, solution flowchart items 4-5).

The linear solve of each Newton step is built from library primitives - the
plainest solver that reaches the root; Krylov/CPR internals are not part of
what the oracle pins.  Up to 60,000 unknowns it is SciPy's sparse direct
solver.  Above that (where the direct solver's fill on 3-D grids takes
minutes per solve) it is SciPy's GMRES on the row-scaled system to a true
relative residual of 1e-12, preconditioned in two stages from library
primitives: an exact sparse LU of the pressure block (the pressure columns of
the sum of the scaled water and oil rows), then block Jacobi (each cell's 3x3
block inverted by numpy, well rows by their diagonal) on the remaining
residual.

Vectors are block-wise (Sec. 3.4): x[3i+0]=P, x[3i+1]=S, x[3i+2]=C of cell i,
x[3N+w]=bottom-hole pressure of well w.

Convergence reading (the paper gives only ||b|| < eps, Algorithm 1): the
residual is scaled per cell to pore volumes - water and oil rows by
rho0*PV_ref, polymer rows by C_ref*PV_ref with C_ref = max(max C_inj, 1) -
rate rows by |target|, BHP rows by 1 bar; a timestep is converged when the
scaled residual's max-norm is <= tol_res and the last applied update's scaled
max-norm (|dP|/bar, |dS|, |dC|/C_ref, |dPb|/bar) is <= tol_upd.
Newton update chop: |dS| <= 0.2 per cell, C >= 0 after the update.
Timestep control: the schedule step is the maximum; sub-steps start from
the length remembered from the previous step (dt_init at the start of a
run, 0 meaning the scheduled step); a failed Newton solve (max_newton
iterations) rolls back and halves dt, up to max_cuts times per scheduled
step; after a success dt doubles again up to the schedule step.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "polyflood_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
BAR = 1.0e5


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (no GPU code involved)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared",
                               "-ffp-contract=off", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        vp, dp, i64 = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int64
        L.ora_create.restype = vp
        L.ora_create.argtypes = [ctypes.c_void_p]
        L.ora_destroy.argtypes = [vp]
        L.ora_n_perf.restype = i64
        L.ora_n_perf.argtypes = [vp]
        L.ora_set_well_control.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_double]
        L.ora_set_well_cinj.argtypes = [vp, ctypes.c_int, ctypes.c_double]
        L.ora_well_index_x.restype = ctypes.c_double
        L.ora_well_index_x.argtypes = [ctypes.c_double] * 7
        L.ora_static.argtypes = [vp] + [ctypes.c_void_p] * 7
        L.ora_well_index_z.restype = ctypes.c_double
        L.ora_well_index_z.argtypes = [ctypes.c_double] * 7
        L.ora_cell_props.argtypes = [vp, i64, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_void_p]
        L.ora_accum.argtypes = [vp, ctypes.c_void_p, ctypes.c_void_p]
        L.ora_face_flux.argtypes = [vp, ctypes.c_void_p, i64, ctypes.c_int, ctypes.c_void_p]
        L.ora_perf_rates.argtypes = [vp, ctypes.c_void_p, ctypes.c_void_p]
        L.ora_residual.argtypes = [vp, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p]
        L.ora_residual_cells.argtypes = [vp, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                         ctypes.c_void_p, i64, ctypes.c_void_p]
        L.ora_accum_range.argtypes = [vp, ctypes.c_void_p, i64, i64, ctypes.c_void_p]
        L.ora_isotherm.argtypes = [vp, ctypes.c_void_p, ctypes.c_void_p]
        L.ora_set_ads_hist.argtypes = [vp, ctypes.c_void_p]
        L.ora_cell_rock.argtypes = [vp, ctypes.c_void_p, ctypes.c_void_p]
        L.ora_well_residuals.argtypes = [vp, ctypes.c_void_p, ctypes.c_void_p]
        L.ora_jacobian.restype = i64
        L.ora_jacobian.argtypes = [vp, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                   ctypes.c_void_p, i64, ctypes.c_int,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, i64]
        _lib = L
    return _lib


class _OraModel(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("nwell", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("top", ctypes.c_double),
                ("poro", ctypes.c_void_p), ("kx", ctypes.c_void_p), ("ky", ctypes.c_void_p),
                ("kz", ctypes.c_void_p),
                ("cr", ctypes.c_double), ("pref", ctypes.c_double),
                ("rho_w0", ctypes.c_double), ("rho_o0", ctypes.c_double),
                ("c_w", ctypes.c_double), ("c_o", ctypes.c_double),
                ("mu_w", ctypes.c_double), ("mu_o", ctypes.c_double),
                ("swc", ctypes.c_double), ("sor", ctypes.c_double),
                ("n_w", ctypes.c_double), ("n_o", ctypes.c_double),
                ("krw0", ctypes.c_double), ("kro0", ctypes.c_double), ("grav", ctypes.c_double),
                ("a1", ctypes.c_double), ("a2", ctypes.c_double), ("omega", ctypes.c_double),
                ("cmax", ctypes.c_double), ("ads_max", ctypes.c_double), ("ads_b", ctypes.c_double),
                ("rrf", ctypes.c_double), ("ipv", ctypes.c_double),
                ("w_ix", ctypes.c_void_p), ("w_iy", ctypes.c_void_p), ("w_k0", ctypes.c_void_p),
                ("w_k1", ctypes.c_void_p), ("w_inj", ctypes.c_void_p), ("w_ctrl", ctypes.c_void_p),
                ("w_target", ctypes.c_void_p), ("w_cinj", ctypes.c_void_p),
                ("w_rw", ctypes.c_void_p), ("w_skin", ctypes.c_void_p),
                ("w_dir", ctypes.c_void_p), ("w_ix1", ctypes.c_void_p),
                ("mix_rule", ctypes.c_int32), ("n_ads", ctypes.c_int32), ("n_visc", ctypes.c_int32),
                ("n_pc", ctypes.c_int32), ("mu_p_ref", ctypes.c_double),
                ("ads_c", ctypes.c_void_p), ("ads_a", ctypes.c_void_p), ("visc_c", ctypes.c_void_p),
                ("visc_m", ctypes.c_void_p), ("pc_s", ctypes.c_void_p), ("pc_v", ctypes.c_void_p),
                ("ads_res", ctypes.c_double), ("n_kperm", ctypes.c_int32), ("pad_k", ctypes.c_int32),
                ("kperm_k", ctypes.c_void_p), ("kperm_rrf", ctypes.c_void_p), ("kperm_admax", ctypes.c_void_p)]


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def well_index_z(dx, dy, h, kx, ky, rw, skin=0.0) -> float:
    """Peaceman index of one vertical perforation."""
    return lib().ora_well_index_z(dx, dy, h, kx, ky, rw, skin)


def well_index_x(h, hy, hz, ky, kz, rw, skin=0.0) -> float:
    """Peaceman index of one perforation of a well along x (eq:wi:re:k as printed)."""
    return lib().ora_well_index_x(h, hy, hz, ky, kz, rw, skin)


@dataclass
class NewtonOpts:
    tol_res: float = 1e-10
    tol_upd: float = 1e-9
    max_newton: int = 12
    max_cuts: int = 5
    ds_max: float = 0.2
    dt_init: float = 0.0          # first sub-step length (s); 0: the scheduled step


@dataclass
class StepLog:
    dts: List[float] = field(default_factory=list)
    newton_its: List[int] = field(default_factory=list)
    cuts: int = 0
    switches: List[tuple] = field(default_factory=list)     # (time, well, new control)


class Oracle:
    """The oracle for one case (a ``paper_1807_05298_amd.inputs.Case``)."""

    def __init__(self, case):
        self.case = case
        L = lib()
        f, p = case.fluid, case.polymer
        self._keep = []

        def arr(a, dt=np.float64):
            a = np.ascontiguousarray(a, dtype=dt)
            self._keep.append(a)
            return _ptr(a)

        ws = case.wells
        m = _OraModel()
        m.nx, m.ny, m.nz, m.nwell = case.nx, case.ny, case.nz, len(ws)
        m.dx, m.dy, m.dz, m.top = case.dx, case.dy, case.dz, case.top
        m.poro, m.kx, m.ky, m.kz = arr(case.poro), arr(case.kx), arr(case.ky), arr(case.kz)
        m.cr, m.pref = case.cr, case.p_ref
        m.rho_w0, m.rho_o0, m.c_w, m.c_o = f.rho_w0, f.rho_o0, f.c_w, f.c_o
        m.mu_w, m.mu_o, m.swc, m.sor = f.mu_w, f.mu_o, f.swc, f.sor
        m.n_w, m.n_o, m.krw0, m.kro0, m.grav = f.n_w, f.n_o, f.krw0, f.kro0, f.gravity
        m.a1, m.a2, m.omega, m.cmax = p.a1, p.a2, p.omega, p.c_max
        m.ads_max, m.ads_b, m.rrf, m.ipv = p.ads_max, p.ads_b, p.rrf, p.ipv
        i32 = np.int32
        m.w_ix = arr([w.ix for w in ws] or [0], i32)
        m.w_iy = arr([w.iy for w in ws] or [0], i32)
        m.w_k0 = arr([w.k_top for w in ws] or [0], i32)
        m.w_k1 = arr([w.k_bot for w in ws] or [0], i32)
        m.w_inj = arr([int(w.injector) for w in ws] or [0], i32)
        m.w_ctrl = arr([w.control for w in ws] or [0], i32)
        m.w_target = arr([w.target for w in ws] or [0.0])
        m.w_cinj = arr([w.c_inj for w in ws] or [0.0])
        m.w_rw = arr([w.rw for w in ws] or [0.1])
        m.w_skin = arr([w.skin for w in ws] or [0.0])
        m.w_dir = arr([int(getattr(w, "direction", 0)) for w in ws] or [0], i32)
        m.w_ix1 = arr([int(getattr(w, "ix_last", w.ix)) if getattr(w, "direction", 0) == 1 else w.ix
                       for w in ws] or [0], i32)
        def table(points):
            pts = list(points or [])
            return len(pts), arr([a for a, _ in pts] or [0.0]), arr([b for _, b in pts] or [0.0])
        m.mix_rule = int(getattr(p, "mix_rule", 0))
        m.mu_p_ref = float(getattr(p, "mu_p_ref", 0.0))
        m.n_ads, m.ads_c, m.ads_a = table(getattr(p, "ads_table", None))
        m.n_visc, m.visc_c, m.visc_m = table(getattr(p, "visc_table", None))
        m.n_pc, m.pc_s, m.pc_v = table(getattr(f, "pc_table", None))
        m.ads_res = float(getattr(p, "ads_res", 0.0) or 0.0)
        kp = list(getattr(p, "kperm_table", None) or [])
        m.n_kperm = len(kp)
        m.kperm_k = arr([a for a, _, _ in kp] or [1.0])
        m.kperm_rrf = arr([b for _, b, _ in kp] or [1.0])
        m.kperm_admax = arr([c for _, _, c in kp] or [1.0])
        self._model = m
        self.h = L.ora_create(ctypes.byref(m))
        self.n = case.n
        self.nw = len(ws)
        self.size = 3 * self.n + self.nw
        self.n_perf = int(L.ora_n_perf(self.h))
        st = self.static()
        self.pvr = st["PVr"]
        cinj = [w.c_inj for w in ws if w.injector]
        self.c_ref = max(max(cinj) if cinj else 0.0, 1.0)
        scale = np.empty(self.size)
        scale[0:3 * self.n:3] = f.rho_w0 * self.pvr
        scale[1:3 * self.n:3] = f.rho_o0 * self.pvr
        scale[2:3 * self.n:3] = self.c_ref * self.pvr
        for k, w in enumerate(ws):
            scale[3 * self.n + k] = BAR if w.control == 0 else max(abs(w.target), 1e-30)
        self.res_scale = scale
        # well controls: as given (primary) and active (after switches at BHP limits)
        self.ctrl0 = [int(w.control) for w in ws]
        self.target0 = [float(w.target) for w in ws]
        self.limit = [float(getattr(w, "bhp_limit", 0.0) or 0.0) for w in ws]
        self.ctrl = list(self.ctrl0)
        self.target = list(self.target0)
        self.ads_res = m.ads_res
        self.ads_hist = np.zeros(self.n)

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().ora_destroy(self.h)
                self.h = None
        except Exception:
            pass

    # ---- layout helpers --------------------------------------------------------
    def pack(self, P, S, C, Pb) -> np.ndarray:
        x = np.empty(self.size)
        x[0:3 * self.n:3] = P
        x[1:3 * self.n:3] = S
        x[2:3 * self.n:3] = C
        x[3 * self.n:] = Pb
        return x

    def unpack(self, x):
        n = self.n
        return x[0:3 * n:3].copy(), x[1:3 * n:3].copy(), x[2:3 * n:3].copy(), x[3 * n:].copy()

    def initial_state(self) -> np.ndarray:
        c = self.case
        return self.pack(c.P0, c.S0, c.C0, c.Pb0)

    # ---- C entry points ----------------------------------------------------------
    def static(self):
        n, npf = self.n, self.n_perf
        Tx, Ty, Tz, PVr = (np.zeros(n) for _ in range(4))
        pw = np.zeros(max(npf, 1), np.int32)
        pc = np.zeros(max(npf, 1), np.int32)
        pwi = np.zeros(max(npf, 1))
        lib().ora_static(self.h, _ptr(Tx), _ptr(Ty), _ptr(Tz), _ptr(PVr), _ptr(pw), _ptr(pc), _ptr(pwi))
        return dict(Tx=Tx, Ty=Ty, Tz=Tz, PVr=PVr, perf_well=pw[:npf], perf_cell=pc[:npf],
                    perf_wi=pwi[:npf])

    def cell_props(self, i, P, S, C) -> dict:
        out = np.zeros(9)
        lib().ora_cell_props(self.h, int(i), float(P), float(S), float(C), _ptr(out))
        keys = ["phi", "rho_w", "rho_o", "krw", "kro", "mu_we", "mu_pe", "ads", "rk"]
        return dict(zip(keys, out))

    def accum(self, x) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        M = np.zeros(3 * self.n)
        lib().ora_accum(self.h, _ptr(x), _ptr(M))
        return M

    def face_flux(self, x, L, direction) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        F = np.zeros(3)
        lib().ora_face_flux(self.h, _ptr(x), int(L), int(direction), _ptr(F))
        return F

    def perf_rates(self, x) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        q = np.zeros(3 * max(self.n_perf, 1))
        lib().ora_perf_rates(self.h, _ptr(x), _ptr(q))
        return q[:3 * self.n_perf].reshape(-1, 3)

    def residual(self, x, Mn, dt) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        Mn = np.ascontiguousarray(Mn, dtype=np.float64)
        R = np.zeros(self.size)
        lib().ora_residual(self.h, _ptr(x), _ptr(Mn), float(dt), _ptr(R))
        return R

    def residual_cells(self, x, Mn, dt, cells) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        Mn = np.ascontiguousarray(Mn, dtype=np.float64)
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        out = np.zeros(3 * len(cells))
        lib().ora_residual_cells(self.h, _ptr(x), _ptr(Mn), float(dt), _ptr(cells),
                                 len(cells), _ptr(out))
        return out.reshape(-1, 3)

    def isotherm(self, x) -> np.ndarray:
        """Equilibrium adsorption of every cell at the concentrations of x."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        out = np.zeros(self.n)
        lib().ora_isotherm(self.h, _ptr(x), _ptr(out))
        return out

    def cell_rock(self):
        """Per-cell RRF and A_d,max (the permeability table's values)."""
        rrf, admax = np.zeros(self.n), np.zeros(self.n)
        lib().ora_cell_rock(self.h, _ptr(rrf), _ptr(admax))
        return rrf, admax

    def set_ads_hist(self, H):
        self.ads_hist = np.ascontiguousarray(H, dtype=np.float64).copy()
        lib().ora_set_ads_hist(self.h, _ptr(self.ads_hist))

    def note_converged_state(self, x):
        """Retention (Sec. 2.3): the largest past adsorption of every cell
        takes in the equilibrium adsorption of a converged state."""
        if self.ads_res > 0.0:
            self.set_ads_hist(np.maximum(self.ads_hist, self.isotherm(x)))

    def accum_threaded(self, x, threads=None, chunk=1 << 18) -> np.ndarray:
        """accum() evaluated in independent chunks of cells on a thread pool."""
        import concurrent.futures as cf
        x = np.ascontiguousarray(x, dtype=np.float64)
        M = np.zeros(3 * self.n)
        threads = threads or max(1, min(16, os.cpu_count() or 1))

        def work(a):
            lib().ora_accum_range(self.h, _ptr(x), a, min(a + chunk, self.n), _ptr(M))

        with cf.ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(work, range(0, self.n, chunk)))
        return M

    def well_residuals(self, x) -> np.ndarray:
        """The well rows of the residual (n_wells values)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        W = np.zeros(max(self.nw, 1))
        lib().ora_well_residuals(self.h, _ptr(x), _ptr(W))
        return W[:self.nw]

    def cell_residuals(self, x, Mn, dt, threads=None, chunk=1 << 17) -> np.ndarray:
        """The three residual rows of every cell, shape (N, 3), evaluated in
        independent chunks of cells on a pool of threads (the C call runs
        without the interpreter lock); the same values as residual()."""
        import concurrent.futures as cf
        x = np.ascontiguousarray(x, dtype=np.float64)
        Mn = np.ascontiguousarray(Mn, dtype=np.float64)
        out = np.zeros((self.n, 3))
        threads = threads or max(1, min(16, os.cpu_count() or 1))

        def work(a):
            b = min(a + chunk, self.n)
            cells = np.arange(a, b, dtype=np.int64)
            res = np.zeros(3 * (b - a))
            lib().ora_residual_cells(self.h, _ptr(x), _ptr(Mn), float(dt), _ptr(cells), b - a, _ptr(res))
            out[a:b] = res.reshape(-1, 3)

        with cf.ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(work, range(0, self.n, chunk)))
        return out

    def jacobian(self, x, Mn, dt, cells=None, with_wells=True) -> sp.csr_matrix:
        """Jacobian d[R;W]/d[x] as CSR (rows of ``cells`` only when given)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        Mn = np.ascontiguousarray(Mn, dtype=np.float64)
        ncell = self.n if cells is None else len(cells)
        cap = ncell * (9 + 6 * 18) + 12 * self.n_perf + 4 * self.n_perf + self.nw + 16
        I = np.zeros(cap, np.int32)
        J = np.zeros(cap, np.int32)
        V = np.zeros(cap)
        if cells is None:
            cp, nc = None, 0
        else:
            cells = np.ascontiguousarray(cells, dtype=np.int64)
            cp, nc = _ptr(cells), len(cells)
        nnz = lib().ora_jacobian(self.h, _ptr(x), _ptr(Mn), float(dt), cp, nc, int(with_wells),
                                 _ptr(I), _ptr(J), _ptr(V), cap)
        assert nnz <= cap, (nnz, cap)
        return sp.coo_matrix((V[:nnz], (I[:nnz], J[:nnz])), shape=(self.size, self.size)).tocsr()

    # ---- linear solve ------------------------------------------------------------
    DIRECT_MAX = 60000

    def linear_solve(self, J, R):
        """dx with J dx = -R (see the module notes); None when the solver fails."""
        if self.size <= self.DIRECT_MAX:
            dx = spla.spsolve(J.tocsc(), -R)
            return dx if np.all(np.isfinite(dx)) else None
        n = self.n
        A = (sp.diags(1.0 / self.res_scale) @ J).tocsr()
        b = -R / self.res_scale
        nb = float(np.linalg.norm(b))
        if nb == 0.0:
            return np.zeros_like(b)
        Ap = (A[0:3 * n:3] + A[1:3 * n:3])[:, 0:3 * n:3].tocsc()
        lup = spla.splu(Ap, permc_spec="MMD_AT_PLUS_A")
        C = A.tocoo()
        m = (C.row < 3 * n) & (C.col < 3 * n) & (C.row // 3 == C.col // 3)
        blocks = np.zeros((n, 3, 3))
        np.add.at(blocks, (C.row[m] // 3, C.row[m] % 3, C.col[m] % 3), C.data[m])
        binv = np.linalg.inv(blocks)
        dw = A.diagonal()[3 * n:]

        def prec(v):
            v = np.asarray(v, dtype=np.float64)
            z = np.zeros_like(v)
            z[0:3 * n:3] = lup.solve(v[0:3 * n:3] + v[1:3 * n:3])
            r = v - A @ z
            z[:3 * n] += np.einsum("nij,nj->ni", binv, r[:3 * n].reshape(n, 3)).reshape(-1)
            z[3 * n:] += r[3 * n:] / dw
            return z

        M = spla.LinearOperator(A.shape, prec, dtype=np.float64)
        dx = np.zeros_like(b)
        for _ in range(5):
            dx, _ = spla.gmres(A, b, x0=dx, M=M, rtol=1e-12, atol=0.0, restart=80, maxiter=10)
            if not np.all(np.isfinite(dx)):
                return None
            if np.linalg.norm(A @ dx - b) <= 1e-12 * nb:
                return dx
        return None

    # ---- nonlinear solve ---------------------------------------------------------
    def scaled_residual(self, R) -> np.ndarray:
        return R / self.res_scale

    def apply_update(self, x, dx, ds_max=0.2):
        """Chopped Newton update; returns the new state and the scaled max-norm
        of the change actually applied."""
        n = self.n
        xn = x + dx
        s_old = x[1:3 * n:3]
        ds = np.clip(dx[1:3 * n:3], -ds_max, ds_max)
        xn[1:3 * n:3] = s_old + ds
        xn[2:3 * n:3] = np.maximum(xn[2:3 * n:3], 0.0)
        d = xn - x
        upd = max(np.max(np.abs(d[0:3 * n:3])) / BAR, np.max(np.abs(d[1:3 * n:3])),
                  np.max(np.abs(d[2:3 * n:3])) / self.c_ref,
                  np.max(np.abs(d[3 * n:])) / BAR if self.nw else 0.0)
        return xn, upd

    def newton(self, x0, dt, opts: NewtonOpts, Mn=None, timing=None):
        """Newton solve of one backward-Euler step from x0 (= x^n).  Returns
        (x, iterations, converged, final scaled residual max-norm)."""
        self.note_converged_state(x0)      # x0 = x^n, the last converged state
        if Mn is None:
            Mn = self.accum(x0)
        x = x0.copy()
        upd = np.inf
        for it in range(opts.max_newton + 1):
            t0 = time.perf_counter()
            R = self.residual(x, Mn, dt)
            rmax = float(np.max(np.abs(self.scaled_residual(R))))
            if not np.isfinite(rmax):
                return x, it, False, rmax
            if it > 0 and rmax <= opts.tol_res and upd <= opts.tol_upd:
                return x, it, True, rmax
            if it == opts.max_newton:
                return x, it, False, rmax
            J = self.jacobian(x, Mn, dt)
            t1 = time.perf_counter()
            try:
                dx = self.linear_solve(J, R)
            except Exception:
                return x, it, False, rmax
            if dx is None:
                return x, it, False, rmax
            t2 = time.perf_counter()
            if timing is not None:
                timing["assemble"] = timing.get("assemble", 0.0) + (t1 - t0)
                timing["solve"] = timing.get("solve", 0.0) + (t2 - t1)
            x, upd = self.apply_update(x, dx, opts.ds_max)
        return x, opts.max_newton, False, rmax

    # ---- well operations between timesteps (Sec. 3 item 4) -------------------
    def set_controls(self, ctrl, target):
        """Active control and target of every well; the well rows' scale
        follows (BHP rows by 1 bar, rate rows by |target|)."""
        for w, (c, t) in enumerate(zip(ctrl, target)):
            lib().ora_set_well_control(self.h, w, int(c), float(t))
            self.res_scale[3 * self.n + w] = BAR if c == 0 else max(abs(t), 1e-30)
        self.ctrl, self.target = list(ctrl), list(target)

    def set_well_operation(self, w, control, target, c_inj=0.0, bhp_limit=0.0):
        """Change well w's operation between timesteps: it becomes the given
        operation and the active one."""
        self.ctrl0[w], self.target0[w], self.limit[w] = int(control), float(target), float(bhp_limit)
        lib().ora_set_well_cinj(self.h, w, float(c_inj))
        ctrl, target_a = list(self.ctrl), list(self.target)
        ctrl[w], target_a[w] = int(control), float(target)
        self.set_controls(ctrl, target_a)

    def apply_events(self, step):
        """The case's well-operation changes scheduled before ``step``."""
        for k, w, ch in getattr(self.case, "events", []):
            if k == step:
                W = self.case.wells[w]
                op = dict(control=W.control, target=W.target, c_inj=W.c_inj, bhp_limit=W.bhp_limit)
                op.update(self._ops.get(w, {}))
                op.update(ch)
                self._ops[w] = op
                self.set_well_operation(w, **op)

    def well_rates(self, x):
        """Surface water and oil rates (m^3/s, into the reservoir) of every well."""
        f = self.case.fluid
        q = self.perf_rates(x)
        pw = self.static()["perf_well"]
        qw, qo = np.zeros(self.nw), np.zeros(self.nw)
        for k in range(self.n_perf):
            qw[pw[k]] += q[k, 0] / f.rho_w0
            qo[pw[k]] += q[k, 1] / f.rho_o0
        return qw, qo

    def apply_well_limits(self, x):
        """After a converged timestep: a rate-controlled well beyond its BHP
        limit (above it for an injector, below for a producer) continues at
        the limit; a well held at its limit whose controlled rate there
        exceeds its target returns to the target.  Returns the switches as
        (well, new control)."""
        if not any(l > 0 and c0 != 0 for l, c0 in zip(self.limit, self.ctrl0)):
            return []
        Pb = x[3 * self.n:]
        qw, qo = self.well_rates(x)
        ctrl, target, out = list(self.ctrl), list(self.target), []
        for w, W in enumerate(self.case.wells):
            lim, c0 = self.limit[w], self.ctrl0[w]
            if not lim > 0 or c0 == 0:
                continue
            if ctrl[w] != 0:
                if (Pb[w] > lim) if W.injector else (Pb[w] < lim):
                    ctrl[w], target[w] = 0, lim
                    out.append((w, 0))
            else:
                q = qw[w] if c0 == 1 else qo[w] if c0 == 2 else qw[w] + qo[w]
                if abs(q) > abs(self.target0[w]):
                    ctrl[w], target[w] = c0, self.target0[w]
                    out.append((w, c0))
        if out:
            self.set_controls(ctrl, target)
        return out

    def advance(self, x, step_len, opts: NewtonOpts, log: Optional[StepLog] = None):
        """Advance one scheduled step of length ``step_len``: sub-steps start
        from the length remembered from the previous step, are halved on
        failure (at most max_cuts times) and doubled after each success, never
        beyond the scheduled step."""
        remaining = step_len
        dt = min(self.dt_next, step_len) if getattr(self, "dt_next", 0.0) > 0 else step_len
        cuts = 0
        while remaining > 1e-9 * step_len:
            dt = min(dt, remaining)
            xn, its, ok, _ = self.newton(x, dt, opts)
            if not ok:
                cuts += 1
                if cuts > opts.max_cuts:
                    raise RuntimeError("Newton failed after maximum timestep cuts")
                dt *= 0.5
                continue
            x = xn
            remaining -= dt
            if log is not None:
                log.dts.append(dt)
                log.newton_its.append(its)
            for w, c in self.apply_well_limits(x):
                if log is not None:
                    log.switches.append((sum(log.dts) if log is not None else 0.0, w, c))
            dt = min(2.0 * dt, step_len)
        self.dt_next = dt
        if log is not None:
            log.cuts += cuts
        return x

    def run(self, opts: Optional[NewtonOpts] = None, n_steps: Optional[int] = None, x0=None):
        """Run the schedule (or its first n_steps); returns the states after
        every scheduled step and the step log."""
        opts = opts or NewtonOpts()
        x = self.initial_state() if x0 is None else x0.copy()
        self.dt_next = opts.dt_init
        ws = self.case.wells
        self.ctrl0 = [int(w.control) for w in ws]
        self.target0 = [float(w.target) for w in ws]
        self.limit = [float(getattr(w, "bhp_limit", 0.0) or 0.0) for w in ws]
        for k, w in enumerate(ws):
            lib().ora_set_well_cinj(self.h, k, float(w.c_inj))
        self.set_controls(self.ctrl0, self.target0)
        self.set_ads_hist(np.zeros(self.n))
        dts = self.case.dts if n_steps is None else self.case.dts[:n_steps]
        log = StepLog()
        states = []
        self._ops = {}
        for k, d in enumerate(dts):
            self.apply_events(k)
            x = self.advance(x, float(d), opts, log)
            states.append(x.copy())
        return states, log


# ---- capillary-gravity equilibrium initial state (Sec. 4.1.3) ------------------
MARCH_STEP = 0.25        # m: the longest pressure-marching step


def _march(p0, z0, z1, rho0, c, p_ref, g):
    """Pressure at depth z1 from p0 at depth z0 under dP/dz = rho(P) g with
    rho(P) = rho0 exp(c (P - p_ref)): classical fourth-order Runge-Kutta in
    equal steps of at most MARCH_STEP, the density recomputed at every
    stage."""
    dz = z1 - z0
    n = max(1, int(math.ceil(abs(dz) / MARCH_STEP)))
    h = dz / n
    f = lambda p: rho0 * math.exp(c * (p - p_ref)) * g
    p = p0
    for _ in range(n):
        k1 = f(p)
        k2 = f(p + 0.5 * h * k1)
        k3 = f(p + 0.5 * h * k2)
        k4 = f(p + h * k3)
        p = p + h / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return p


def _invert_pc(delta, pts):
    """Saturation whose capillary pressure (the table, decreasing in S) is
    delta; the table's end saturations beyond its range."""
    s = [a for a, _ in pts]
    v = [b for _, b in pts]
    if delta >= v[0]:
        return s[0]
    if delta <= v[-1]:
        return s[-1]
    k = 0
    while not (v[k] >= delta > v[k + 1]):
        k += 1
    return s[k] + (delta - v[k]) * (s[k + 1] - s[k]) / (v[k + 1] - v[k])


def _march_water(p_fwl, z0, z1, f, p_ref, pc_last):
    """Oil and water pressure together from the free-water level (both p_fwl
    there) to depth z1: dP_o/dz = rho_o(P_o) g, dP_w/dz = rho_w(P) g with the
    water density evaluated, as in the discrete fluxes, at the cell pressure
    unknown P (P_o where the oil phase is continuous, P_w + P_c(S_last)
    below); the same Runge-Kutta steps as _march.  Returns P_w."""
    g = f.gravity
    dz = z1 - z0
    n = max(1, int(math.ceil(abs(dz) / MARCH_STEP)))
    h = dz / n

    def rhs(po, pw):
        p = po if po - pw > pc_last else pw + pc_last
        return (f.rho_o0 * math.exp(f.c_o * (po - p_ref)) * g, f.rho_w0 * math.exp(f.c_w * (p - p_ref)) * g)

    po = pw = p_fwl
    for _ in range(n):
        a1, b1 = rhs(po, pw)
        a2, b2 = rhs(po + 0.5 * h * a1, pw + 0.5 * h * b1)
        a3, b3 = rhs(po + 0.5 * h * a2, pw + 0.5 * h * b2)
        a4, b4 = rhs(po + h * a3, pw + h * b3)
        po = po + h / 6.0 * (a1 + 2.0 * a2 + 2.0 * a3 + a4)
        pw = pw + h / 6.0 * (b1 + 2.0 * b2 + 2.0 * b3 + b4)
    return pw


def equilibrium_state(case, datum_depth, datum_p, fwl_depth):
    """Initial state in capillary-gravity equilibrium (Sec. 4.1.3): the oil
    pressure is marched from the datum (depth, oil pressure) to every layer
    centre and to the free-water level, where the water pressure equals it
    (zero capillary pressure); the water pressure is marched from there
    (_march_water).  At each depth the saturation is the one whose capillary
    pressure balances P_o - P_w (without a table: S_wc above the free-water
    level, 1 - S_or below), the cell's pressure unknown (the oil pressure) is
    P_o where the oil phase is continuous (P_o - P_w above the table's last
    capillary pressure) and P_w + P_c(S) below, and no polymer is present.
    Wells: BHP-controlled at their target, rate-controlled at the pressure of
    their datum layer.  Returns P, S, C (N) and Pb (n_wells)."""
    f = case.fluid
    g = f.gravity
    pts = list(f.pc_table) if f.pc_table else [(f.swc, 0.0), (1.0 - f.sor, 0.0)]
    pc_last = pts[-1][1]
    p_fwl = _march(datum_p, datum_depth, fwl_depth, f.rho_o0, f.c_o, case.p_ref, g)
    depth = case.top + (np.arange(case.nz) + 0.5) * case.dz
    P_l, S_l = np.zeros(case.nz), np.zeros(case.nz)
    for k, z in enumerate(depth):
        po = _march(datum_p, datum_depth, z, f.rho_o0, f.c_o, case.p_ref, g)
        pw = _march_water(p_fwl, fwl_depth, z, f, case.p_ref, pc_last)
        delta = po - pw
        if f.pc_table:
            S_l[k] = _invert_pc(delta, pts)
        else:
            S_l[k] = f.swc if delta > 0.0 else 1.0 - f.sor
        P_l[k] = po if delta > pc_last else pw + pc_last
    nxy = case.nx * case.ny
    P, S = np.repeat(P_l, nxy), np.repeat(S_l, nxy)
    C = np.zeros(case.n)
    Pb = np.array([w.target if w.control == 0 else P_l[w.k_top] for w in case.wells], dtype=np.float64)
    return P, S, C, Pb
