"""Seeded synthetic reservoir inputs shared by the HIP library, its tests and the bench.

This module only *draws* inputs: grid geometry, rock fields, fluid and polymer
constants, well placement and controls, the initial state and the timestep
schedule.  It holds none of the simulator's arithmetic (no property model, no
transmissibility, no well index, no residual); both the oracle and the HIP path
derive everything from these arrays on their own.

Units are SI throughout: m, m^2, Pa, Pa*s, kg/m^3, s.  Cells are stored in
natural order i = ix + nx*(iy + ny*iz) (x fastest), matching the global
ordering of the paper's Section 3 (grid distribution).  Arrays are therefore
shaped (nz, ny, nx) before flattening.

Workload recipes (the five named workloads plus small test cases):
  * ``c1``  10x10x3 quarter five-spot, 300 cells, 30 daily steps.
  * ``c2``  60x220x85 layered/channelised field (1.12M cells), central
            polymer injector + 4 corner producers, 100 x 5 d.
  * ``c3``  200x200x50 lognormal field (2M cells), 5x5 line drive, 50 x 5 d.
  * ``c4``  64 serving realisations of 20k-500k cells (``serving_batch``).
  * ``c5``  300^3 lognormal field (27M cells), 100-well checkerboard, 20 x 10 d.
The 60x220x85 shape matches the public SPE10 model-2 grid; that dataset is
not used, and the seeded field of ``c2`` stands in for it.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# --- unit constants (inputs, not model arithmetic) -------------------------
MD = 9.869233e-16          # m^2 per millidarcy
CP = 1.0e-3                # Pa*s per centipoise
BAR = 1.0e5                # Pa per bar
DAY = 86400.0              # s per day
PSI = 6894.757293168       # Pa per psi
FT = 0.3048                # m per foot
GRAVITY = 9.80665          # m/s^2

CTRL_BHP = 0
CTRL_WRATE = 1
CTRL_ORATE = 2
CTRL_LRATE = 3
WELL_Z = 0
WELL_X = 1
MIX_POLY = 0
MIX_LINEAR = 1
MIX_EXP = 2
MIX_TABLE = 3


@dataclasses.dataclass
class Fluid:
    """Water/oil constants.  Densities at the reference pressure, isothermal
    compressibilities (1/Pa), constant viscosities, Corey parameters."""
    rho_w0: float = 1025.18
    rho_o0: float = 832.96
    c_w: float = 3.03e-6 / BAR
    c_o: float = 1.0e-5 / BAR
    mu_w: float = 0.5 * CP
    mu_o: float = 5.0 * CP
    swc: float = 0.2
    sor: float = 0.2
    n_w: float = 2.0
    n_o: float = 2.0
    krw0: float = 1.0
    kro0: float = 1.0
    gravity: float = GRAVITY
    # capillary pressure P_o - P_w: (S, Pa) points, piecewise linear; None: 0
    pc_table: Optional[List[tuple]] = None


@dataclasses.dataclass
class Polymer:
    """Polymer constants: viscosity polynomial mu_w*(1 + a1*C + a2*C^2) (C in
    kg/m^3), Todd-Longstaff omega, reference (maximum) concentration, Langmuir
    plateau (kg per m^3 of rock) and affinity (m^3/kg), residual resistance
    factor and inaccessible pore-volume fraction."""
    a1: float = 2.0
    a2: float = 1.0
    omega: float = 1.0
    c_max: float = 1.0
    ads_max: float = 0.1
    ads_b: float = 1.0
    rrf: float = 1.5
    ipv: float = 0.1
    # variants: mixing rule (MIX_POLY / MIX_LINEAR / MIX_EXP / MIX_TABLE),
    # viscosity at c_max for the mixing rules (0: the polynomial's), tables
    # of (C, A) adsorption and (C, multiplier) viscosity points
    mix_rule: int = 0
    mu_p_ref: float = 0.0
    ads_table: Optional[List[tuple]] = None
    visc_table: Optional[List[tuple]] = None
    # retention: part of a cell's largest past adsorption that cannot desorb
    # (0: equilibrium sorption); RRF and A_d,max against rock permeability:
    # (k in m^2, RRF, A_d,max in kg per m^3 rock) points
    ads_res: float = 0.0
    kperm_table: Optional[List[tuple]] = None


@dataclasses.dataclass
class Well:
    """A vertical well at column (ix, iy) perforated in layers k_top..k_bot,
    or (direction = WELL_X) a horizontal well along x in row iy of layer
    k_top (= k_bot) perforated in cells ix..ix_last.

    ``target`` is Pa for BHP control, m^3/s at reference density for rate
    controls (positive = into the reservoir)."""
    ix: int
    iy: int
    k_top: int
    k_bot: int
    injector: bool
    control: int
    target: float
    c_inj: float = 0.0
    rw: float = 0.1
    skin: float = 0.0
    bhp_limit: float = 0.0    # BHP bound of a rate-controlled well (Pa; 0: none)
    direction: int = 0        # WELL_Z or WELL_X
    ix_last: int = -1         # last perforated column of a WELL_X well


@dataclasses.dataclass
class Case:
    name: str
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    top: float
    poro: np.ndarray          # (N,) reference porosity
    kx: np.ndarray            # (N,) m^2
    ky: np.ndarray
    kz: np.ndarray
    cr: float                 # rock compressibility, 1/Pa
    p_ref: float              # reference pressure, Pa
    fluid: Fluid
    polymer: Polymer
    wells: List[Well]
    P0: np.ndarray            # (N,) initial oil pressure, Pa
    S0: np.ndarray            # (N,) initial water saturation
    C0: np.ndarray            # (N,) initial polymer concentration, kg/m^3
    Pb0: np.ndarray           # (n_wells,) initial bottom-hole pressure, Pa
    dts: np.ndarray           # schedule, s
    # well operation changes: (step index, well index, fields of Well to set
    # before that step: control, target, c_inj, bhp_limit)
    events: List[tuple] = dataclasses.field(default_factory=list)

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_wells(self) -> int:
        return len(self.wells)

    @property
    def n_perf(self) -> int:
        return sum((w.ix_last - w.ix + 1) if w.direction == WELL_X else (w.k_bot - w.k_top + 1)
                   for w in self.wells)

    def copy(self) -> "Case":
        return dataclasses.replace(
            self, poro=self.poro.copy(), kx=self.kx.copy(), ky=self.ky.copy(),
            kz=self.kz.copy(), P0=self.P0.copy(), S0=self.S0.copy(),
            C0=self.C0.copy(), Pb0=self.Pb0.copy(), dts=self.dts.copy(), events=list(self.events),
            fluid=dataclasses.replace(self.fluid),
            polymer=dataclasses.replace(self.polymer),
            wells=[dataclasses.replace(w) for w in self.wells])


# --- random fields -----------------------------------------------------------
def gaussian_field(rng: np.random.Generator, shape, corr) -> np.ndarray:
    """Unit-variance Gaussian random field of ``shape`` = (nz, ny, nx).

    White noise is filtered in Fourier space by a Gaussian kernel whose
    standard deviation (in cells) per axis is ``corr`` = (cz, cy, cx); a zero
    entry leaves that axis uncorrelated.  The result is rescaled to zero mean
    and unit variance."""
    noise = rng.standard_normal(shape)
    if all(c <= 0 for c in corr):
        return noise
    spec = np.fft.rfftn(noise)
    kz = np.fft.fftfreq(shape[0])[:, None, None]
    ky = np.fft.fftfreq(shape[1])[None, :, None]
    kx = np.fft.rfftfreq(shape[2])[None, None, :]
    cz, cy, cx = (max(c, 0.0) for c in corr)
    filt = np.exp(-2.0 * math.pi ** 2 * ((cz * kz) ** 2 + (cy * ky) ** 2 + (cx * kx) ** 2))
    spec *= filt
    del filt
    out = np.fft.irfftn(spec, s=shape, axes=(0, 1, 2))
    out -= out.mean()
    sd = out.std()
    if sd > 0:
        out /= sd
    return out


def _poro_from_logk(rng, log10k_md: np.ndarray) -> np.ndarray:
    """Porosity correlated to log-permeability (mD), with a little noise."""
    phi = 0.05 + 0.0625 * (log10k_md + 1.0) + rng.normal(0.0, 0.01, log10k_md.shape)
    return np.clip(phi, 0.05, 0.35)


def _initial_state(nx, ny, nz, dz, top, p_top, fluid: Fluid, wells: List[Well]):
    """Oil-filled reservoir at connate water, no polymer, pressure rising
    linearly with depth at the surface oil density gradient (an initial guess;
    the first timestep settles the small residual imbalance)."""
    n = nx * ny * nz
    depth = top + (np.arange(nz) + 0.5) * dz
    p_layer = p_top + fluid.rho_o0 * fluid.gravity * (depth - depth[0])
    P0 = np.repeat(p_layer, nx * ny).astype(np.float64)
    S0 = np.full(n, fluid.swc)
    C0 = np.zeros(n)
    Pb0 = np.zeros(len(wells))
    for k, w in enumerate(wells):
        if w.control == CTRL_BHP:
            Pb0[k] = w.target
        else:
            cell = w.ix + nx * (w.iy + ny * w.k_top)
            Pb0[k] = P0[cell] + (10.0 * BAR if w.injector else -10.0 * BAR)
    return P0, S0, C0, Pb0


DEFAULT_TOP = 6150.0 * FT           # 1874.52 m
DEFAULT_PTOP = 4000.0 * PSI         # 275.79 bar


def _finish(name, nx, ny, nz, dx, dy, dz, poro, kx, ky, kz, wells, dts,
            fluid=None, polymer=None, top=DEFAULT_TOP, p_top=DEFAULT_PTOP,
            cr=1.0e-6 / BAR) -> Case:
    fluid = fluid or Fluid()
    polymer = polymer or Polymer()
    P0, S0, C0, Pb0 = _initial_state(nx, ny, nz, dz, top, p_top, fluid, wells)
    return Case(name=name, nx=nx, ny=ny, nz=nz, dx=dx, dy=dy, dz=dz, top=top,
                poro=np.ascontiguousarray(poro.reshape(-1), dtype=np.float64),
                kx=np.ascontiguousarray(kx.reshape(-1), dtype=np.float64),
                ky=np.ascontiguousarray(ky.reshape(-1), dtype=np.float64),
                kz=np.ascontiguousarray(kz.reshape(-1), dtype=np.float64),
                cr=cr, p_ref=p_top, fluid=fluid, polymer=polymer, wells=wells,
                P0=P0, S0=S0, C0=C0, Pb0=Pb0, dts=np.asarray(dts, dtype=np.float64))


def _vwell(ix, iy, nz, injector, control, target, c_inj=0.0):
    return Well(ix=ix, iy=iy, k_top=0, k_bot=nz - 1, injector=injector,
                control=control, target=target, c_inj=c_inj)


# --- the named workloads -------------------------------------------------------
def case_c1(seed: int = 1) -> Case:
    """10x10x3 quarter five-spot, 20x20x5 m blocks; phi ~ U(0.2,0.3) iid;
    ln k iid normal, sigma 1, arithmetic mean 100 mD; water-rate polymer
    injector (50 m^3/d, C=1 kg/m^3) at (0,0), BHP producer (200 bar) at (9,9);
    30 daily steps."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = 10, 10, 3
    shape = (nz, ny, nx)
    poro = rng.uniform(0.2, 0.3, shape)
    lnk = (math.log(100.0) - 0.5) + 1.0 * rng.standard_normal(shape)
    k = np.exp(lnk) * MD
    wells = [_vwell(0, 0, nz, True, CTRL_WRATE, 50.0 / DAY, 1.0),
             _vwell(nx - 1, ny - 1, nz, False, CTRL_BHP, 200.0 * BAR)]
    return _finish("c1", nx, ny, nz, 20.0, 20.0, 5.0, poro, k, k.copy(), k.copy(),
                   wells, [DAY] * 30)


def case_c2(seed: int = 2, nz_override: Optional[int] = None) -> Case:
    """60x220x85 layered/channelised field with 20x10x2 ft blocks.

    Layers 0-34: correlated lognormal (correlation 8x16x1 cells, geometric
    mean 100 mD).  Layers 35-84: 3-6 sinuous channels per layer running along
    y (width 4-8 cells) at geometric mean 500 mD in a 0.5 mD background.  Per
    layer log-spread sigma ~ U(1.5, 3.0); log10 k clipped to [-1, 3] (four
    decades).  Porosity correlated to log k.  Central polymer injector at
    (30,110), 800 m^3/d, C=1; BHP producers (200 bar) at the 4 corners;
    100 x 5 d.  ``nz_override`` keeps the recipe but truncates the layer
    count (used for bounded CPU samples)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz_full = 60, 220, 85
    nz = nz_full if nz_override is None else int(nz_override)
    g = gaussian_field(rng, (nz_full, ny, nx), (0.0, 16.0, 8.0))
    sig = rng.uniform(1.5, 3.0, nz_full)
    lnk = np.empty((nz_full, ny, nx))
    yy = np.arange(ny)[:, None]
    xx = np.arange(nx)[None, :]
    for z in range(nz_full):
        if z < 35:
            lnk[z] = math.log(100.0) + sig[z] * g[z]
        else:
            base = math.log(0.5) + 0.5 * sig[z] * g[z]
            chan = math.log(500.0) + 0.5 * sig[z] * g[z]
            mask = np.zeros((ny, nx), dtype=bool)
            for _ in range(int(rng.integers(3, 7))):
                x0 = rng.uniform(0, nx)
                amp = rng.uniform(2.0, 10.0)
                lam = rng.uniform(40.0, 120.0)
                th = rng.uniform(0, 2 * math.pi)
                wid = rng.uniform(4.0, 8.0)
                xc = x0 + amp * np.sin(2 * math.pi * yy / lam + th)
                mask |= np.abs(xx - xc) <= 0.5 * wid
            lnk[z] = np.where(mask, chan, base)
    log10k = np.clip(lnk / math.log(10.0), -1.0, 3.0)[:nz]
    k = (10.0 ** log10k) * MD
    poro = _poro_from_logk(rng, log10k)
    wells = [_vwell(30, 110, nz, True, CTRL_WRATE, 800.0 / DAY, 1.0)]
    for (ix, iy) in [(0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1)]:
        wells.append(_vwell(ix, iy, nz, False, CTRL_BHP, 200.0 * BAR))
    return _finish("c2" if nz_override is None else f"c2_nz{nz}", nx, ny, nz,
                   20 * FT, 10 * FT, 2 * FT, poro, k, k.copy(), k.copy(), wells,
                   [5 * DAY] * 100)


def case_c3(seed: int = 3, nz_override: Optional[int] = None) -> Case:
    """200x200x50 lognormal field (sigma 2, correlation 5x5x2 cells, geometric
    mean 100 mD), 10x10x2 m blocks; 5x5 line drive at x,y in
    {20,60,100,140,180}: lines x=20,100,180 inject (500 m^3/d, C=1), lines
    x=60,140 produce at 200 bar BHP; 50 x 5 d.  ``nz_override`` keeps the
    top layers of the same field and the injection rate per perforated
    layer (a slice a direct solver can take)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz_full = 200, 200, 50
    nz = nz_full if nz_override is None else int(nz_override)
    g = gaussian_field(rng, (nz_full, ny, nx), (2.0, 5.0, 5.0))
    log10k = np.clip((math.log(100.0) + 2.0 * g) / math.log(10.0), -1.0, 4.0)
    k = (10.0 ** log10k) * MD
    poro = _poro_from_logk(rng, log10k)
    k, poro = k[:nz], poro[:nz]
    wells = []
    pos = [20, 60, 100, 140, 180]
    q_inj = 500.0 / DAY if nz == nz_full else 500.0 / DAY * nz / nz_full
    for li, x in enumerate(pos):
        for y in pos:
            if li % 2 == 0:
                wells.append(_vwell(x, y, nz, True, CTRL_WRATE, q_inj, 1.0))
            else:
                wells.append(_vwell(x, y, nz, False, CTRL_BHP, 200.0 * BAR))
    return _finish("c3" if nz_override is None else f"c3_nz{nz}", nx, ny, nz, 10.0, 10.0, 2.0, poro,
                   k, k.copy(), k.copy(), wells, [5 * DAY] * 50)


def case_c5(seed: int = 5, n_override: Optional[int] = None) -> Case:
    """300^3 lognormal field (sigma 2.5, correlation 20 cells horizontally and
    10 vertically), 10x10x1 m blocks; 100 vertical wells on a 10x10 lattice
    (spacing 30, offset 15) alternating polymer injection (1000 m^3/d, C=1)
    and production (200 bar BHP) in a checkerboard; 20 x 10 d."""
    rng = np.random.default_rng(seed)
    n = 300 if n_override is None else int(n_override)
    nx = ny = nz = n
    g = gaussian_field(rng, (nz, ny, nx), (10.0, 20.0, 20.0))
    log10k = np.clip((math.log(100.0) + 2.5 * g) / math.log(10.0), -1.0, 4.0)
    del g
    k = (10.0 ** log10k) * MD
    poro = _poro_from_logk(rng, log10k)
    del log10k
    wells = []
    sp = max(n // 10, 1)
    for a in range(10):
        for b in range(10):
            ix = min(sp // 2 + a * sp, nx - 1)
            iy = min(sp // 2 + b * sp, ny - 1)
            if (a + b) % 2 == 0:
                wells.append(_vwell(ix, iy, nz, True, CTRL_WRATE, 1000.0 / DAY, 1.0))
            else:
                wells.append(_vwell(ix, iy, nz, False, CTRL_BHP, 200.0 * BAR))
    return _finish("c5" if n_override is None else f"c5_n{n}", nx, ny, nz,
                   10.0, 10.0, 1.0, poro, k, k, k, wells, [10 * DAY] * 20)


# the paper's performance-test reservoir (Sec. 4.2, Table 3): porosity and
# directional permeabilities (mD) of its five layers, top to bottom
TABLE3_LAYERS = [(0.17393, 326.4, 980.6, 163.4),
                 (0.1694, 445.3, 1335.8, 222.6),
                 (0.25714, 148.9, 446.6, 74.4),
                 (0.17344, 118.8, 356.4, 59.4),
                 (0.1187, 71.2, 213.6, 35.6)]


def case_paper(nx: int, ny: int, nz: int, name: str, dt_days: float = 10.0) -> Case:
    """The reservoir of the paper's performance tests (Sec. 4.2.1, 4.2.2):
    Table 3's five layers (each split into nz/5 sub-layers of the same
    properties), initial pressure 4000 psi at 6150 ft, four vertical water
    injectors at the corners and a horizontal producer along x at the centre;
    3980 days of water flood, then polymer (C = 1 kg/m^3) for 360 days.
    Not given by the paper, taken here: one 1900 x 3840 x 25 m domain for
    every resolution; injectors on 1890 m^3/d of water each (about one pore
    volume over the schedule) with an upper BHP limit of 6000 psi; the
    producer at 3000 psi BHP along the middle half of the centre row of the
    middle layer."""
    assert nz % 5 == 0
    sub = nz // 5
    Lx, Ly, Lz = 1900.0, 3840.0, 25.0
    dx, dy, dz = Lx / nx, Ly / ny, Lz / nz
    poro = np.empty((nz, ny, nx))
    kx = np.empty((nz, ny, nx))
    ky = np.empty((nz, ny, nx))
    kz = np.empty((nz, ny, nx))
    for k in range(nz):
        ph, px, py, pz = TABLE3_LAYERS[k // sub]
        poro[k], kx[k], ky[k], kz[k] = ph, px * MD, py * MD, pz * MD
    q = 1890.0 / DAY
    lim = 6000.0 * PSI
    wells = [Well(ix, iy, 0, nz - 1, True, CTRL_WRATE, q, c_inj=0.0, bhp_limit=lim)
             for ix, iy in ((0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1))]
    kmid = nz // 2
    wells.append(Well(nx // 4, ny // 2, kmid, kmid, False, CTRL_BHP, 3000.0 * PSI,
                      direction=WELL_X, ix_last=(3 * nx) // 4))
    n_water = int(round(3980.0 / dt_days))
    n_poly = int(round(360.0 / dt_days))
    dts = [dt_days * DAY] * (n_water + n_poly)
    c = _finish(name, nx, ny, nz, dx, dy, dz, poro, kx, ky, kz, wells, dts)
    c.events = [(n_water, w, dict(c_inj=1.0)) for w in range(4)]
    return c


def case_paper_low() -> Case:
    """Sec. 4.2.1: 95 x 192 x 5 (91,200 blocks)."""
    return case_paper(95, 192, 5, "paper_low")


def case_paper_high() -> Case:
    """Sec. 4.2.2: the same reservoir refined to 951 x 1920 x 15 (27,388,800 blocks)."""
    return case_paper(951, 1920, 15, "paper_high")


def serving_realisation(r: int, size_seed: int = 4) -> Case:
    """Realisation ``r`` of the 64-realisation serving batch: N ~ U(20k, 500k),
    nz ~ U{5..50}, aspect nx/ny ~ U(0.5, 2); 10x10x2 m blocks; lognormal
    sigma 1.5 with 4-cell correlation; injector/producer at opposite corners,
    injection 10 m^3/d per perforated layer with C=1, producer at 200 bar;
    20 x 5 d."""
    srng = np.random.default_rng(size_seed)
    draws = srng.uniform(size=(64, 3))
    u = draws[r % 64]
    ncell = 20000 + u[0] * (500000 - 20000)
    nz = 5 + int(u[1] * 46)
    aspect = 0.5 + 1.5 * u[2]
    nx = max(int(round(math.sqrt(ncell / nz * aspect))), 2)
    ny = max(int(round(ncell / (nz * nx))), 2)
    rng = np.random.default_rng(1000 + r)
    g = gaussian_field(rng, (nz, ny, nx), (4.0, 4.0, 4.0))
    log10k = np.clip((math.log(100.0) + 1.5 * g) / math.log(10.0), -1.0, 4.0)
    k = (10.0 ** log10k) * MD
    poro = _poro_from_logk(rng, log10k)
    wells = [_vwell(0, 0, nz, True, CTRL_WRATE, 10.0 * nz / DAY, 1.0),
             _vwell(nx - 1, ny - 1, nz, False, CTRL_BHP, 200.0 * BAR)]
    return _finish(f"c4_r{r}", nx, ny, nz, 10.0, 10.0, 2.0, poro, k, k.copy(), k.copy(),
                   wells, [5 * DAY] * 20)


def serving_arrivals(n: int = 64, rate_per_s: float = 1.0, seed: int = 4) -> np.ndarray:
    """Poisson arrival times (s) for the serving batch."""
    rng = np.random.default_rng(seed + 7)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, n))


# --- small cases for tests ------------------------------------------------------
def box_case(nx, ny, nz, seed=0, dx=20.0, dy=20.0, dz=5.0, sigma=1.0, mean_md=100.0,
             wells: Optional[List[Well]] = None, dts=None, corr=(0.0, 0.0, 0.0),
             anisotropy=(1.0, 1.0, 1.0), fluid=None, polymer=None,
             poro_range=(0.2, 0.3)) -> Case:
    """Small heterogeneous box with a default quarter-five-spot (water-rate
    polymer injector at (0,0), BHP producer at the far corner)."""
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    poro = rng.uniform(poro_range[0], poro_range[1], shape)
    g = gaussian_field(rng, shape, corr)
    k = np.exp(math.log(mean_md) - 0.5 * sigma * sigma + sigma * g) * MD
    if wells is None:
        wells = [_vwell(0, 0, nz, True, CTRL_WRATE, 20.0 / DAY * nz, 1.0),
                 _vwell(nx - 1, ny - 1, nz, False, CTRL_BHP, 200.0 * BAR)]
    if dts is None:
        dts = [DAY] * 5
    return _finish(f"box{nx}x{ny}x{nz}", nx, ny, nz, dx, dy, dz, poro,
                   k * anisotropy[0], k * anisotropy[1], k * anisotropy[2],
                   wells, dts, fluid=fluid, polymer=polymer)


def make_case(name: str, seed: Optional[int] = None) -> Case:
    if name == "c1":
        return case_c1(1 if seed is None else seed)
    if name == "c2":
        return case_c2(2 if seed is None else seed)
    if name == "c3":
        return case_c3(3 if seed is None else seed)
    if name == "c5":
        return case_c5(5 if seed is None else seed)
    if name.startswith("c4_r"):
        return serving_realisation(int(name[4:]))
    raise KeyError(name)


def build_case(name, nx, ny, nz, dx, dy, dz, poro, k, wells, dts, fluid=None, polymer=None,
               P0=None, S0=None, C0=None, Pb0=None, top=DEFAULT_TOP, p_top=DEFAULT_PTOP,
               cr=1.0e-6 / BAR, kxyz=None) -> Case:
    """Explicit case for tests: scalar or per-cell porosity / permeability,
    optional explicit initial state (defaults as in the named workloads)."""
    n = nx * ny * nz
    poro = np.broadcast_to(np.asarray(poro, dtype=np.float64), (n,)).copy()
    if kxyz is None:
        kk = np.broadcast_to(np.asarray(k, dtype=np.float64), (n,)).copy()
        kx, ky, kz = kk, kk.copy(), kk.copy()
    else:
        kx, ky, kz = (np.broadcast_to(np.asarray(a, dtype=np.float64), (n,)).copy() for a in kxyz)
    c = _finish(name, nx, ny, nz, dx, dy, dz, poro, kx, ky, kz, list(wells), dts,
                fluid=fluid, polymer=polymer, top=top, p_top=p_top, cr=cr)
    if P0 is not None:
        c.P0 = np.broadcast_to(np.asarray(P0, dtype=np.float64), (n,)).copy()
    if S0 is not None:
        c.S0 = np.broadcast_to(np.asarray(S0, dtype=np.float64), (n,)).copy()
    if C0 is not None:
        c.C0 = np.broadcast_to(np.asarray(C0, dtype=np.float64), (n,)).copy()
    if Pb0 is not None:
        c.Pb0 = np.asarray(Pb0, dtype=np.float64).copy()
    return c


def sub_box(case: Case, x0: int, x1: int, y0: int, y1: int, z0: int, z1: int, name: str = "") -> Case:
    """The cells [x0, x1) x [y0, y1) x [z0, z1) of a case as a case of their
    own: the same rock, fluids and timestep schedule, the initial state of
    those cells, the vertical wells whose column lies inside (perforations
    clipped to the layers kept, a rate target scaled by the fraction of its
    perforations kept, so the rate per perforation is that of the full
    model).  For bounded samples of a large workload."""
    nx, ny, nz = x1 - x0, y1 - y0, z1 - z0
    assert 0 <= x0 < x1 <= case.nx and 0 <= y0 < y1 <= case.ny and 0 <= z0 < z1 <= case.nz

    def cut(a):
        return np.ascontiguousarray(a.reshape(case.nz, case.ny, case.nx)[z0:z1, y0:y1, x0:x1].reshape(-1))

    wells, pb0 = [], []
    for w, pb in zip(case.wells, case.Pb0):
        if w.direction != WELL_Z or not (x0 <= w.ix < x1 and y0 <= w.iy < y1):
            continue
        k0, k1 = max(w.k_top, z0), min(w.k_bot, z1 - 1)
        if k0 > k1:
            continue
        frac = (k1 - k0 + 1) / (w.k_bot - w.k_top + 1)
        target = w.target if w.control == CTRL_BHP or frac == 1.0 else w.target * frac
        wells.append(dataclasses.replace(w, ix=w.ix - x0, iy=w.iy - y0, k_top=k0 - z0, k_bot=k1 - z0,
                                         target=target))
        pb0.append(pb)
    top = case.top + z0 * case.dz
    return Case(name=name or f"{case.name}_sub{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, dx=case.dx, dy=case.dy,
                dz=case.dz, top=top, poro=cut(case.poro), kx=cut(case.kx), ky=cut(case.ky), kz=cut(case.kz),
                cr=case.cr, p_ref=case.p_ref, fluid=dataclasses.replace(case.fluid),
                polymer=dataclasses.replace(case.polymer), wells=wells, P0=cut(case.P0), S0=cut(case.S0),
                C0=cut(case.C0), Pb0=np.asarray(pb0, dtype=np.float64), dts=case.dts.copy())
