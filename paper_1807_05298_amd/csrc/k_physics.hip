// Physics kernels: static set-up, accumulation, residual + Jacobian assembly,
// well terms, convergence norms and the chopped Newton update.
//
// One thread per cell, cell-gather form: every cell evaluates its own
// accumulation and the six faces around it (each face in its canonical
// lower-index/higher-index orientation, so both cells of a face use the same
// flux), then writes its residual row and its seven 3x3 Jacobian blocks.  No
// atomics; every value is written by exactly one thread.  Derivatives are
// the analytic derivatives of the selected upstream branch.
#include "pf_internal.h"

#include <algorithm>
#include <cfloat>
#include <vector>

namespace pf {
namespace {

// ---------------------------------------------------------------------------
// Cell properties (Sec. 2.1 rock, 2.2 fluid, 2.3 polymer) with derivatives:
// d/dP for porosity and densities, d/dS for relative permeabilities, d/dC
// for viscosities, adsorption and permeability reduction.
// 1/b from the hardware reciprocal estimate refined by two Newton-Raphson
// steps y <- y + y (1 - b y) (each roughly doubles the correct bits), within
// an ulp of the quotient; about half the instructions of a full division.
// For the positive, normal operands of the assembly (pore volumes,
// viscosities, permeability reduction factors).
__device__ __forceinline__ double rcp_nr(double b) {
    double y = __builtin_amdgcn_rcp(b);
    double e = fma(-b, y, 1.0);
    y = fma(y, e, y);
    e = fma(-b, y, 1.0);
    return fma(y, e, y);
}

// exp(x) for the density law.  Its exponents c (P - P_ref) are small (c is
// 1e-6..1e-5 per bar), so for |x| <= 1/16 the Taylor polynomial of degree 8
// is used: its truncation error is below x^9/9! e^{2|x|} < 4.6e-17 relative,
// under half an ulp; Horner adds a few roundings.  Larger |x| calls exp.
__device__ __forceinline__ double exp_density(double x) {
    if (fabs(x) > 0.0625) return exp(x);
    double p = 1.0 / 40320.0;
    p = fma(p, x, 1.0 / 5040.0);
    p = fma(p, x, 1.0 / 720.0);
    p = fma(p, x, 1.0 / 120.0);
    p = fma(p, x, 1.0 / 24.0);
    p = fma(p, x, 1.0 / 6.0);
    p = fma(p, x, 0.5);
    p = fma(p, x, 1.0);
    return fma(p, x, 1.0);
}

struct CellP {
    double phi;
    double rw, drw, ro, dro;
    double krw, dkrw, kro, dkro;
    double muwe, dmuwe, mupe, dmupe;
    double ads, dads, rk, drk;
    double pc, dpc;                  // capillary pressure P_o - P_w and dPc/dS
};

// Piecewise-linear table of n points (x strictly increasing): the segment
// [x_k, x_k+1) holding v gives value and slope; outside the table the end
// value holds with slope 0.
__device__ __forceinline__ void table_eval(const double* x, const double* y, int n, double v, double& f,
                                           double& df) {
    if (v < x[0]) { f = y[0]; df = 0.0; return; }
    if (v >= x[n - 1]) { f = y[n - 1]; df = 0.0; return; }
    int k = 0;
    while (k + 2 < n && v >= x[k + 1]) ++k;
    df = (y[k + 1] - y[k]) / (x[k + 1] - x[k]);
    f = y[k] + df * (v - x[k]);
}

// Equilibrium adsorption of cell i at concentration C and its slope: the
// Langmuir isotherm or the table, scaled by the rock's capacity A_d,max /
// ads_max when the rock table is in use (VAR).
template <bool VAR>
__device__ __forceinline__ void isotherm(const DevModel& m, int64_t i, double C, double& a, double& da) {
    if (!VAR || m.n_ads == 0) {
        const double iden = rcp_nr(1.0 + m.ads_b * C);
        const double amb = m.ads_max * m.ads_b;
        a = amb * C * iden;
        da = amb * iden * iden;
    } else {
        table_eval(m.tab + kTabAdsC * PF_TABLE_MAX, m.tab + kTabAdsA * PF_TABLE_MAX, m.n_ads, C, a, da);
    }
    if (VAR && m.cell_cap) {
        const double cap = m.cell_cap[i];
        a *= cap;
        da *= cap;
    }
}

// VAR: the model may use a mixing rule other than the polynomial, tables,
// capillary pressure, retention or the rock table; without VAR those
// branches are compiled out (the plain model's arithmetic is the same on both
// paths).  i: the cell (its rock values and adsorption history).
template <bool VAR = true>
__device__ __forceinline__ CellP cell_props(const DevModel& m, double phir, double P, double S, double C,
                                            int64_t i) {
    CellP p;
    const double dp = P - m.pref;
    p.phi = phir + m.cr * dp;
    p.rw = m.rho_w0 * exp_density(m.c_w * dp);
    p.drw = m.c_w * p.rw;
    p.ro = m.rho_o0 * exp_density(m.c_o * dp);
    p.dro = m.c_o * p.ro;
    // normalised saturation; the interior formula applies on the closed
    // interval [swc, 1-sor], the clamped branches have zero slope
    double sn, dsn;
    if (S < m.swc) {
        sn = 0.0; dsn = 0.0;
    } else if (S > 1.0 - m.sor) {
        sn = 1.0; dsn = 0.0;
    } else {
        sn = (S - m.swc) * m.inv_den; dsn = m.inv_den;
    }
    const double on = 1.0 - sn;
    if (m.corey2_w) {
        p.krw = m.krw0 * sn * sn;
        p.dkrw = 2.0 * m.krw0 * sn * dsn;
    } else {
        const double t = pow(sn, m.n_w - 1.0);
        p.krw = m.krw0 * t * sn;
        p.dkrw = m.krw0 * m.n_w * t * dsn;
    }
    if (m.corey2_o) {
        p.kro = m.kro0 * on * on;
        p.dkro = -2.0 * m.kro0 * on * dsn;
    } else {
        const double t = pow(on, m.n_o - 1.0);
        p.kro = m.kro0 * t * on;
        p.dkro = -m.kro0 * m.n_o * t * dsn;
    }
    // fully mixed viscosity mu_m(C) by the mixing rule, then the
    // Todd-Longstaff effective viscosities
    double mum, dmum;
    if (!VAR || m.mix_rule == PF_MIX_POLY) {
        mum = m.mu_w * (1.0 + C * (m.a1 + m.a2 * C));
        dmum = m.mu_w * (m.a1 + 2.0 * m.a2 * C);
    } else if (m.mix_rule == PF_MIX_LINEAR) {
        const double beta = C / m.cmax;
        mum = beta * m.mup_ref + (1.0 - beta) * m.mu_w;
        dmum = (m.mup_ref - m.mu_w) / m.cmax;
    } else if (m.mix_rule == PF_MIX_EXP) {
        // mu_p^ref^beta mu_w^(1-beta) = mu_w exp(beta ln(mu_p^ref / mu_w))
        mum = m.mu_w * exp(C / m.cmax * m.mix_ln);
        dmum = mum * m.mix_ln / m.cmax;
    } else {
        double f, df;
        table_eval(m.tab + kTabViscC * PF_TABLE_MAX, m.tab + kTabViscM * PF_TABLE_MAX, m.n_visc, C, f, df);
        mum = m.mu_w * f;
        dmum = m.mu_w * df;
    }
    if (m.omega1) {
        p.mupe = mum; p.dmupe = dmum;
        p.muwe = mum; p.dmuwe = dmum;
    } else {
        const double mo = pow(mum, m.omega);
        const double dmo = m.omega * mo / mum * dmum;
        p.mupe = mo * m.tl_pref;
        p.dmupe = dmo * m.tl_pref;
        const double mwp = mo * m.tl_pw;
        const double dmwp = dmo * m.tl_pw;
        const double a = C / m.cmax, da = 1.0 / m.cmax;
        const double inv = a / p.mupe + (1.0 - a) / mwp;
        const double dinv = da / p.mupe - a * p.dmupe / (p.mupe * p.mupe)
                          - da / mwp - (1.0 - a) * dmwp / (mwp * mwp);
        p.muwe = 1.0 / inv;
        p.dmuwe = -dinv / (inv * inv);
    }
    // adsorption (equilibrium, or the retained part of the largest past
    // adsorption where that is more) and permeability reduction
    isotherm<VAR>(m, i, C, p.ads, p.dads);
    if (VAR && m.ads_hist) {
        const double held = m.ads_res * m.ads_hist[i];
        if (held > p.ads) { p.ads = held; p.dads = 0.0; }
    }
    const double rks = (VAR && m.cell_rks) ? m.cell_rks[i] : m.rk_slope;
    p.rk = 1.0 + rks * p.ads;
    p.drk = rks * p.dads;
    if (!VAR || m.n_pc == 0) { p.pc = 0.0; p.dpc = 0.0; }
    else table_eval(m.tab + kTabPcS * PF_TABLE_MAX, m.tab + kTabPcV * PF_TABLE_MAX, m.n_pc, S, p.pc, p.dpc);
    return p;
}

// Accumulation M (kg) and dM/d(P,S,C) of one cell.  Here, in the face flux
// and in the perforation rates the oil equation's derivative w.r.t. C is
// exactly zero (polymer moves with the water phase only); the kernels that
// stream J skip that entry of every block.
__device__ __forceinline__ void accumulation(const DevModel& m, const CellP& p, double S, double C,
                                             double M[3], double dM[9]) {
    const double v = m.vol;
    const double acc = 1.0 - m.ipv;
    M[0] = v * p.phi * S * p.rw;
    dM[0] = v * (m.cr * S * p.rw + p.phi * S * p.drw);
    dM[1] = v * p.phi * p.rw;
    dM[2] = 0.0;
    M[1] = v * p.phi * (1.0 - S) * p.ro;
    dM[3] = v * (m.cr * (1.0 - S) * p.ro + p.phi * (1.0 - S) * p.dro);
    dM[4] = -v * p.phi * p.ro;
    dM[5] = 0.0;
    const double cw = C * m.inv_rho_w0;
    M[2] = v * (p.phi * acc * S * p.rw * cw + (1.0 - p.phi) * p.ads);
    dM[6] = v * (acc * S * cw * (m.cr * p.rw + p.phi * p.drw) - m.cr * p.ads);
    dM[7] = v * p.phi * acc * p.rw * cw;
    dM[8] = v * (p.phi * acc * S * p.rw * m.inv_rho_w0 + (1.0 - p.phi) * p.dads);
}

// Face flux (kg/s, L -> R, Sec. 3.2) and its derivatives w.r.t. the
// unknowns of the two cells.  dA: derivatives w.r.t. cell "a" (the cell
// doing the gather), dB: w.r.t. the neighbour "b".  aIsL tells which of the
// two is the lower-index cell L.  Derivative arrays are [eq*3 + var].
__device__ __forceinline__ void face_flux(const DevModel& m, double T, double wL, double gdz, bool aIsL,
                                          double Pa, double Ca, const CellP& a,
                                          double Pb, double Cb, const CellP& b,
                                          double F[3], double dA[9], double dB[9]) {
    // orient: L/R quantities
    const double PL = aIsL ? Pa : Pb, PR = aIsL ? Pb : Pa;
    const double wR = 1.0 - wL;
    const double wa = aIsL ? wL : wR;          // averaging weight of cell a
    const double wb = aIsL ? wR : wL;
    const double rw = wa * a.rw + wb * b.rw;
    const double ro = wa * a.ro + wb * b.ro;
    const double muw = wa * a.muwe + wb * b.muwe;
    const double mup = wa * a.mupe + wb * b.mupe;
    // potential difference (R minus L), depth positive downward; the water
    // phase pressure is P - P_c(S)
    const double pcL = aIsL ? a.pc : b.pc, pcR = aIsL ? b.pc : a.pc;
    const double dpw = ((PR - pcR) - (PL - pcL)) - rw * gdz;
    const double dpo = (PR - PL) - ro * gdz;
    // d(P_R - P_L)/dP_a
    const double sa = aIsL ? -1.0 : 1.0;
    const double ddpw_a = sa - wa * a.drw * gdz, ddpw_b = -sa - wb * b.drw * gdz;
    const double ddpo_a = sa - wa * a.dro * gdz, ddpo_b = -sa - wb * b.dro * gdz;
    // upstream cell: higher potential; a tie selects R
    const bool upR_w = dpw >= 0.0;
    const bool upR_o = dpo >= 0.0;
    const bool wa_up = (upR_w != aIsL);        // cell a is upstream for water
    const bool oa_up = (upR_o != aIsL);
    const double krw = wa_up ? a.krw : b.krw;
    const double dkrw = wa_up ? a.dkrw : b.dkrw;
    const double rk = wa_up ? a.rk : b.rk;
    const double drk = wa_up ? a.drk : b.drk;
    const double Cup = wa_up ? Ca : Cb;
    const double kro = oa_up ? a.kro : b.kro;
    const double dkro = oa_up ? a.dkro : b.dkro;
    // one reciprocal each, then products (FP64 division is a long sequence)
    const double irk = rcp_nr(rk);
    const double imuw = rcp_nr(muw);
    const double imup = rcp_nr(mup);
    // water
    const double mw = krw * irk * imuw;
    const double Gw = -T * rw * dpw;
    F[0] = Gw * mw;
    dA[0] = -T * mw * (wa * a.drw * dpw + rw * ddpw_a);
    dB[0] = -T * mw * (wb * b.drw * dpw + rw * ddpw_b);
    const double dmw_S = Gw * dkrw * irk * imuw;
    // d(dpw)/dS_a = -sa dPc_a, d(dpw)/dS_b = sa dPc_b (capillary pressure)
    const double gs_a = T * rw * sa * a.dpc, gs_b = -T * rw * sa * b.dpc;
    dA[1] = (wa_up ? dmw_S : 0.0) + gs_a * mw;
    dB[1] = (wa_up ? 0.0 : dmw_S) + gs_b * mw;
    const double rkterm = drk * irk;
    dA[2] = Gw * mw * (-(wa_up ? rkterm : 0.0) - wa * a.dmuwe * imuw);
    dB[2] = Gw * mw * (-(wa_up ? 0.0 : rkterm) - wb * b.dmuwe * imuw);

    // oil
    const double mo = kro * m.inv_mu_o;
    const double Go = -T * ro * dpo;
    F[1] = Go * mo;
    dA[3] = -T * mo * (wa * a.dro * dpo + ro * ddpo_a);
    dB[3] = -T * mo * (wb * b.dro * dpo + ro * ddpo_b);
    const double dmo_S = Go * dkro * m.inv_mu_o;
    dA[4] = oa_up ? dmo_S : 0.0;
    dB[4] = oa_up ? 0.0 : dmo_S;
    dA[5] = 0.0;
    dB[5] = 0.0;

    // polymer: carried by the water flux with the upstream concentration
    // as mass fraction C/rho_w0 and the polymer effective viscosity
    const double mp = krw * irk * imup;
    const double cf = Cup * m.inv_rho_w0;
    F[2] = Gw * mp * cf;
    dA[6] = -T * mp * cf * (wa * a.drw * dpw + rw * ddpw_a);
    dB[6] = -T * mp * cf * (wb * b.drw * dpw + rw * ddpw_b);
    const double dmp_S = Gw * cf * dkrw * irk * imup;
    dA[7] = (wa_up ? dmp_S : 0.0) + gs_a * mp * cf;
    dB[7] = (wa_up ? 0.0 : dmp_S) + gs_b * mp * cf;
    const double gp = Gw * mp;
    dA[8] = gp * cf * (-(wa_up ? rkterm : 0.0) - wa * a.dmupe * imup) + (wa_up ? gp * m.inv_rho_w0 : 0.0);
    dB[8] = gp * cf * (-(wa_up ? 0.0 : rkterm) - wb * b.dmupe * imup) + (wa_up ? 0.0 : gp * m.inv_rho_w0);
}

__device__ __forceinline__ double row_scale(const DevModel& m, int e, double pvr) {
    const double c = (e == 0) ? m.rho_w0 : (e == 1) ? m.rho_o0 : m.c_ref;
    return 1.0 / (c * pvr);
}

// the three row scales 1/(rho_w0 PV), 1/(rho_o0 PV), 1/(C_ref PV) from one reciprocal
__device__ __forceinline__ void row_scales(const DevModel& m, double pvr, double sc[3]) {
    const double ipv = rcp_nr(pvr);
    sc[0] = ipv * m.inv_rho_w0;
    sc[1] = ipv * m.inv_rho_o0;
    sc[2] = ipv * m.inv_c_ref;
}

// ---------------------------------------------------------------------------
__device__ __forceinline__ void k_static_cells_d(const Blk& wg, DevModel m, const double* __restrict__ poro,
                                                 const double* __restrict__ kx, const double* __restrict__ ky,
                                                 const double* __restrict__ kz, double* __restrict__ pvr,
                                                 double* __restrict__ Tx, double* __restrict__ Ty,
                                                 double* __restrict__ Tz, double* __restrict__ rscale) {
    const int64_t i = (int64_t)wg.x * blockDim.x + threadIdx.x;
    if (i >= m.n) return;
    const int64_t iz = i / m.nxy;
    const int64_t rem = i - iz * m.nxy;
    const int64_t iy = rem / m.nx;
    const int64_t ix = rem - iy * m.nx;
    const double pv = poro[i] * m.vol;
    pvr[i] = pv;
    // harmonic interface transmissibility: area / (sum of half-cell resistances)
    Tx[i] = (ix + 1 < m.nx) ? (m.dy * m.dz) / (0.5 * m.dx / kx[i] + 0.5 * m.dx / kx[i + 1]) : 0.0;
    Ty[i] = (iy + 1 < m.ny) ? (m.dx * m.dz) / (0.5 * m.dy / ky[i] + 0.5 * m.dy / ky[i + m.nx]) : 0.0;
    Tz[i] = (iz + 1 < m.nz) ? (m.dx * m.dy) / (0.5 * m.dz / kz[i] + 0.5 * m.dz / kz[i + m.nxy]) : 0.0;
    rscale[i] = 1.0 / (m.rho_w0 * pv);
    rscale[m.n + i] = 1.0 / (m.rho_o0 * pv);
    rscale[2 * m.n + i] = 1.0 / (m.c_ref * pv);
}
__global__ void k_static_cells(DevModel m, const double* __restrict__ poro, const double* __restrict__ kx,
                               const double* __restrict__ ky, const double* __restrict__ kz, double* __restrict__ pvr,
                               double* __restrict__ Tx, double* __restrict__ Ty, double* __restrict__ Tz,
                               double* __restrict__ rscale) {
    k_static_cells_d(PF_BLK, m, poro, kx, ky, kz, pvr, Tx, Ty, Tz, rscale);
}
struct F_k_static_cells {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_static_cells_d(wg, a...);
    }
};

// Peaceman index of a perforation of a vertical well (eq:wi and
// eq:wi:re:k with the roles of the axes permuted to a z-direction well).
// Peaceman well index (eq:wi with f = f_h = 1, eq:wi:re:k): across the well
// the permeabilities (ka, kb) and block sizes (ha, hb), along it h.  For a
// well along x: (ky, kz, dy, dz) and h = dx, the formula as printed; for a
// vertical well the same with (y, z) replaced by (x, y) and h = dz.
__device__ __forceinline__ void k_static_perfs_d(const Blk& wg, DevModel m, const int32_t* __restrict__ perf_cell,
                                                 const int32_t* __restrict__ perf_well,
                                                 const int32_t* __restrict__ w_dir, const double* __restrict__ w_rw,
                                                 const double* __restrict__ w_skin, const double* __restrict__ kx,
                                                 const double* __restrict__ ky, const double* __restrict__ kz,
                                                 double* __restrict__ perf_wi) {
    const int64_t p = (int64_t)wg.x * blockDim.x + threadIdx.x;
    if (p >= m.np) return;
    const int64_t c = perf_cell[p];
    const int w = perf_well[p];
    const bool along_x = w_dir[w] == PF_WELL_X;
    const double ka = along_x ? ky[c] : kx[c], kb = along_x ? kz[c] : ky[c];
    const double ha = along_x ? m.dy : m.dx, hb = along_x ? m.dz : m.dy, h = along_x ? m.dx : m.dz;
    const double gf = 0.249;
    const double rba = sqrt(kb / ka), rab = sqrt(ka / kb);
    const double num = sqrt(rba * ha * ha + rab * hb * hb);
    const double den = sqrt(rba) + sqrt(rab);          // (kb/ka)^(1/4) + (ka/kb)^(1/4)
    const double re = 2.0 * gf / sqrt(M_PI) * num / den;
    perf_wi[p] = 2.0 * M_PI * h * sqrt(ka * kb) / (log(re / w_rw[w]) + w_skin[w]);
}
__global__ void k_static_perfs(DevModel m, const int32_t* __restrict__ perf_cell,
                               const int32_t* __restrict__ perf_well, const int32_t* __restrict__ w_dir,
                               const double* __restrict__ w_rw, const double* __restrict__ w_skin,
                               const double* __restrict__ kx, const double* __restrict__ ky,
                               const double* __restrict__ kz, double* __restrict__ perf_wi) {
    k_static_perfs_d(PF_BLK, m, perf_cell, perf_well, w_dir, w_rw, w_skin, kx, ky, kz, perf_wi);
}
struct F_k_static_perfs {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_static_perfs_d(wg, a...);
    }
};

__device__ __forceinline__ void k_accum_d(const Blk& wg, DevModel m, const double* __restrict__ x,
                                          const double* __restrict__ pvr, double* __restrict__ M) {
    const int64_t i = (int64_t)wg.x * blockDim.x + threadIdx.x;
    if (i >= m.n) return;
    const double P = x[i], S = x[m.n + i], C = x[2 * m.n + i];
    const CellP p = cell_props(m, pvr[i] / m.vol, P, S, C, i);
    double Mv[3], dM[9];
    accumulation(m, p, S, C, Mv, dM);
    M[i] = Mv[0];
    M[m.n + i] = Mv[1];
    M[2 * m.n + i] = Mv[2];
}
__global__ void k_accum(DevModel m, const double* __restrict__ x, const double* __restrict__ pvr,
                        double* __restrict__ M) {
    k_accum_d(PF_BLK, m, x, pvr, M);
}
struct F_k_accum {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_accum_d(wg, a...);
    }
};

// Residual (3 rows) and Jacobian (7 blocks) of every cell.
template <bool VAR>
__device__ __forceinline__ void k_assemble_d(const Blk& wg, DevModel m, const double* __restrict__ x,
                                             const double* __restrict__ Mn, const double* __restrict__ pvr,
                                             const double* __restrict__ Tx, const double* __restrict__ Ty,
                                             const double* __restrict__ Tz, double dt, double* __restrict__ R,
                                             double* __restrict__ J, int with_jac, double* __restrict__ Lcs,
                                             double* __restrict__ Jdcs) {
    // With Jdcs (FP64 red-black ILU(0) in PF order) the blocks go to the
    // colour-split storage that the smoother and the product stream, instead of
    // the natural-order planes of J: cell colour (ix+iy+iz)&1, slot
    // (iy + ny*iz)*ceil(nx/2) + ix/2; diagonal blocks in Jdcs (9 planes per
    // colour), face f's block in Lcs (54 planes per colour).  The threads are
    // then colour-major: a wavefront takes 64 consecutive slots of one colour
    // and the next one the same slots of the other colour, so that every store
    // into that storage is one whole run and the pair reads the same lines of
    // the natural-order inputs.
    const bool cs = Jdcs != nullptr;
    const int64_t nsl = cs_ns(m);
    const int64_t n = m.n;
    int64_t i, ix, iy, iz, cl, sl;
    if (cs) {
        const int64_t nxh = (m.nx + 1) >> 1;
        const int64_t v = xcd_block(wg) * blockDim.x + threadIdx.x;
        const int64_t w = v >> 6;
        cl = w & 1;
        sl = (w >> 1) * 64 + (v & 63);
        if (sl >= nsl) return;
        const int64_t line = sl / nxh;
        iz = line / m.ny;
        iy = line - iz * m.ny;
        ix = 2 * (sl - line * nxh) + ((iy + iz + cl) & 1);
        if (ix >= m.nx) return;      // the pad slot of an odd-length line
        i = ix + m.nx * iy + m.nxy * iz;
    } else {
        i = xcd_block(wg) * blockDim.x + threadIdx.x;
        if (i >= n) return;
        iz = i / m.nxy;
        const int64_t rem = i - iz * m.nxy;
        iy = rem / m.nx;
        ix = rem - iy * m.nx;
        cl = (ix + iy + iz) & 1;
        sl = (iy + m.ny * iz) * ((m.nx + 1) >> 1) + (ix >> 1);
    }
    const double P = x[i], S = x[n + i], C = x[2 * n + i];
    const double pv = pvr[i];
    const CellP a = cell_props<VAR>(m, pv * m.inv_vol, P, S, C, i);
    double r[3], jd[9];
    accumulation(m, a, S, C, r, jd);
    r[0] -= Mn[i];
    r[1] -= Mn[n + i];
    r[2] -= Mn[2 * n + i];
    double sc[3];
    row_scales(m, pv, sc);

    // Face f's neighbour j and the cell holding the face value (lower index);
    // a missing face points at the cell itself so its loads stay valid.
    auto face_geom = [&](int f, bool& exists, int64_t& j, const double*& Tdir, int64_t& lo) {
        const int dir = f >> 1;
        const bool plus = (f & 1) != 0;
        int64_t stride;
        if (dir == 0) { exists = plus ? (ix + 1 < m.nx) : (ix > 0); stride = 1; Tdir = Tx; }
        else if (dir == 1) { exists = plus ? (iy + 1 < m.ny) : (iy > 0); stride = m.nx; Tdir = Ty; }
        else { exists = plus ? (iz + 1 < m.nz) : (iz > 0); stride = m.nxy; Tdir = Tz; }
        j = !exists ? i : (plus ? i + stride : i - stride);
        lo = plus ? i : j;
    };
    // software pipeline: the loads of face f + 1 are in flight while face f is computed.
    // R and J are written once and not read back here: streaming (non-temporal) stores.
    // Entry 5, (oil, C), of every block is zero: its planes were cleared when the
    // simulator was created and are not written here.
    bool ex_n;
    int64_t j_n, lo_n;
    const double* T_n;
    face_geom(0, ex_n, j_n, T_n, lo_n);
    double nP = x[j_n], nS = x[n + j_n], nC = x[2 * n + j_n], npv = pvr[j_n], nT = T_n[lo_n];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const bool plus = (f & 1) != 0;
        const bool exists = ex_n;
        const double Pj = nP, Sj = nS, Cj = nC, pvj = npv, T = nT;
        const int64_t j = j_n;
        if (f < 5) {
            face_geom(f + 1, ex_n, j_n, T_n, lo_n);
            nP = x[j_n]; nS = x[n + j_n]; nC = x[2 * n + j_n]; npv = pvr[j_n]; nT = T_n[lo_n];
        }
        // entry e of face f's block: natural-order plane, or the colour-split copy
        double* Jd = cs ? Lcs + (cl * 54 + f * 9) * nsl + sl : J + (int64_t)(f + 1) * 9 * n + i;
        const int64_t je = cs ? nsl : n;
        if (!exists) {
            if (with_jac)
                for (int e = 0; e < 9; ++e)
                    if (e != 5) __builtin_nontemporal_store(0.0, &Jd[e * je]);
            continue;
        }
        const double wL = (plus ? pv : pvj) * rcp_nr(pv + pvj);
        const double gdz = ((f >> 1) == 2) ? m.grav * m.dz : 0.0;
        const CellP b = cell_props<VAR>(m, pvj * m.inv_vol, Pj, Sj, Cj, j);
        double F[3], dA[9], dB[9];
        face_flux(m, T, wL, gdz, plus, P, C, a, Pj, Cj, b, F, dA, dB);
        const double sg = plus ? dt : -dt;               // outflow from L, inflow to R
        for (int e = 0; e < 3; ++e) r[e] += sg * F[e];
        for (int e = 0; e < 9; ++e) jd[e] += sg * dA[e];
        if (with_jac)
            for (int e = 0; e < 9; ++e)
                if (e != 5) __builtin_nontemporal_store(sg * dB[e] * sc[e / 3], &Jd[e * je]);
    }
    for (int e = 0; e < 3; ++e) __builtin_nontemporal_store(r[e] * sc[e], &R[e * n + i]);
    double* J0 = cs ? Jdcs + cl * 9 * nsl + sl : J + i;
    const int64_t j0e = cs ? nsl : n;
    if (with_jac)
        for (int e = 0; e < 9; ++e)
            if (e != 5) __builtin_nontemporal_store(jd[e] * sc[e / 3], &J0[e * j0e]);
}
template <bool VAR>
__global__ __launch_bounds__(256) void k_assemble(DevModel m, const double* __restrict__ x,
                                                  const double* __restrict__ Mn, const double* __restrict__ pvr,
                                                  const double* __restrict__ Tx, const double* __restrict__ Ty,
                                                  const double* __restrict__ Tz, double dt, double* __restrict__ R,
                                                  double* __restrict__ J, int with_jac, double* __restrict__ Lcs,
                                                  double* __restrict__ Jdcs) {
    k_assemble_d<VAR>(PF_BLK, m, x, Mn, pvr, Tx, Ty, Tz, dt, R, J, with_jac, Lcs, Jdcs);
}
template <bool VAR>
struct F_k_assemble {
    static constexpr int kLB = 256;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_assemble_d<VAR>(wg, a...);
    }
};

// Well terms of the perforated cells (eq:ssw:Q, eq:ssw:dp): one thread per
// perforated cell adds the rates of all its perforations to the residual
// and diagonal block, writes the border blocks and the per-perforation
// contribution to the well equations.
__device__ __forceinline__ void k_wells_d(const Blk& wg, DevModel m, const double* __restrict__ x,
                                          const double* __restrict__ pvr, const int32_t* __restrict__ pc_cell,
                                          const int32_t* __restrict__ pc_first, const int32_t* __restrict__ perf_well,
                                          const double* __restrict__ perf_wi, const double* __restrict__ perf_depth,
                                          const int32_t* __restrict__ w_inj, const int32_t* __restrict__ w_ctrl,
                                          const double* __restrict__ w_cinj, const double* __restrict__ w_gamma,
                                          const double* __restrict__ w_zref, const double* __restrict__ w_scale,
                                          double dt, double* __restrict__ R, double* __restrict__ J,
                                          double* __restrict__ B, double* __restrict__ Cw, double* __restrict__ wv,
                                          double* __restrict__ wdp, double* __restrict__ perf_q, int with_jac,
                                          double* __restrict__ Jdcs) {
    const int64_t t = (int64_t)wg.x * blockDim.x + threadIdx.x;
    if (t >= m.npc) return;
    const int64_t n = m.n;
    const int64_t i = pc_cell[t];
    const double P = x[i], S = x[n + i], C = x[2 * n + i];
    const double pv = pvr[i];
    const CellP p = cell_props(m, pv / m.vol, P, S, C, i);
    const double sc0 = row_scale(m, 0, pv), sc1 = row_scale(m, 1, pv), sc2 = row_scale(m, 2, pv);
    const double lw = p.krw / (p.rk * p.muwe);
    const double dlw_S = p.dkrw / (p.rk * p.muwe);
    const double dlw_C = -lw * (p.drk / p.rk + p.dmuwe / p.muwe);
    const double lo = p.kro / m.mu_o;
    const double dlo_S = p.dkro / m.mu_o;
    double dr[3] = {0.0, 0.0, 0.0};
    double dj[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t k = pc_first[t]; k < pc_first[t + 1]; ++k) {
        const int w = perf_well[k];
        const double wi = perf_wi[k];
        const double pb = x[3 * n + w];
        const double draw = pb + w_gamma[w] * (perf_depth[k] - w_zref[w]) - P;
        double q[3], dq[12];   // dq[e*4 + (P,S,C,Pb)]
        // injection when the wellbore pressure is at or above the cell's; an
        // injector perforation below it produces the cell's fluids (eq:ssw:Q)
        if (w_inj[w] && draw >= 0.0) {
            const double lt = lw + lo;
            q[0] = wi * lt * p.rw * draw;
            dq[0] = wi * lt * (p.drw * draw - p.rw);
            dq[1] = wi * (dlw_S + dlo_S) * p.rw * draw;
            dq[2] = wi * dlw_C * p.rw * draw;
            dq[3] = wi * lt * p.rw;
            q[1] = 0.0;
            dq[4] = dq[5] = dq[6] = dq[7] = 0.0;
            const double f = w_cinj[w] / m.rho_w0;
            q[2] = q[0] * f;
            for (int v = 0; v < 4; ++v) dq[8 + v] = dq[v] * f;
        } else {
            q[0] = wi * lw * p.rw * draw;
            dq[0] = wi * lw * (p.drw * draw - p.rw);
            dq[1] = wi * dlw_S * p.rw * draw;
            dq[2] = wi * dlw_C * p.rw * draw;
            dq[3] = wi * lw * p.rw;
            q[1] = wi * lo * p.ro * draw;
            dq[4] = wi * lo * (p.dro * draw - p.ro);
            dq[5] = wi * dlo_S * p.ro * draw;
            dq[6] = 0.0;   // no C in the oil rate (skipped by the product kernels)
            dq[7] = wi * lo * p.ro;
            const double f = C / m.rho_w0;
            q[2] = q[0] * f;
            dq[8] = dq[0] * f;
            dq[9] = dq[1] * f;
            dq[10] = dq[2] * f + q[0] / m.rho_w0;
            dq[11] = dq[3] * f;
        }
        perf_q[2 * k] = q[0] / m.rho_w0;        // surface rates (switching at BHP limits)
        perf_q[2 * k + 1] = q[1] / m.rho_o0;
        const double scs[3] = {sc0, sc1, sc2};
        for (int e = 0; e < 3; ++e) {
            dr[e] -= dt * q[e];
            for (int v = 0; v < 3; ++v) dj[e * 3 + v] -= dt * dq[e * 4 + v];
            B[3 * k + e] = -dt * dq[e * 4 + 3] * scs[e];
        }
        // contribution to the well equation: the controlled surface stream
        const int ctrl = w_ctrl[w];
        const double ws = w_scale[w];
        double val = 0.0, dv[4] = {0.0, 0.0, 0.0, 0.0};
        if (ctrl == PF_CTRL_WRATE || ctrl == PF_CTRL_LRATE) {
            val += q[0] / m.rho_w0;
            for (int v = 0; v < 4; ++v) dv[v] += dq[v] / m.rho_w0;
        }
        if (ctrl == PF_CTRL_ORATE || ctrl == PF_CTRL_LRATE) {
            val += q[1] / m.rho_o0;
            for (int v = 0; v < 4; ++v) dv[v] += dq[4 + v] / m.rho_o0;
        }
        wv[k] = val * ws;
        for (int v = 0; v < 3; ++v) Cw[3 * k + v] = dv[v] * ws;
        wdp[k] = dv[3] * ws;
    }
    R[i] += dr[0] * sc0;
    R[n + i] += dr[1] * sc1;
    R[2 * n + i] += dr[2] * sc2;
    if (with_jac) {
        const double scs[3] = {sc0, sc1, sc2};
        // the diagonal block: natural-order planes, or its colour-split copy (Jdcs)
        int64_t base = i, step = n;
        double* Jw = J;
        if (Jdcs) {
            const int64_t iz = i / m.nxy, rem = i - iz * m.nxy, iy = rem / m.nx, ix = rem - iy * m.nx;
            step = cs_ns(m);
            base = ((ix + iy + iz) & 1) * 9 * step + (iy + m.ny * iz) * ((m.nx + 1) >> 1) + (ix >> 1);
            Jw = Jdcs;
        }
        for (int e = 0; e < 9; ++e)
            if (e != 5) Jw[base + e * step] += dj[e] * scs[e / 3];     // (oil, C) stays zero
    }
}
__global__ void k_wells(DevModel m, const double* __restrict__ x, const double* __restrict__ pvr,
                        const int32_t* __restrict__ pc_cell, const int32_t* __restrict__ pc_first,
                        const int32_t* __restrict__ perf_well, const double* __restrict__ perf_wi,
                        const double* __restrict__ perf_depth, const int32_t* __restrict__ w_inj,
                        const int32_t* __restrict__ w_ctrl, const double* __restrict__ w_cinj,
                        const double* __restrict__ w_gamma, const double* __restrict__ w_zref,
                        const double* __restrict__ w_scale, double dt, double* __restrict__ R, double* __restrict__ J,
                        double* __restrict__ B, double* __restrict__ Cw, double* __restrict__ wv,
                        double* __restrict__ wdp, double* __restrict__ perf_q, int with_jac,
                        double* __restrict__ Jdcs) {
    k_wells_d(PF_BLK, m, x, pvr, pc_cell, pc_first, perf_well, perf_wi, perf_depth, w_inj, w_ctrl, w_cinj, w_gamma,
              w_zref, w_scale, dt, R, J, B, Cw, wv, wdp, perf_q, with_jac, Jdcs);
}
struct F_k_wells {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_wells_d(wg, a...);
    }
};

// Well equations (Sec. 2.4 constraints), one thread per well; sums the
// per-perforation terms in a fixed order.
__device__ __forceinline__ void k_well_rows_d(const Blk& wg, DevModel m, const double* __restrict__ x,
                                              const int32_t* __restrict__ w_ctrl, const double* __restrict__ w_target,
                                              const double* __restrict__ w_scale,
                                              const int32_t* __restrict__ wp_first,
                                              const int32_t* __restrict__ wp_idx, const double* __restrict__ wv,
                                              const double* __restrict__ wdp, double* __restrict__ R,
                                              double* __restrict__ Dw) {
    const int w = wg.x * blockDim.x + threadIdx.x;
    if (w >= m.nw) return;
    const int64_t row = 3 * m.n + w;
    const double ws = w_scale[w];
    if (w_ctrl[w] == PF_CTRL_BHP) {
        R[row] = (x[row] - w_target[w]) * ws;
        Dw[w] = ws;
        return;
    }
    double val = 0.0, d = 0.0;
    for (int k = wp_first[w]; k < wp_first[w + 1]; ++k) {
        const int p = wp_idx[k];
        val += wv[p];
        d += wdp[p];
    }
    R[row] = val - w_target[w] * ws;
    Dw[w] = d;
}
__global__ void k_well_rows(DevModel m, const double* __restrict__ x, const int32_t* __restrict__ w_ctrl,
                            const double* __restrict__ w_target, const double* __restrict__ w_scale,
                            const int32_t* __restrict__ wp_first, const int32_t* __restrict__ wp_idx,
                            const double* __restrict__ wv, const double* __restrict__ wdp, double* __restrict__ R,
                            double* __restrict__ Dw) {
    k_well_rows_d(PF_BLK, m, x, w_ctrl, w_target, w_scale, wp_first, wp_idx, wv, wdp, R, Dw);
}
struct F_k_well_rows {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_well_rows_d(wg, a...);
    }
};

// ---------------------------------------------------------------------------
// Deterministic reductions: a fixed grid of kRedBlocks blocks, fixed
// grid-stride assignment, wavefront shuffles, then one finishing block that
// folds the partials in index order.
__device__ __forceinline__ double safe_abs(double v) {
    const double a = fabs(v);
    return (a <= DBL_MAX) ? a : INFINITY;   // NaN -> +inf
}

template <int K>
__device__ __forceinline__ void block_reduce(double (&v)[K], const bool (&is_max)[K], double* lds) {
    // wavefront (64 lanes) reduction
    for (int k = 0; k < K; ++k) {
        double a = v[k];
        for (int o = 32; o > 0; o >>= 1) {
            const double b = __shfl_down(a, o, 64);
            a = is_max[k] ? fmax(a, b) : a + b;
        }
        v[k] = a;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nwarp = blockDim.x >> 6;
    if (lane == 0)
        for (int k = 0; k < K; ++k) lds[k * 16 + wid] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < K; ++k) {
            double a = lds[k * 16];
            for (int q = 1; q < nwarp; ++q) a = is_max[k] ? fmax(a, lds[k * 16 + q]) : a + lds[k * 16 + q];
            v[k] = a;
        }
    }
    __syncthreads();
}

// partials of: max|v_w|, max|v_o|, max|v_p|, sum v^2 over the cell planes
__device__ __forceinline__ void k_norm_part_d(const Blk& wg, int64_t n, const double* __restrict__ v,
                                              double* __restrict__ part) {
    __shared__ double lds[4 * 16];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const bool mx[4] = {true, true, true, false};
    for (int64_t i = (int64_t)wg.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)wg.n * blockDim.x) {
        const double a = v[i], b = v[n + i], c = v[2 * n + i];
        acc[0] = fmax(acc[0], safe_abs(a));
        acc[1] = fmax(acc[1], safe_abs(b));
        acc[2] = fmax(acc[2], safe_abs(c));
        acc[3] += a * a + b * b + c * c;
    }
    block_reduce<4>(acc, mx, lds);
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; ++k) part[k * wg.n + wg.x] = acc[k];
}
__global__ __launch_bounds__(256) void k_norm_part(int64_t n, const double* __restrict__ v,
                                                   double* __restrict__ part) {
    k_norm_part_d(PF_BLK, n, v, part);
}
struct F_k_norm_part {
    static constexpr int kLB = 256;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_norm_part_d(wg, a...);
    }
};

// out: [0..2] max per equation, [3] max well row, [4] overall max, [5] 2-norm
__device__ __forceinline__ void k_norm_finish_d(const Blk& wg, int64_t n, int nw, int nblk,
                                                const double* __restrict__ v, const double* __restrict__ part,
                                                double* __restrict__ out) {
    __shared__ double lds[4 * 16];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const bool mx[4] = {true, true, true, false};
    for (int b = threadIdx.x; b < nblk; b += blockDim.x)
        for (int k = 0; k < 4; ++k)
            acc[k] = mx[k] ? fmax(acc[k], part[k * nblk + b]) : acc[k] + part[k * nblk + b];
    block_reduce<4>(acc, mx, lds);
    if (threadIdx.x == 0) {
        double wm = 0.0, ws = 0.0;
        for (int w = 0; w < nw; ++w) {
            const double a = v[3 * n + w];
            wm = fmax(wm, safe_abs(a));
            ws += a * a;
        }
        const double ss = acc[3] + ws;
        out[0] = acc[0];
        out[1] = acc[1];
        out[2] = acc[2];
        out[3] = wm;
        out[4] = fmax(fmax(acc[0], acc[1]), fmax(acc[2], wm));
        out[5] = (ss <= DBL_MAX) ? sqrt(ss) : INFINITY;
    }
}
__global__ __launch_bounds__(256) void k_norm_finish(int64_t n, int nw, int nblk, const double* __restrict__ v,
                                                     const double* __restrict__ part, double* __restrict__ out) {
    k_norm_finish_d(PF_BLK, n, nw, nblk, v, part, out);
}
struct F_k_norm_finish {
    static constexpr int kLB = 256;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_norm_finish_d(wg, a...);
    }
};

// Chopped Newton update of the cells (|dS| <= ds_max, C >= 0) with partial
// maxima of the applied change in scaled units.
// dx in the natural (cs 0) or the solver's colour-split layout (cs 1: planes
// of 2 cs_ns slots, the wells after the three planes)
__device__ __forceinline__ void k_update_part_d(const Blk& wg, DevModel m, double ds_max,
                                                const double* __restrict__ dx, double* __restrict__ x,
                                                double* __restrict__ part, int cs) {
    __shared__ double lds[3 * 16];
    double acc[3] = {0.0, 0.0, 0.0};
    const bool mx[3] = {true, true, true};
    const int64_t n = m.n, lp = cs ? 2 * cs_ns(m) : n;
    for (int64_t i = (int64_t)wg.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)wg.n * blockDim.x) {
        const int64_t j = cs ? cs_index(m, i) : i;
        const double dP = dx[j];
        const double dS = fmin(fmax(dx[lp + j], -ds_max), ds_max);
        const double C0 = x[2 * n + i];
        const double C1 = fmax(C0 + dx[2 * lp + j], 0.0);
        x[i] += dP;
        x[n + i] += dS;
        x[2 * n + i] = C1;
        acc[0] = fmax(acc[0], safe_abs(dP) / kBar);
        acc[1] = fmax(acc[1], safe_abs(dS));
        acc[2] = fmax(acc[2], safe_abs(C1 - C0) / m.c_ref);
    }
    block_reduce<3>(acc, mx, lds);
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) part[k * wg.n + wg.x] = acc[k];
}
__global__ __launch_bounds__(256) void k_update_part(DevModel m, double ds_max, const double* __restrict__ dx,
                                                     double* __restrict__ x, double* __restrict__ part, int cs) {
    k_update_part_d(PF_BLK, m, ds_max, dx, x, part, cs);
}
struct F_k_update_part {
    static constexpr int kLB = 256;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_update_part_d(wg, a...);
    }
};

// out: [0] dP/bar, [1] dS, [2] dC/Cref, [3] dPb/bar, [4] max of all
__device__ __forceinline__ void k_update_finish_d(const Blk& wg, DevModel m, int nblk, const double* __restrict__ dx,
                                                  double* __restrict__ x, const double* __restrict__ part,
                                                  double* __restrict__ out, int cs) {
    __shared__ double lds[3 * 16];
    double acc[3] = {0.0, 0.0, 0.0};
    const bool mx[3] = {true, true, true};
    for (int b = threadIdx.x; b < nblk; b += blockDim.x)
        for (int k = 0; k < 3; ++k) acc[k] = fmax(acc[k], part[k * nblk + b]);
    block_reduce<3>(acc, mx, lds);
    if (threadIdx.x == 0) {
        double wm = 0.0;
        for (int w = 0; w < m.nw; ++w) {
            const double d = dx[3 * (cs ? 2 * cs_ns(m) : m.n) + w];
            x[3 * m.n + w] += d;
            wm = fmax(wm, safe_abs(d) / kBar);
        }
        out[0] = acc[0];
        out[1] = acc[1];
        out[2] = acc[2];
        out[3] = wm;
        out[4] = fmax(fmax(acc[0], acc[1]), fmax(acc[2], wm));
    }
}
__global__ __launch_bounds__(256) void k_update_finish(DevModel m, int nblk, const double* __restrict__ dx,
                                                       double* __restrict__ x, const double* __restrict__ part,
                                                       double* __restrict__ out, int cs) {
    k_update_finish_d(PF_BLK, m, nblk, dx, x, part, out, cs);
}
struct F_k_update_finish {
    static constexpr int kLB = 256;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_update_finish_d(wg, a...);
    }
};

}  // namespace

// ---------------------------------------------------------------------------
void launch_static(Sim& s) {
    const DevModel& m = s.m;
    launch<F_k_static_cells>(s, s.stream, k_static_cells, dim3(grid_for(m.n)), dim3(kBlock), 0, m, s.poro, s.kx, s.ky,
                             s.kz, s.pvr, s.Tx, s.Ty, s.Tz, s.rscale);
    PF_LAUNCH_CHECK();
    if (m.np > 0) {
        launch<F_k_static_perfs>(s, s.stream, k_static_perfs, dim3(grid_for(m.np)), dim3(kBlock), 0, m, s.perf_cell,
                                 s.perf_well, s.w_dir, s.w_rw, s.w_skin, s.kx, s.ky, s.kz, s.perf_wi);
        PF_LAUNCH_CHECK();
    }
}

void launch_accum(Sim& s, const double* x, double* M) {
    launch<F_k_accum>(s, s.stream, k_accum, dim3(grid_for(s.m.n)), dim3(kBlock), 0, s.m, x, s.pvr, M);
    PF_LAUNCH_CHECK();
}

// Per-cell RRF and A_d,max from the rock table (Sec. 2.3: functions of the
// rock permeability), interpolated in log10 kx: the cell's capacity
// A_d,max / ads_max and (RRF - 1) / A_d,max.
__device__ __forceinline__ void k_kperm_d(const Blk& wg, DevModel m, const double* __restrict__ kx,
                                          double* __restrict__ cap, double* __restrict__ rks) {
    const int64_t i = (int64_t)wg.x * blockDim.x + threadIdx.x;
    if (i >= m.n) return;
    const double lk = log10(kx[i]);
    double rrf, admax, d;
    table_eval(m.tab + kTabKpK * PF_TABLE_MAX, m.tab + kTabKpRrf * PF_TABLE_MAX, m.n_kperm, lk, rrf, d);
    table_eval(m.tab + kTabKpK * PF_TABLE_MAX, m.tab + kTabKpAdm * PF_TABLE_MAX, m.n_kperm, lk, admax, d);
    cap[i] = admax / m.ads_max;
    rks[i] = (rrf - 1.0) / admax;
}
__global__ void k_kperm(DevModel m, const double* __restrict__ kx, double* __restrict__ cap,
                        double* __restrict__ rks) {
    k_kperm_d(PF_BLK, m, kx, cap, rks);
}
struct F_k_kperm {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_kperm_d(wg, a...);
    }
};

// Retention: the largest past equilibrium adsorption of every cell takes in
// the state x (a converged state: the start of a timestep).
__device__ __forceinline__ void k_ads_hist_d(const Blk& wg, DevModel m, const double* __restrict__ x,
                                             double* __restrict__ hist) {
    const int64_t i = (int64_t)wg.x * blockDim.x + threadIdx.x;
    if (i >= m.n) return;
    double a, da;
    isotherm<true>(m, i, x[2 * m.n + i], a, da);
    hist[i] = fmax(hist[i], a);
}
__global__ void k_ads_hist(DevModel m, const double* __restrict__ x, double* __restrict__ hist) {
    k_ads_hist_d(PF_BLK, m, x, hist);
}
struct F_k_ads_hist {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_ads_hist_d(wg, a...);
    }
};

// Capillary-gravity equilibrium (Sec. 4.1.3), one thread per layer: the
// oil pressure marched from the datum to the layer centre, the water
// pressure marched (with the oil pressure alongside, for the water density
// at the cell pressure unknown) from the free-water level, then the
// saturation from the capillary-pressure table and the cell pressure.
// Classical fourth-order Runge-Kutta in equal steps of at most 0.25 m.
constexpr double kMarchStep = 0.25;

__device__ double march_oil(const DevModel& m, double p, double z0, double z1) {
    const double dz = z1 - z0;
    const int nstep = max(1, (int)ceil(fabs(dz) / kMarchStep));
    const double h = dz / nstep;
    for (int k = 0; k < nstep; ++k) {
        const double k1 = m.rho_o0 * exp(m.c_o * (p - m.pref)) * m.grav;
        const double k2 = m.rho_o0 * exp(m.c_o * (p + 0.5 * h * k1 - m.pref)) * m.grav;
        const double k3 = m.rho_o0 * exp(m.c_o * (p + 0.5 * h * k2 - m.pref)) * m.grav;
        const double k4 = m.rho_o0 * exp(m.c_o * (p + h * k3 - m.pref)) * m.grav;
        p = p + h / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4);
    }
    return p;
}

__device__ void water_rhs(const DevModel& m, double pc_last, double po, double pw, double& fo, double& fw) {
    const double pcell = (po - pw > pc_last) ? po : pw + pc_last;
    fo = m.rho_o0 * exp(m.c_o * (po - m.pref)) * m.grav;
    fw = m.rho_w0 * exp(m.c_w * (pcell - m.pref)) * m.grav;
}

__device__ double march_water(const DevModel& m, double pc_last, double p_fwl, double z0, double z1) {
    const double dz = z1 - z0;
    const int nstep = max(1, (int)ceil(fabs(dz) / kMarchStep));
    const double h = dz / nstep;
    double po = p_fwl, pw = p_fwl;
    for (int k = 0; k < nstep; ++k) {
        double a1, b1, a2, b2, a3, b3, a4, b4;
        water_rhs(m, pc_last, po, pw, a1, b1);
        water_rhs(m, pc_last, po + 0.5 * h * a1, pw + 0.5 * h * b1, a2, b2);
        water_rhs(m, pc_last, po + 0.5 * h * a2, pw + 0.5 * h * b2, a3, b3);
        water_rhs(m, pc_last, po + h * a3, pw + h * b3, a4, b4);
        po = po + h / 6.0 * (a1 + 2.0 * a2 + 2.0 * a3 + a4);
        pw = pw + h / 6.0 * (b1 + 2.0 * b2 + 2.0 * b3 + b4);
    }
    return pw;
}

__device__ __forceinline__ void k_equilibrium_layers_d(const Blk& wg, DevModel m, double datum_depth, double datum_p,
                                                       double fwl_depth, double* __restrict__ layer_p,
                                                       double* __restrict__ layer_s) {
    const int k = wg.x * blockDim.x + threadIdx.x;
    if (k >= m.nz) return;
    const double* pcs = m.tab + kTabPcS * PF_TABLE_MAX;
    const double* pcv = m.tab + kTabPcV * PF_TABLE_MAX;
    const int npc = m.n_pc;
    const double pc_last = npc > 0 ? pcv[npc - 1] : 0.0;
    const double z = m.top + (k + 0.5) * m.dz;
    const double p_fwl = march_oil(m, datum_p, datum_depth, fwl_depth);
    const double po = march_oil(m, datum_p, datum_depth, z);
    const double pw = march_water(m, pc_last, p_fwl, fwl_depth, z);
    const double delta = po - pw;
    double S;
    if (npc == 0) {
        S = delta > 0.0 ? m.swc : 1.0 - m.sor;
    } else if (delta >= pcv[0]) {
        S = pcs[0];
    } else if (delta <= pcv[npc - 1]) {
        S = pcs[npc - 1];
    } else {
        int q = 0;
        while (!(pcv[q] >= delta && delta > pcv[q + 1])) ++q;
        S = pcs[q] + (delta - pcv[q]) * (pcs[q + 1] - pcs[q]) / (pcv[q + 1] - pcv[q]);
    }
    layer_p[k] = delta > pc_last ? po : pw + pc_last;
    layer_s[k] = S;
}
__global__ void k_equilibrium_layers(DevModel m, double datum_depth, double datum_p, double fwl_depth,
                                     double* __restrict__ layer_p, double* __restrict__ layer_s) {
    k_equilibrium_layers_d(PF_BLK, m, datum_depth, datum_p, fwl_depth, layer_p, layer_s);
}
struct F_k_equilibrium_layers {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_equilibrium_layers_d(wg, a...);
    }
};

// The layer values to every cell (C = 0) and the wells' starting bottom-hole
// pressures (BHP target, or the pressure of the datum layer).
__device__ __forceinline__ void k_equilibrium_fill_d(const Blk& wg, DevModel m, const double* __restrict__ layer_p,
                                                     const double* __restrict__ layer_s,
                                                     const int32_t* __restrict__ w_ctrl0,
                                                     const double* __restrict__ w_target0,
                                                     const int32_t* __restrict__ w_ktop, double* __restrict__ x) {
    const int64_t i = (int64_t)wg.x * blockDim.x + threadIdx.x;
    if (i < m.n) {
        const int64_t iz = i / m.nxy;
        x[i] = layer_p[iz];
        x[m.n + i] = layer_s[iz];
        x[2 * m.n + i] = 0.0;
    } else if (i < m.n + m.nw) {
        const int w = (int)(i - m.n);
        x[3 * m.n + w] = w_ctrl0[w] == PF_CTRL_BHP ? w_target0[w] : layer_p[w_ktop[w]];
    }
}
__global__ void k_equilibrium_fill(DevModel m, const double* __restrict__ layer_p, const double* __restrict__ layer_s,
                                   const int32_t* __restrict__ w_ctrl0, const double* __restrict__ w_target0,
                                   const int32_t* __restrict__ w_ktop, double* __restrict__ x) {
    k_equilibrium_fill_d(PF_BLK, m, layer_p, layer_s, w_ctrl0, w_target0, w_ktop, x);
}
struct F_k_equilibrium_fill {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_equilibrium_fill_d(wg, a...);
    }
};

void launch_kperm(Sim& s) {
    launch<F_k_kperm>(s, s.stream, k_kperm, dim3(grid_for(s.m.n)), dim3(kBlock), 0, s.m, s.kx, s.cell_cap, s.cell_rks);
    PF_LAUNCH_CHECK();
}

void launch_ads_hist(Sim& s) {
    launch<F_k_ads_hist>(s, s.stream, k_ads_hist, dim3(grid_for(s.m.n)), dim3(kBlock), 0, s.m, s.x, s.ads_hist);
    PF_LAUNCH_CHECK();
}

void launch_equilibrium(Sim& s, double datum_depth, double datum_p, double fwl_depth) {
    // layer values in the first Krylov work vector (3N + nw >= 2 nz doubles); the
    // wells' primary controls and datum layers in the second
    double* lp = s.t1;
    double* ls = s.t1 + s.m.nz;
    int32_t* wc = reinterpret_cast<int32_t*>(s.t2);
    int32_t* wk = wc + std::max<int32_t>(s.m.nw, 1);
    double* wt = s.t2 + std::max<int32_t>(s.m.nw, 1);
    const int nw = s.m.nw;
    if (2 * std::max<int64_t>(nw, 1) > s.nv) throw HipError{"more wells than the work vector holds"};
    std::vector<int32_t> ctrl(s.h_ctrl0), ktop(nw);
    for (int w = 0; w < nw; ++w) ktop[w] = s.h_wktop[w];
    if (nw > 0) {
        PF_HIP(hipMemcpyAsync(wc, ctrl.data(), nw * 4, hipMemcpyHostToDevice, s.stream));
        PF_HIP(hipMemcpyAsync(wk, ktop.data(), nw * 4, hipMemcpyHostToDevice, s.stream));
        PF_HIP(hipMemcpyAsync(wt, s.h_target0.data(), nw * 8, hipMemcpyHostToDevice, s.stream));
    }
    launch<F_k_equilibrium_layers>(s, s.stream, k_equilibrium_layers, dim3(grid_for(s.m.nz, 64)), dim3(64), 0, s.m,
                                   datum_depth, datum_p, fwl_depth, lp, ls);
    PF_LAUNCH_CHECK();
    launch<F_k_equilibrium_fill>(s, s.stream, k_equilibrium_fill, dim3(grid_for(s.m.n + s.m.nw)), dim3(kBlock), 0,
                                 s.m, lp, ls, wc, wt, wk, s.x);
    PF_LAUNCH_CHECK();
    PF_HIP(hipStreamSynchronize(s.stream));     // the host vectors above outlive their copies
}

void launch_assemble(Sim& s, double dt, bool with_jacobian) {
    const DevModel& m = s.m;
    // FP64 red-black ILU(0) in PF order: J in the colour-split layout only (the
    // smoother set-up, the stage residual, the ILU phases and the product read
    // that layout; natural-order J is formed from it when something needs it)
    const bool cs = with_jacobian && j_colour_split_mode(s);
    double* lcs = cs ? s.Lc : nullptr;
    double* jdcs = cs ? s.Jdc : nullptr;
    if (with_jacobian) {
        s.j_cs = cs;
        s.j_nat = !cs;
    }
    {
        ProfScope ps(s, PF_K_ASSEMBLE);
        const bool var = m.mix_rule != PF_MIX_POLY || m.n_ads > 0 || m.n_pc > 0 || m.cell_cap || m.ads_hist;
        // colour-major threads in the colour-split mode: both colours' slots, in pairs of wavefronts
        const dim3 grid(grid_for(cs ? 2 * cs_ns(m) : m.n));
        if (var)
            launch<F_k_assemble<true>>(s, s.stream, k_assemble<true>, grid, dim3(kBlock), 0, m, s.x, s.Mn, s.pvr, s.Tx,
                                       s.Ty, s.Tz, dt, s.R, s.J, (int)with_jacobian, lcs, jdcs);
        else
            launch<F_k_assemble<false>>(s, s.stream, k_assemble<false>, grid, dim3(kBlock), 0, m, s.x, s.Mn, s.pvr,
                                        s.Tx, s.Ty, s.Tz, dt, s.R, s.J, (int)with_jacobian, lcs, jdcs);
        PF_LAUNCH_CHECK();
    }
    if (m.npc > 0) {
        launch<F_k_wells>(s, s.stream, k_wells, dim3(grid_for(m.npc, 64)), dim3(64), 0, m, s.x, s.pvr, s.pc_cell,
                          s.pc_first, s.perf_well, s.perf_wi, s.perf_depth, s.w_inj, s.w_ctrl, s.w_cinj, s.w_gamma,
                          s.w_zref, s.w_scale, dt, s.R, s.J, s.B, s.Cw, s.wv, s.wdp, s.perf_q, (int)with_jacobian,
                          jdcs);
        PF_LAUNCH_CHECK();
    }
    if (m.nw > 0) {
        launch<F_k_well_rows>(s, s.stream, k_well_rows, dim3(grid_for(m.nw, 64)), dim3(64), 0, m, s.x, s.w_ctrl,
                              s.w_target, s.w_scale, s.wp_first, s.wp_idx, s.wv, s.wdp, s.R, s.Dw);
        PF_LAUNCH_CHECK();
    }
}

void launch_norms(Sim& s, const double* v, double* out) {
    const int G = kRedBlocks;
    launch<F_k_norm_part>(s, s.stream, k_norm_part, dim3(G), dim3(kBlock), 0, s.m.n, v, s.part);
    PF_LAUNCH_CHECK();
    launch<F_k_norm_finish>(s, s.stream, k_norm_finish, dim3(1), dim3(kBlock), 0, s.m.n, s.m.nw, G, v, s.part, out);
    PF_LAUNCH_CHECK();
}

void launch_update(Sim& s, const double* dx, double* out, bool cs) {
    const int G = kRedBlocks;
    launch<F_k_update_part>(s, s.stream, k_update_part, dim3(G), dim3(kBlock), 0, s.m, s.opts.ds_max, dx, s.x, s.part,
                            (int)cs);
    PF_LAUNCH_CHECK();
    launch<F_k_update_finish>(s, s.stream, k_update_finish, dim3(1), dim3(kBlock), 0, s.m, G, dx, s.x, s.part, out,
                              (int)cs);
    PF_LAUNCH_CHECK();
}

}  // namespace pf
