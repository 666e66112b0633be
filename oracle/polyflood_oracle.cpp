/*
 * Plain FP64 CPU oracle for the fully implicit water / oil / polymer model of
 * Zhong et al., "Numerical simulations of polymer flooding process in porous
 * media on distributed-memory parallel computers" (arXiv 1807.05298).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may load this
 * library; only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, table or constant with
 * the HIP library: every formula below is written again from the paper.
 *
 * What it computes (all SI units):
 *   - static quantities: harmonic face transmissibilities and pore-volume
 *     weights (Sec. 3.2 "Spatial discretization", interface averaging),
 *     Peaceman well indices for vertical wells (Sec. 2.4, eq:wi, eq:wi:re:k
 *     with the x/y/z roles permuted for a z-direction well);
 *   - the backward-Euler residual of water, oil and polymer mass balance
 *     (Sec. 3.1 time discretization; Sec. 2 conservation laws) with upstream
 *     relative permeability chosen by phase potential (Sec. 3.2, ties go to
 *     the higher-index cell) plus the well equations (Sec. 2.4, fixed BHP,
 *     water / oil / liquid rate);
 *   - its Jacobian by forward-mode automatic differentiation of that same
 *     residual (a dual number type below), so no derivative is derived by
 *     hand here.
 *
 * Readings where the paper is silent (each one listed in the design notes):
 * polymer concentration C is in kg/m^3 and enters the polymer mass as the
 * mass fraction C/rho_w0; inaccessible pore volume scales the accessible
 * pore space of the polymer accumulation by (1 - IPV); adsorption is a
 * Langmuir isotherm A = Amax*b*C/(1+b*C) in kg per m^3 of rock with
 * A_d,max = Amax; density rho = rho0*exp(c*(P - Pref)); viscosities do not
 * depend on pressure; capillary pressure is zero; the face value of R_k and
 * of C in the polymer flux is taken upstream with the water relative
 * permeability; the wellbore unit weight is rho0*g of the injected (water)
 * or produced (oil) phase and the datum is the top perforation.
 *
 * Vector layout ("block-wise", Sec. 3.4 linear solver): unknown 3*i+0 is the
 * oil pressure of cell i, 3*i+1 its water saturation, 3*i+2 its polymer
 * concentration; unknown 3*N+w is the bottom-hole pressure of well w.
 * Equations follow the same order: water, oil, polymer mass, then one well
 * equation per well.  Cells are in natural order i = ix + nx*(iy + ny*iz).
 */
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>
#include <algorithm>

namespace {

/* ---------------- forward-mode dual number --------------------------------
 * Slots 0-2: (P, S, C) of the first cell in play; 3-5: of the second cell
 * (the other side of a face); 6: bottom-hole pressure of the well. */
constexpr int ND = 7;

struct Dual {
    double v;
    double d[ND];
    Dual() : v(0.0) { for (int k = 0; k < ND; ++k) d[k] = 0.0; }
    Dual(double x) : v(x) { for (int k = 0; k < ND; ++k) d[k] = 0.0; }
    static Dual var(double x, int slot) { Dual r(x); r.d[slot] = 1.0; return r; }
};

inline Dual operator+(const Dual& a, const Dual& b) { Dual r(a.v + b.v); for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
inline Dual operator-(const Dual& a, const Dual& b) { Dual r(a.v - b.v); for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
inline Dual operator-(const Dual& a) { Dual r(-a.v); for (int k = 0; k < ND; ++k) r.d[k] = -a.d[k]; return r; }
inline Dual operator*(const Dual& a, const Dual& b) { Dual r(a.v * b.v); for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r; }
inline Dual operator/(const Dual& a, const Dual& b) {
    Dual r(a.v / b.v);
    for (int k = 0; k < ND; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v);
    return r;
}
inline Dual operator+(const Dual& a, double b) { return a + Dual(b); }
inline Dual operator+(double a, const Dual& b) { return Dual(a) + b; }
inline Dual operator-(const Dual& a, double b) { return a - Dual(b); }
inline Dual operator-(double a, const Dual& b) { return Dual(a) - b; }
inline Dual operator*(const Dual& a, double b) { return a * Dual(b); }
inline Dual operator*(double a, const Dual& b) { return Dual(a) * b; }
inline Dual operator/(const Dual& a, double b) { return a / Dual(b); }
inline Dual operator/(double a, const Dual& b) { return Dual(a) / b; }
inline Dual dexp(const Dual& a) { double e = std::exp(a.v); Dual r(e); for (int k = 0; k < ND; ++k) r.d[k] = e * a.d[k]; return r; }
/* a^p for a constant exponent p; the derivative p*a^(p-1) is taken as 0 when a == 0 and p >= 1 */
inline Dual dpow(const Dual& a, double p) {
    Dual r(std::pow(a.v, p));
    double dp = (a.v == 0.0) ? (p == 1.0 ? 1.0 : 0.0) : p * std::pow(a.v, p - 1.0);
    for (int k = 0; k < ND; ++k) r.d[k] = dp * a.d[k];
    return r;
}

/* Move the derivative of slots 0-2 into slots 3-5 (the same cell seen as the
 * second member of a face). */
inline Dual to_second(const Dual& a) {
    Dual r(a.v);
    for (int k = 0; k < 3; ++k) { r.d[3 + k] = a.d[k]; }
    r.d[6] = a.d[6];
    return r;
}

}  // namespace

extern "C" {

/* Model description handed in from Python (ctypes mirror in oracle/__init__.py). */
typedef struct {
    int32_t nx, ny, nz, nwell;
    double dx, dy, dz, top;
    const double *poro, *kx, *ky, *kz;
    double cr, pref;
    double rho_w0, rho_o0, c_w, c_o, mu_w, mu_o, swc, sor, n_w, n_o, krw0, kro0, grav;
    double a1, a2, omega, cmax, ads_max, ads_b, rrf, ipv;
    const int32_t *w_ix, *w_iy, *w_k0, *w_k1, *w_inj, *w_ctrl;
    const double *w_target, *w_cinj, *w_rw, *w_skin;
    const int32_t *w_dir, *w_ix1;            /* 0 vertical, 1 along x (cells w_ix..w_ix1) */
    /* property variants: mixing rule (0 polynomial, 1 linear, 2 nonlinear,
       3 viscosity-multiplier table), mu_p^ref (0: the polynomial at cmax),
       tables of n points: adsorption (C, A), viscosity multiplier (C, m),
       capillary pressure (S, Pc) */
    int32_t mix_rule, n_ads, n_visc, n_pc;
    double mu_p_ref;
    const double *ads_c, *ads_a, *visc_c, *visc_m, *pc_s, *pc_v;
    /* retention beyond equilibrium sorption (Sec. 2.3): ads_res is the part of
       a cell's largest past adsorption that cannot desorb (0: equilibrium);
       RRF and A_d,max as functions of rock permeability: a table of n_kperm
       points (permeability in m^2, RRF, A_d,max in kg per m^3 rock),
       interpolated linearly in log10 of the cell's kx */
    double ads_res;
    int32_t n_kperm, pad_k;
    const double *kperm_k, *kperm_rrf, *kperm_admax;
} OraModel;

}  // extern "C"

namespace {

struct Perf { int well; int cell; double wi; double depth; };

struct Oracle {
    OraModel m;
    int64_t n;
    std::vector<double> poro, kx, ky, kz;
    std::vector<double> pvr;                 /* reference pore volume phi_r*V */
    std::vector<int32_t> w_ix, w_iy, w_k0, w_k1, w_inj, w_ctrl, w_dir, w_ix1;
    std::vector<double> ads_c, ads_a, visc_c, visc_m, pc_s, pc_v;
    std::vector<double> w_target, w_cinj, w_rw, w_skin, w_zref, w_gamma;
    std::vector<double> cap;                 /* A_d,max of the cell / ads_max (1 without the table) */
    std::vector<double> rrf;                 /* RRF of the cell */
    std::vector<double> hist;                /* largest past adsorption of the cell (kg/m^3 rock) */
    std::vector<Perf> perfs;                 /* sorted by cell */
    std::vector<int64_t> perf_start;         /* n+1 offsets into perfs */
    std::vector<std::vector<int>> well_perfs;
    double vol;
};

inline int64_t cell_index(const Oracle& o, int ix, int iy, int iz) {
    return (int64_t)ix + (int64_t)o.m.nx * ((int64_t)iy + (int64_t)o.m.ny * iz);
}

inline double cell_depth(const Oracle& o, int iz) { return o.m.top + (iz + 0.5) * o.m.dz; }

/* Harmonic interface transmissibility (Sec. 3.2): area over the two
 * half-cell resistances, geometric part and permeability together. */
double face_trans(double area, double len, double kL, double kR) {
    return area / (0.5 * len / kL + 0.5 * len / kR);
}

/* Peaceman well index for a well along z (eq:wi with eq:wi:re:k, axes
 * permuted so that the block sizes / permeabilities perpendicular to the
 * well are those of x and y), f = f_h = 1, g_f = 0.249. */
double well_index_z(double dx, double dy, double h, double kx, double ky, double rw, double skin) {
    const double gf = 0.249;
    const double pi = 3.14159265358979323846;
    double ryx = std::sqrt(ky / kx), rxy = std::sqrt(kx / ky);
    double num = std::sqrt(ryx * dx * dx + rxy * dy * dy);
    double den = std::pow(ky / kx, 0.25) + std::pow(kx / ky, 0.25);
    double re = 2.0 * gf / std::sqrt(pi) * num / den;
    double ka = std::sqrt(kx * ky);
    return 2.0 * pi * h * ka / (std::log(re / rw) + skin);
}

/* eq:wi with f = f_h = 1 for a well parallel to x, and eq:wi:re:k as
   printed: r_e from ky, kz and the block sizes hy, hz across the well;
   k_a = sqrt(ky kz); h the block size along the well (dx). */
double well_index_x(double h, double hy, double hz, double ky, double kz, double rw, double skin) {
    const double gf = 0.249;
    const double pi = 3.14159265358979323846;
    double num = std::sqrt(std::sqrt(kz / ky) * hy * hy + std::sqrt(ky / kz) * hz * hz);
    double den = std::pow(kz / ky, 0.25) + std::pow(ky / kz, 0.25);
    double re = 2.0 * gf / std::sqrt(pi) * num / den;
    double ka = std::sqrt(ky * kz);
    return 2.0 * pi * h * ka / (std::log(re / rw) + skin);
}

/* ---------------- cell properties (Sec. 2.1-2.3) -------------------------- */
template <class T> struct Props {
    T phi, rho_w, rho_o, krw, kro, mu_we, mu_pe, ads, rk, pc;
};

/* A table given by points (x_k, y_k), x increasing: linear between
   neighbouring points, the end value beyond the first and last point. */
Dual table_lookup(const std::vector<double>& x, const std::vector<double>& y, const Dual& v) {
    size_t n = x.size();
    if (v.v < x[0]) return Dual(y[0]);
    if (v.v >= x[n - 1]) return Dual(y[n - 1]);
    size_t k = 0;
    while (k + 2 < n && v.v >= x[k + 1]) ++k;
    return y[k] + (y[k + 1] - y[k]) / (x[k + 1] - x[k]) * (v - x[k]);
}

template <class T>
Props<T> props(const Oracle& o, int64_t cell, const T& P, const T& S, const T& C) {
    const OraModel& m = o.m;
    const double phi_r = o.poro[cell];
    Props<T> p;
    p.phi = phi_r + m.cr * (P - m.pref);                       /* rock model */
    p.rho_w = m.rho_w0 * dexp(m.c_w * (P - m.pref));
    p.rho_o = m.rho_o0 * dexp(m.c_o * (P - m.pref));
    /* normalised saturation, clamped to [0, 1] */
    T sn;
    if (S.v < m.swc) sn = T(0.0);
    else if (S.v > 1.0 - m.sor) sn = T(1.0);
    else sn = (S - m.swc) / (1.0 - m.swc - m.sor);
    p.krw = m.krw0 * dpow(sn, m.n_w);
    p.kro = m.kro0 * dpow(1.0 - sn, m.n_o);
    /* Todd-Longstaff effective viscosities over the fully mixed viscosity
     * mu_m(C) = mu_w (1 + a1 C + a2 C^2); mu_p^ref = mu_m(C_max); the
     * effective saturation of injected solution alpha = C / C_max. */
    double mup_ref = m.mu_p_ref > 0.0 ? m.mu_p_ref : m.mu_w * (1.0 + m.a1 * m.cmax + m.a2 * m.cmax * m.cmax);
    T mum;
    if (m.mix_rule == 1) {                 /* linear mixing rule, beta = C / C_ref */
        T beta = C / m.cmax;
        mum = beta * mup_ref + (1.0 - beta) * m.mu_w;
    } else if (m.mix_rule == 2) {          /* nonlinear: mu_p^ref^beta mu_w^(1-beta) */
        T beta = C / m.cmax;
        mum = dexp(beta * std::log(mup_ref)) * dexp((1.0 - beta) * std::log(m.mu_w));
    } else if (m.mix_rule == 3) {          /* viscosity multiplier table */
        mum = m.mu_w * table_lookup(o.visc_c, o.visc_m, C);
    } else {                               /* the configs' polynomial */
        mum = m.mu_w * (1.0 + m.a1 * C + m.a2 * C * C);
    }
    if (m.omega == 1.0) {
        p.mu_pe = mum;
        p.mu_we = mum;
    } else {
        p.mu_pe = dpow(mum, m.omega) * std::pow(mup_ref, 1.0 - m.omega);
        T mu_wpart = dpow(mum, m.omega) * std::pow(m.mu_w, 1.0 - m.omega);
        T alpha = C / m.cmax;
        p.mu_we = 1.0 / (alpha / p.mu_pe + (1.0 - alpha) / mu_wpart);
    }
    /* equilibrium (Langmuir) adsorption scaled by the rock's capacity
       A_d,max / ads_max, retention of part of the largest past adsorption,
       and permeability reduction with the rock's RRF and A_d,max */
    T eq;
    if (m.n_ads > 0) eq = table_lookup(o.ads_c, o.ads_a, C);          /* tabulated isotherm */
    else eq = m.ads_max * m.ads_b * C / (1.0 + m.ads_b * C);
    eq = o.cap[cell] * eq;
    const double held = m.ads_res * o.hist[cell];
    p.ads = (held > eq.v) ? T(held) : eq;
    p.rk = 1.0 + (o.rrf[cell] - 1.0) * p.ads / (o.cap[cell] * m.ads_max);
    /* capillary pressure P_o - P_w */
    p.pc = m.n_pc > 0 ? table_lookup(o.pc_s, o.pc_v, S) : T(0.0);
    return p;
}

/* accumulation (mass per cell, kg): water, oil, polymer */
template <class T>
void accumulation(const Oracle& o, int64_t i, const T& P, const T& S, const T& C, T out[3]) {
    Props<T> p = props(o, i, P, S, C);
    const OraModel& m = o.m;
    out[0] = o.vol * p.phi * S * p.rho_w;
    out[1] = o.vol * p.phi * (1.0 - S) * p.rho_o;
    out[2] = o.vol * (p.phi * (1.0 - m.ipv) * S * (p.rho_w / m.rho_w0) * C + (1.0 - p.phi) * p.ads);
}

/* Mass flux (kg/s) across the face from cell L to cell R (L has the lower
 * natural index), positive from L to R.  xL in slots 0-2, xR in slots 3-5. */
void face_flux(const Oracle& o, int64_t L, int64_t R, double trans, double dz_depth,
               const Dual xL[3], const Dual xR[3], Dual F[3]) {
    const OraModel& m = o.m;
    Props<Dual> pL = props(o, L, xL[0], xL[1], xL[2]);
    Props<Dual> pR = props(o, R, xR[0], xR[1], xR[2]);
    double wL = o.pvr[L] / (o.pvr[L] + o.pvr[R]);
    double wR = 1.0 - wL;
    /* pore-volume weighted arithmetic averages of density and viscosity */
    Dual rw = wL * pL.rho_w + wR * pR.rho_w;
    Dual ro = wL * pL.rho_o + wR * pR.rho_o;
    Dual muw = wL * pL.mu_we + wR * pR.mu_we;
    Dual mup = wL * pL.mu_pe + wR * pR.mu_pe;
    /* phase potential difference R minus L, depth positive downward */
    Dual dphi_w = ((xR[0] - pR.pc) - (xL[0] - pL.pc)) - rw * m.grav * dz_depth;   /* water pressure P - Pc */
    Dual dphi_o = (xR[0] - xL[0]) - ro * m.grav * dz_depth;
    /* upstream: the cell with the higher potential; equal potentials -> R */
    bool up_w_R = dphi_w.v >= 0.0;
    bool up_o_R = dphi_o.v >= 0.0;
    const Props<Dual>& pw = up_w_R ? pR : pL;
    const Props<Dual>& po = up_o_R ? pR : pL;
    const Dual& Cup = up_w_R ? xR[2] : xL[2];
    Dual lam_w = pw.krw / (pw.rk * muw);
    Dual lam_p = pw.krw / (pw.rk * mup);
    Dual lam_o = po.kro / m.mu_o;
    F[0] = -trans * lam_w * rw * dphi_w;
    F[1] = -trans * lam_o * ro * dphi_o;
    F[2] = -trans * lam_p * rw * (Cup / m.rho_w0) * dphi_w;
}

/* Perforation rates (kg/s, positive into the reservoir): water, oil,
 * polymer.  Cell unknowns in slots 0-2, bottom-hole pressure in slot 6. */
void perf_rates(const Oracle& o, const Perf& pf, const Dual x[3], const Dual& pb, Dual q[3]) {
    const OraModel& m = o.m;
    int w = pf.well;
    Props<Dual> p = props(o, pf.cell, x[0], x[1], x[2]);
    Dual pbm = pb + o.w_gamma[w] * (pf.depth - o.w_zref[w]);   /* eq:ssw:dp */
    Dual draw = pbm - x[0];
    Dual lw = p.krw / (p.rk * p.mu_we);
    Dual lo = p.kro / m.mu_o;
    if (o.w_inj[w] && draw.v >= 0.0) {
        /* injection (wellbore pressure at or above the cell's): the injected
           water enters with the cell's total mobility and carries C_inj */
        q[0] = pf.wi * (lw + lo) * p.rho_w * draw;                  /* eq:ssw:Q, total mobility */
        q[1] = Dual(0.0);
        q[2] = q[0] * (o.w_cinj[w] / m.rho_w0);
    } else {
        /* production, and backflow into an injector's wellbore: eq:ssw:Q as
           written, each phase with the cell's mobility; polymer leaves at the
           cell's concentration */
        q[0] = pf.wi * lw * p.rho_w * draw;
        q[1] = pf.wi * lo * p.rho_o * draw;
        q[2] = q[0] * (x[2] / m.rho_w0);
    }
}

void load_cell(const double* x, int64_t i, int slot0, Dual out[3]) {
    for (int k = 0; k < 3; ++k) out[k] = Dual::var(x[3 * i + k], slot0 + k);
}

struct Sink {
    /* receives residual values and (optionally) Jacobian triplets */
    double* R;
    int32_t* I; int32_t* J; double* V; int64_t nnz; int64_t cap;
    double* Rcell;   /* when set: the three residual values of the cell just evaluated go here */
    void add(int64_t row, int64_t col, double v) {
        if (!I) return;
        if (nnz < cap) { I[nnz] = (int32_t)row; J[nnz] = (int32_t)col; V[nnz] = v; }
        ++nnz;
    }
};

/* All equations of cell i (gather form: accumulation, the six faces, the
 * perforations in the cell). */
void cell_equations(const Oracle& o, int64_t i, const double* x, const double* Mn, double dt, Sink& s) {
    const OraModel& m = o.m;
    int nx = m.nx, ny = m.ny, nz = m.nz;
    int ix = (int)(i % nx), iy = (int)((i / nx) % ny), iz = (int)(i / ((int64_t)nx * ny));
    Dual xi[3];
    load_cell(x, i, 0, xi);
    Dual acc[3];
    accumulation(o, i, xi[0], xi[1], xi[2], acc);
    Dual res[3];
    for (int e = 0; e < 3; ++e) res[e] = acc[e] - Mn[3 * i + e];
    for (int e = 0; e < 3; ++e)
        for (int k = 0; k < 3; ++k) s.add(3 * i + e, 3 * i + k, res[e].d[k]);

    /* six faces */
    struct Nb { int dix, diy, diz; };
    const Nb nbs[6] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
    for (int f = 0; f < 6; ++f) {
        int jx = ix + nbs[f].dix, jy = iy + nbs[f].diy, jz = iz + nbs[f].diz;
        if (jx < 0 || jx >= nx || jy < 0 || jy >= ny || jz < 0 || jz >= nz) continue;
        int64_t j = cell_index(o, jx, jy, jz);
        int dir = f / 2;
        double area, len, kL, kR;
        int64_t L = std::min(i, j), R = std::max(i, j);
        if (dir == 0) { area = m.dy * m.dz; len = m.dx; kL = o.kx[L]; kR = o.kx[R]; }
        else if (dir == 1) { area = m.dx * m.dz; len = m.dy; kL = o.ky[L]; kR = o.ky[R]; }
        else { area = m.dx * m.dy; len = m.dz; kL = o.kz[L]; kR = o.kz[R]; }
        double T = face_trans(area, len, kL, kR);
        int izL = (int)(L / ((int64_t)nx * ny)), izR = (int)(R / ((int64_t)nx * ny));
        double dzd = cell_depth(o, izR) - cell_depth(o, izL);
        Dual xL[3], xR[3];
        load_cell(x, L, 0, xL);
        load_cell(x, R, 3, xR);
        Dual F[3];
        face_flux(o, L, R, T, dzd, xL, xR, F);
        double sgn = (i == L) ? 1.0 : -1.0;     /* outflow from L is inflow to R */
        int si = (i == L) ? 0 : 3;              /* derivative slots of cell i */
        int sj = (i == L) ? 3 : 0;
        for (int e = 0; e < 3; ++e) {
            res[e].v += sgn * dt * F[e].v;
            for (int k = 0; k < 3; ++k) {
                s.add(3 * i + e, 3 * i + k, sgn * dt * F[e].d[si + k]);
                s.add(3 * i + e, 3 * j + k, sgn * dt * F[e].d[sj + k]);
            }
        }
    }

    /* perforations in this cell */
    for (int64_t p = o.perf_start[i]; p < o.perf_start[i + 1]; ++p) {
        const Perf& pf = o.perfs[p];
        Dual pb = Dual::var(x[3 * o.n + pf.well], 6);
        Dual q[3];
        perf_rates(o, pf, xi, pb, q);
        for (int e = 0; e < 3; ++e) {
            res[e].v -= dt * q[e].v;
            for (int k = 0; k < 3; ++k) s.add(3 * i + e, 3 * i + k, -dt * q[e].d[k]);
            s.add(3 * i + e, 3 * o.n + pf.well, -dt * q[e].d[6]);
        }
    }
    if (s.R)
        for (int e = 0; e < 3; ++e) s.R[3 * i + e] = res[e].v;
    if (s.Rcell)
        for (int e = 0; e < 3; ++e) s.Rcell[e] = res[e].v;
}

/* Well equation of well w (Sec. 2.4 well constraints). */
void well_equation(const Oracle& o, int w, const double* x, Sink& s) {
    const OraModel& m = o.m;
    int64_t row = 3 * o.n + w;
    int ctrl = o.w_ctrl[w];
    if (ctrl == 0) {    /* fixed bottom-hole pressure */
        if (s.R) s.R[row] = x[row] - o.w_target[w];
        s.add(row, row, 1.0);
        return;
    }
    double val = 0.0;
    double dpb = 0.0;
    for (int pi : o.well_perfs[w]) {
        const Perf& pf = o.perfs[pi];
        Dual xc[3];
        load_cell(x, pf.cell, 0, xc);
        Dual pb = Dual::var(x[row], 6);
        Dual q[3];
        perf_rates(o, pf, xc, pb, q);
        Dual vol;   /* surface volume rate of the controlled stream */
        if (ctrl == 1) vol = q[0] / m.rho_w0;
        else if (ctrl == 2) vol = q[1] / m.rho_o0;
        else vol = q[0] / m.rho_w0 + q[1] / m.rho_o0;
        val += vol.v;
        dpb += vol.d[6];
        for (int k = 0; k < 3; ++k) s.add(row, 3 * pf.cell + k, vol.d[k]);
    }
    if (s.R) s.R[row] = val - o.w_target[w];
    s.add(row, row, dpb);
}

}  // namespace

extern "C" {

void* ora_create(const OraModel* mp) {
    Oracle* o = new Oracle();
    o->m = *mp;
    const OraModel& m = o->m;
    o->n = (int64_t)m.nx * m.ny * m.nz;
    o->poro.assign(m.poro, m.poro + o->n);
    o->kx.assign(m.kx, m.kx + o->n);
    o->ky.assign(m.ky, m.ky + o->n);
    o->kz.assign(m.kz, m.kz + o->n);
    o->m.poro = o->poro.data(); o->m.kx = o->kx.data(); o->m.ky = o->ky.data(); o->m.kz = o->kz.data();
    o->vol = m.dx * m.dy * m.dz;
    o->cap.assign(o->n, 1.0);
    o->rrf.assign(o->n, m.rrf);
    o->hist.assign(o->n, 0.0);
    if (m.n_kperm > 0) {
        /* the table in log10 of permeability; end values held outside it */
        std::vector<double> lk(m.n_kperm), r(m.kperm_rrf, m.kperm_rrf + m.n_kperm),
            a(m.kperm_admax, m.kperm_admax + m.n_kperm);
        for (int k = 0; k < m.n_kperm; ++k) lk[k] = std::log10(m.kperm_k[k]);
        for (int64_t i = 0; i < o->n; ++i) {
            const Dual v(std::log10(o->kx[i]));
            o->rrf[i] = table_lookup(lk, r, v).v;
            o->cap[i] = table_lookup(lk, a, v).v / m.ads_max;
        }
    }
    o->pvr.resize(o->n);
    for (int64_t i = 0; i < o->n; ++i) o->pvr[i] = o->poro[i] * o->vol;
    int nw = m.nwell;
    o->w_ix.assign(m.w_ix, m.w_ix + nw); o->w_iy.assign(m.w_iy, m.w_iy + nw);
    o->w_k0.assign(m.w_k0, m.w_k0 + nw); o->w_k1.assign(m.w_k1, m.w_k1 + nw);
    o->w_inj.assign(m.w_inj, m.w_inj + nw); o->w_ctrl.assign(m.w_ctrl, m.w_ctrl + nw);
    o->w_target.assign(m.w_target, m.w_target + nw); o->w_cinj.assign(m.w_cinj, m.w_cinj + nw);
    o->w_rw.assign(m.w_rw, m.w_rw + nw); o->w_skin.assign(m.w_skin, m.w_skin + nw);
    o->w_dir.assign(m.w_dir, m.w_dir + nw); o->w_ix1.assign(m.w_ix1, m.w_ix1 + nw);
    o->ads_c.assign(m.ads_c, m.ads_c + m.n_ads); o->ads_a.assign(m.ads_a, m.ads_a + m.n_ads);
    o->visc_c.assign(m.visc_c, m.visc_c + m.n_visc); o->visc_m.assign(m.visc_m, m.visc_m + m.n_visc);
    o->pc_s.assign(m.pc_s, m.pc_s + m.n_pc); o->pc_v.assign(m.pc_v, m.pc_v + m.n_pc);
    o->w_zref.resize(nw); o->w_gamma.resize(nw);
    o->well_perfs.assign(nw, {});
    std::vector<Perf> pl;
    for (int w = 0; w < nw; ++w) {
        o->w_zref[w] = cell_depth(*o, o->w_k0[w]);
        o->w_gamma[w] = (o->w_inj[w] ? m.rho_w0 : m.rho_o0) * m.grav;
        if (o->w_dir[w] == 1) {      /* horizontal along x in row w_iy of layer w_k0 */
            for (int i = o->w_ix[w]; i <= o->w_ix1[w]; ++i) {
                int64_t c = cell_index(*o, i, o->w_iy[w], o->w_k0[w]);
                Perf p;
                p.well = w; p.cell = (int)c; p.depth = cell_depth(*o, o->w_k0[w]);
                p.wi = well_index_x(m.dx, m.dy, m.dz, o->ky[c], o->kz[c], o->w_rw[w], o->w_skin[w]);
                pl.push_back(p);
            }
            continue;
        }
        for (int k = o->w_k0[w]; k <= o->w_k1[w]; ++k) {
            int64_t c = cell_index(*o, o->w_ix[w], o->w_iy[w], k);
            Perf p;
            p.well = w; p.cell = (int)c; p.depth = cell_depth(*o, k);
            p.wi = well_index_z(m.dx, m.dy, m.dz, o->kx[c], o->ky[c], o->w_rw[w], o->w_skin[w]);
            pl.push_back(p);
        }
    }
    std::stable_sort(pl.begin(), pl.end(), [](const Perf& a, const Perf& b) { return a.cell < b.cell; });
    o->perfs = pl;
    o->perf_start.assign(o->n + 1, 0);
    for (const Perf& p : pl) o->perf_start[p.cell + 1]++;
    for (int64_t i = 0; i < o->n; ++i) o->perf_start[i + 1] += o->perf_start[i];
    for (size_t p = 0; p < o->perfs.size(); ++p) o->well_perfs[o->perfs[p].well].push_back((int)p);
    return o;
}

void ora_destroy(void* h) { delete (Oracle*)h; }

int64_t ora_n_perf(void* h) { return (int64_t)((Oracle*)h)->perfs.size(); }

/* Change a well's control and target (well operations change only between
   timesteps, Sec. 3 item 4). */
void ora_set_well_control(void* h, int w, int ctrl, double target) {
    Oracle& o = *(Oracle*)h;
    o.w_ctrl[w] = ctrl;
    o.w_target[w] = target;
}

/* Static data for tests: transmissibility to the +x/+y/+z neighbour of every
 * cell (0 on the outer boundary), reference pore volume, and per perforation
 * (in cell order) its well, cell and index. */
void ora_static(void* h, double* Tx, double* Ty, double* Tz, double* PVr,
                int32_t* perf_well, int32_t* perf_cell, double* perf_wi) {
    Oracle& o = *(Oracle*)h;
    const OraModel& m = o.m;
    for (int iz = 0; iz < m.nz; ++iz)
        for (int iy = 0; iy < m.ny; ++iy)
            for (int ix = 0; ix < m.nx; ++ix) {
                int64_t i = cell_index(o, ix, iy, iz);
                Tx[i] = ix + 1 < m.nx ? face_trans(m.dy * m.dz, m.dx, o.kx[i], o.kx[i + 1]) : 0.0;
                Ty[i] = iy + 1 < m.ny ? face_trans(m.dx * m.dz, m.dy, o.ky[i], o.ky[i + m.nx]) : 0.0;
                Tz[i] = iz + 1 < m.nz ? face_trans(m.dx * m.dy, m.dz, o.kz[i], o.kz[i + (int64_t)m.nx * m.ny]) : 0.0;
                PVr[i] = o.pvr[i];
            }
    for (size_t p = 0; p < o.perfs.size(); ++p) {
        perf_well[p] = o.perfs[p].well;
        perf_cell[p] = o.perfs[p].cell;
        perf_wi[p] = o.perfs[p].wi;
    }
}

/* Peaceman index of one vertical perforation (exposed for its pins). */
double ora_well_index_z(double dx, double dy, double h, double kx, double ky, double rw, double skin) {
    return well_index_z(dx, dy, h, kx, ky, rw, skin);
}

double ora_well_index_x(double h, double hy, double hz, double ky, double kz, double rw, double skin) {
    return well_index_x(h, hy, hz, ky, kz, rw, skin);
}

/* Change a well's injected polymer concentration (between timesteps). */
void ora_set_well_cinj(void* h, int w, double cinj) { ((Oracle*)h)->w_cinj[w] = cinj; }

/* Property values at one state of cell i:
 * out = {phi, rho_w, rho_o, krw, kro, mu_we, mu_pe, ads, Rk}. */
void ora_cell_props(void* h, int64_t i, double P, double S, double C, double* out) {
    Oracle& o = *(Oracle*)h;
    Props<Dual> p = props(o, i, Dual(P), Dual(S), Dual(C));
    out[0] = p.phi.v; out[1] = p.rho_w.v; out[2] = p.rho_o.v; out[3] = p.krw.v; out[4] = p.kro.v;
    out[5] = p.mu_we.v; out[6] = p.mu_pe.v; out[7] = p.ads.v; out[8] = p.rk.v;
}

/* Equilibrium adsorption of every cell at the concentrations of x (the
   isotherm scaled by the cell's capacity), N values. */
void ora_isotherm(void* h, const double* x, double* out) {
    Oracle& o = *(Oracle*)h;
    const OraModel& m = o.m;
    for (int64_t i = 0; i < o.n; ++i) {
        const Dual C(x[3 * i + 2]);
        Dual eq = m.n_ads > 0 ? table_lookup(o.ads_c, o.ads_a, C) : m.ads_max * m.ads_b * C / (1.0 + m.ads_b * C);
        out[i] = o.cap[i] * eq.v;
    }
}

/* The largest past adsorption of every cell (N values). */
void ora_set_ads_hist(void* h, const double* H) {
    Oracle& o = *(Oracle*)h;
    o.hist.assign(H, H + o.n);
}

/* Per-cell RRF and A_d,max (N values each). */
void ora_cell_rock(void* h, double* rrf, double* admax) {
    Oracle& o = *(Oracle*)h;
    for (int64_t i = 0; i < o.n; ++i) {
        rrf[i] = o.rrf[i];
        admax[i] = o.cap[i] * o.m.ads_max;
    }
}

/* Accumulation of every cell, block-wise (3N). */
void ora_accum(void* h, const double* x, double* M) {
    Oracle& o = *(Oracle*)h;
    for (int64_t i = 0; i < o.n; ++i) {
        Dual a[3];
        accumulation(o, i, Dual(x[3 * i]), Dual(x[3 * i + 1]), Dual(x[3 * i + 2]), a);
        for (int e = 0; e < 3; ++e) M[3 * i + e] = a[e].v;
    }
}

/* Face flux between cell L and its +dir neighbour (dir 0,1,2 = x,y,z) at
 * state x; F[3] = water, oil, polymer mass rate L -> R (kg/s). */
void ora_face_flux(void* h, const double* x, int64_t L, int dir, double* F) {
    Oracle& o = *(Oracle*)h;
    const OraModel& m = o.m;
    int64_t R = L + (dir == 0 ? 1 : dir == 1 ? m.nx : (int64_t)m.nx * m.ny);
    double area = dir == 0 ? m.dy * m.dz : dir == 1 ? m.dx * m.dz : m.dx * m.dy;
    double len = dir == 0 ? m.dx : dir == 1 ? m.dy : m.dz;
    const std::vector<double>& k = dir == 0 ? o.kx : dir == 1 ? o.ky : o.kz;
    double T = face_trans(area, len, k[L], k[R]);
    double dzd = dir == 2 ? m.dz : 0.0;
    Dual xL[3], xR[3], Fd[3];
    load_cell(x, L, 0, xL);
    load_cell(x, R, 3, xR);
    face_flux(o, L, R, T, dzd, xL, xR, Fd);
    for (int e = 0; e < 3; ++e) F[e] = Fd[e].v;
}

/* Perforation rates at state x, per perforation in cell order: q[3p+e]. */
void ora_perf_rates(void* h, const double* x, double* q) {
    Oracle& o = *(Oracle*)h;
    for (size_t p = 0; p < o.perfs.size(); ++p) {
        const Perf& pf = o.perfs[p];
        Dual xc[3];
        load_cell(x, pf.cell, 0, xc);
        Dual pb = Dual::var(x[3 * o.n + pf.well], 6);
        Dual qq[3];
        perf_rates(o, pf, xc, pb, qq);
        for (int e = 0; e < 3; ++e) q[3 * p + e] = qq[e].v;
    }
}

/* Residual [R; W] of length 3N + nwell. */
void ora_residual(void* h, const double* x, const double* Mn, double dt, double* R) {
    Oracle& o = *(Oracle*)h;
    Sink s{R, nullptr, nullptr, nullptr, 0, 0, nullptr};
    for (int64_t i = 0; i < o.n; ++i) cell_equations(o, i, x, Mn, dt, s);
    for (int w = 0; w < o.m.nwell; ++w) well_equation(o, w, x, s);
}

/* Accumulation of the cells i0 <= i < i1 (block-wise, into M[3*i0 ..]). */
void ora_accum_range(void* h, const double* x, int64_t i0, int64_t i1, double* M) {
    Oracle& o = *(Oracle*)h;
    for (int64_t i = i0; i < i1; ++i) {
        Dual a[3];
        accumulation(o, i, Dual(x[3 * i]), Dual(x[3 * i + 1]), Dual(x[3 * i + 2]), a);
        for (int e = 0; e < 3; ++e) M[3 * i + e] = a[e].v;
    }
}

/* The well equations' residuals alone (n_wells values). */
void ora_well_residuals(void* h, const double* x, double* W) {
    Oracle& o = *(Oracle*)h;
    std::vector<double> tmp(3 * o.n + o.m.nwell, 0.0);
    Sink s{tmp.data(), nullptr, nullptr, nullptr, 0, 0, nullptr};
    for (int w = 0; w < o.m.nwell; ++w) {
        well_equation(o, w, x, s);
        W[w] = tmp[3 * o.n + w];
    }
}

/* Residual rows of a subset of cells (3 per listed cell, in list order). */
void ora_residual_cells(void* h, const double* x, const double* Mn, double dt,
                        const int64_t* cells, int64_t ncells, double* Rsub) {
    Oracle& o = *(Oracle*)h;
    for (int64_t c = 0; c < ncells; ++c) {
        Sink s{nullptr, nullptr, nullptr, nullptr, 0, 0, Rsub + 3 * c};
        cell_equations(o, cells[c], x, Mn, dt, s);
    }
}

/* Jacobian triplets (duplicates to be summed) of the rows of the listed
 * cells (all cells when cells == NULL) and, if with_wells, of the well rows.
 * Returns the number of triplets; nothing beyond cap is written. */
int64_t ora_jacobian(void* h, const double* x, const double* Mn, double dt,
                     const int64_t* cells, int64_t ncells, int with_wells,
                     int32_t* I, int32_t* J, double* V, int64_t cap) {
    Oracle& o = *(Oracle*)h;
    Sink s{nullptr, I, J, V, 0, cap, nullptr};
    if (cells) {
        for (int64_t c = 0; c < ncells; ++c) cell_equations(o, cells[c], x, Mn, dt, s);
    } else {
        for (int64_t i = 0; i < o.n; ++i) cell_equations(o, i, x, Mn, dt, s);
    }
    if (with_wells)
        for (int w = 0; w < o.m.nwell; ++w) well_equation(o, w, x, s);
    return s.nnz;
}

}  // extern "C"
