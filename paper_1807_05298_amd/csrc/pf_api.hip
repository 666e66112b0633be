// Host orchestration and the C ABI of polyflood.h: workspace plan, static
// set-up, Newton iteration (Algorithm 1 with the forcing term of eq. fterm),
// the flexible GMRES driver and the timestep rules (Sec. 3 item 4).
#include "pf_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <mutex>
#include <stdexcept>

namespace pf {

// Visits every cell of a multigrid level: f(natural index, slot).
template <class F>
void for_level_cells(const MGLevel& L, F&& f) {
    int64_t i = 0;
    for (int iz = 0; iz < L.nz; ++iz)
        for (int iy = 0; iy < L.ny; ++iy)
            for (int ix = 0; ix < L.nx; ++ix, ++i) f(i, mg_slot(L, ix, iy, iz));
}

static thread_local std::string g_error;
void set_error(const std::string& msg) { g_error = msg; }

struct InvalidArg { std::string msg; };

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}


void validate(const pf_model_desc* d, const pf_solver_opts* o) {
    if (!d || !o) throw InvalidArg{"null model or options"};
    const pf_grid& g = d->grid;
    if (g.nx < 1 || g.ny < 1 || g.nz < 1) throw InvalidArg{"grid dimensions must be >= 1"};
    if (!(g.dx > 0 && g.dy > 0 && g.dz > 0)) throw InvalidArg{"block sizes must be > 0"};
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    if (n > (int64_t)1 << 31) throw InvalidArg{"more than 2^31 cells"};
    if (!d->rock.poro || !d->rock.kx || !d->rock.ky || !d->rock.kz) throw InvalidArg{"missing rock arrays"};
    const pf_fluid& f = d->fluid;
    if (!(f.swc >= 0 && f.sor >= 0 && f.swc + f.sor < 1)) throw InvalidArg{"need 0 <= swc, sor and swc + sor < 1"};
    if (!(f.n_w >= 1 && f.n_o >= 1)) throw InvalidArg{"Corey exponents must be >= 1"};
    if (!(f.mu_w > 0 && f.mu_o > 0 && f.rho_w0 > 0 && f.rho_o0 > 0)) throw InvalidArg{"bad fluid constants"};
    const pf_polymer& p = d->polymer;
    if (!(p.ads_max > 0 && p.ads_b >= 0 && p.rrf >= 1 && p.ipv >= 0 && p.ipv < 1))
        throw InvalidArg{"bad polymer constants"};
    if (!(p.omega >= 0 && p.omega <= 1)) throw InvalidArg{"omega must lie in [0, 1]"};
    auto check_table = [](int n, const double* x, const double* y, const char* what, bool positive) {
        if (n == 0) return;
        if (n < 2 || n > PF_TABLE_MAX) throw InvalidArg{std::string(what) + ": need 2.." + std::to_string(PF_TABLE_MAX) + " points"};
        for (int k = 0; k < n; ++k) {
            if (!std::isfinite(x[k]) || !std::isfinite(y[k]) || (positive && !(y[k] > 0)))
                throw InvalidArg{std::string(what) + ": bad value"};
            if (k > 0 && !(x[k] > x[k - 1])) throw InvalidArg{std::string(what) + ": abscissae must increase"};
        }
    };
    check_table(p.n_ads, p.ads_c, p.ads_a, "adsorption table", false);
    check_table(p.n_visc, p.visc_c, p.visc_m, "viscosity table", true);
    check_table(f.n_pc, f.pc_s, f.pc_v, "capillary pressure table", false);
    check_table(p.n_kperm, p.kperm_k, p.kperm_rrf, "rock permeability table (RRF)", true);
    check_table(p.n_kperm, p.kperm_k, p.kperm_admax, "rock permeability table (A_d,max)", true);
    for (int k = 0; k < p.n_kperm; ++k)
        if (!(p.kperm_k[k] > 0 && p.kperm_rrf[k] >= 1.0)) throw InvalidArg{"rock permeability table: need k > 0 and RRF >= 1"};
    if (!(p.ads_res >= 0.0 && p.ads_res <= 1.0)) throw InvalidArg{"ads_res must lie in [0, 1]"};
    if (p.mix_rule < PF_MIX_POLY || p.mix_rule > PF_MIX_TABLE) throw InvalidArg{"bad mixing rule"};
    if (p.mix_rule == PF_MIX_TABLE && p.n_visc == 0) throw InvalidArg{"PF_MIX_TABLE needs the viscosity table"};
    if (p.mix_rule != PF_MIX_POLY && p.mix_rule != PF_MIX_TABLE && !(p.c_max > 0))
        throw InvalidArg{"the mixing rules need c_max > 0"};
    if (!(p.mu_p_ref >= 0)) throw InvalidArg{"mu_p_ref must be >= 0"};
    if (p.omega != 1.0 && !(p.c_max > 0)) throw InvalidArg{"c_max must be > 0 when omega < 1"};
    if (d->n_wells < 0 || (d->n_wells > 0 && !d->wells)) throw InvalidArg{"bad well list"};
    for (int w = 0; w < d->n_wells; ++w) {
        const pf_well& W = d->wells[w];
        if (W.ix < 0 || W.ix >= g.nx || W.iy < 0 || W.iy >= g.ny || W.k_top < 0 || W.k_bot >= g.nz ||
            W.k_top > W.k_bot)
            throw InvalidArg{"well " + std::to_string(w) + " outside the grid"};
        if (W.control < PF_CTRL_BHP || W.control > PF_CTRL_LRATE) throw InvalidArg{"bad well control"};
        if (W.control != PF_CTRL_BHP && W.target == 0.0) throw InvalidArg{"rate target must be non-zero"};
        if (!(W.rw > 0)) throw InvalidArg{"wellbore radius must be > 0"};
        if (!(W.bhp_limit >= 0.0) || !std::isfinite(W.bhp_limit)) throw InvalidArg{"bhp_limit must be >= 0 (0: none)"};
        if (W.direction != PF_WELL_Z && W.direction != PF_WELL_X) throw InvalidArg{"bad well direction"};
        if (W.direction == PF_WELL_X && (W.k_bot != W.k_top || W.ix_last < W.ix || W.ix_last >= g.nx))
            throw InvalidArg{"horizontal well " + std::to_string(w) + ": need k_bot == k_top and ix <= ix_last < nx"};
    }
    if (o->restart < 1 || o->restart > kMaxRestart) throw InvalidArg{"restart must lie in [1, 64]"};
    if (o->max_lin_it < 1 || o->max_newton < 1 || o->max_cuts < 0) throw InvalidArg{"bad iteration limits"};
    if (o->precision != PF_PREC_FP64 && o->precision != PF_PREC_MIXED) throw InvalidArg{"bad precision"};
    if (o->smoother != PF_SMOOTH_BJAC && o->smoother != PF_SMOOTH_RBILU0) throw InvalidArg{"bad smoother"};
    if (o->cpr_order != PF_CPR_PF && o->cpr_order != PF_CPR_FP) throw InvalidArg{"bad CPR order"};
    if (o->mg_coarse > 1024) throw InvalidArg{"mg_coarse must be <= 1024"};
    if (o->mg_cycles < 1 || o->mg_cycles > 8) throw InvalidArg{"mg_cycles must lie in [1, 8]"};
    if (!(o->dt_init >= 0.0)) throw InvalidArg{"dt_init must be >= 0"};
    if (o->zline_len < 0 || o->zline_len > 4096) throw InvalidArg{"zline_len must lie in [0, 4096]"};
    if (o->mg_pre_small < 0 || o->mg_pre_small > 64) throw InvalidArg{"mg_pre_small must lie in [0, 64]"};
    if (o->mg_small_cells < 0) throw InvalidArg{"mg_small_cells must be >= 0"};
}

struct HostWells {
    std::vector<int32_t> perf_cell, perf_well, pc_cell, pc_first, wp_first, wp_idx, ctrl, inj, dir;
    std::vector<double> perf_depth, target, cinj, gamma, zref, scale, rw, skin, limit;
};

HostWells build_wells(const pf_model_desc* d) {
    HostWells h;
    const pf_grid& g = d->grid;
    struct P { int32_t cell, well; double depth; };
    std::vector<P> perfs;
    for (int w = 0; w < d->n_wells; ++w) {
        const pf_well& W = d->wells[w];
        if (W.direction == PF_WELL_X) {
            for (int i = W.ix; i <= W.ix_last; ++i)
                perfs.push_back({(int32_t)(i + (int64_t)g.nx * (W.iy + (int64_t)g.ny * W.k_top)), w,
                                 g.top_depth + (W.k_top + 0.5) * g.dz});
        } else {
            for (int k = W.k_top; k <= W.k_bot; ++k)
                perfs.push_back({(int32_t)(W.ix + (int64_t)g.nx * (W.iy + (int64_t)g.ny * k)), w,
                                 g.top_depth + (k + 0.5) * g.dz});
        }
    }
    std::stable_sort(perfs.begin(), perfs.end(), [](const P& a, const P& b) { return a.cell < b.cell; });
    for (const P& p : perfs) {
        h.perf_cell.push_back(p.cell);
        h.perf_well.push_back(p.well);
        h.perf_depth.push_back(p.depth);
    }
    for (size_t k = 0; k < perfs.size(); ++k) {
        if (k == 0 || perfs[k].cell != perfs[k - 1].cell) {
            h.pc_cell.push_back(perfs[k].cell);
            h.pc_first.push_back((int32_t)k);
        }
    }
    h.pc_first.push_back((int32_t)perfs.size());
    h.wp_first.assign(d->n_wells + 1, 0);
    for (const P& p : perfs) h.wp_first[p.well + 1]++;
    for (int w = 0; w < d->n_wells; ++w) h.wp_first[w + 1] += h.wp_first[w];
    h.wp_idx.assign(perfs.size(), 0);
    std::vector<int32_t> fill(h.wp_first.begin(), h.wp_first.end() - (d->n_wells > 0 ? 1 : 0));
    for (size_t k = 0; k < perfs.size(); ++k) h.wp_idx[fill[perfs[k].well]++] = (int32_t)k;
    for (int w = 0; w < d->n_wells; ++w) {
        const pf_well& W = d->wells[w];
        h.ctrl.push_back(W.control);
        h.inj.push_back(W.is_injector ? 1 : 0);
        h.target.push_back(W.target);
        h.cinj.push_back(W.c_inj);
        h.gamma.push_back((W.is_injector ? d->fluid.rho_w0 : d->fluid.rho_o0) * d->fluid.gravity);
        h.zref.push_back(g.top_depth + (W.k_top + 0.5) * g.dz);
        h.scale.push_back(W.control == PF_CTRL_BHP ? 1.0 / kBar : 1.0 / std::fabs(W.target));
        h.rw.push_back(W.rw);
        h.skin.push_back(W.skin);
        h.limit.push_back(W.bhp_limit);
        h.dir.push_back(W.direction);
    }
    return h;
}

DevModel make_devmodel(const pf_model_desc* d, const HostWells& h) {
    DevModel m;
    std::memset(&m, 0, sizeof(m));
    const pf_grid& g = d->grid;
    m.nx = g.nx; m.ny = g.ny; m.nz = g.nz; m.nw = d->n_wells;
    m.nxy = (int64_t)g.nx * g.ny;
    m.n = m.nxy * g.nz;
    m.np = (int64_t)h.perf_cell.size();
    m.npc = (int64_t)h.pc_cell.size();
    m.dx = g.dx; m.dy = g.dy; m.dz = g.dz; m.top = g.top_depth; m.vol = g.dx * g.dy * g.dz;
    m.cr = d->rock.cr; m.pref = d->rock.p_ref;
    const pf_fluid& f = d->fluid;
    m.rho_w0 = f.rho_w0; m.rho_o0 = f.rho_o0; m.c_w = f.c_w; m.c_o = f.c_o; m.mu_w = f.mu_w; m.mu_o = f.mu_o;
    m.swc = f.swc; m.sor = f.sor; m.n_w = f.n_w; m.n_o = f.n_o; m.krw0 = f.krw0; m.kro0 = f.kro0; m.grav = f.gravity;
    const pf_polymer& p = d->polymer;
    m.a1 = p.a1; m.a2 = p.a2; m.omega = p.omega; m.cmax = p.c_max;
    m.mup_ref = p.mu_p_ref > 0.0 ? p.mu_p_ref : f.mu_w * (1.0 + p.a1 * p.c_max + p.a2 * p.c_max * p.c_max);
    m.mix_rule = p.mix_rule;
    m.mix_ln = std::log(m.mup_ref / f.mu_w);
    m.n_ads = p.n_ads;
    m.n_visc = p.n_visc;
    m.n_pc = f.n_pc;
    m.tab = nullptr;                 // set once the workspace is planned
    m.ads_max = p.ads_max; m.ads_b = p.ads_b; m.rrf = p.rrf; m.ipv = p.ipv;
    m.inv_den = 1.0 / (1.0 - f.swc - f.sor);
    m.tl_pref = std::pow(m.mup_ref, 1.0 - p.omega);
    m.tl_pw = std::pow(f.mu_w, 1.0 - p.omega);
    double cmax_inj = 0.0;
    for (int w = 0; w < d->n_wells; ++w)
        if (d->wells[w].is_injector) cmax_inj = std::max(cmax_inj, d->wells[w].c_inj);
    m.c_ref = std::max(cmax_inj, 1.0);
    m.inv_mu_o = 1.0 / m.mu_o;
    m.inv_rho_w0 = 1.0 / m.rho_w0;
    m.inv_vol = 1.0 / m.vol;
    m.rk_slope = (m.rrf - 1.0) / m.ads_max;
    m.inv_rho_o0 = 1.0 / m.rho_o0;
    m.inv_c_ref = 1.0 / m.c_ref;
    m.n_kperm = p.n_kperm;
    m.ads_res = p.ads_res;
    m.cell_cap = m.cell_rks = m.ads_hist = nullptr;      // set once the workspace is planned
    m.corey2_w = f.n_w == 2.0;
    m.corey2_o = f.n_o == 2.0;
    m.omega1 = p.omega == 1.0;
    return m;
}

size_t plan(Sim& s, char* base) {
    Bump b{base};
    const DevModel& m = s.m;
    const int64_t n = m.n, nv = s.nv;
    const int64_t np = std::max<int64_t>(m.np, 1), nw = std::max<int32_t>(m.nw, 1);
    const int64_t npc = std::max<int64_t>(m.npc, 1);
    s.poro = b.take<double>(n); s.kx = b.take<double>(n); s.ky = b.take<double>(n); s.kz = b.take<double>(n);
    s.pvr = b.take<double>(n); s.Tx = b.take<double>(n); s.Ty = b.take<double>(n); s.Tz = b.take<double>(n);
    s.rscale = b.take<double>(nv);
    s.perf_cell = b.take<int32_t>(np); s.perf_well = b.take<int32_t>(np);
    s.pc_cell = b.take<int32_t>(npc); s.pc_first = b.take<int32_t>(npc + 1);
    s.pc_map = b.take<int32_t>(n);
    s.wp_first = b.take<int32_t>(nw + 1); s.wp_idx = b.take<int32_t>(np);
    s.perf_wi = b.take<double>(np); s.perf_depth = b.take<double>(np);
    s.w_ctrl = b.take<int32_t>(nw); s.w_inj = b.take<int32_t>(nw); s.w_dir = b.take<int32_t>(nw);
    s.w_target = b.take<double>(nw); s.w_cinj = b.take<double>(nw); s.w_gamma = b.take<double>(nw);
    s.w_zref = b.take<double>(nw); s.w_scale = b.take<double>(nw); s.w_rw = b.take<double>(nw);
    s.w_skin = b.take<double>(nw);
    s.x = b.take<double>(nv); s.xn = b.take<double>(nv); s.Mn = b.take<double>(3 * n);
    s.R = b.take<double>(nv); s.J = b.take<double>(63 * n);
    s.B = b.take<double>(3 * np); s.Cw = b.take<double>(3 * np); s.Dw = b.take<double>(nw);
    s.wv = b.take<double>(np); s.wdp = b.take<double>(np);
    s.perf_q = b.take<double>(2 * np);
    s.tab = b.take<double>(kTabSlots * PF_TABLE_MAX);
    s.cell_cap = m.n_kperm > 0 ? b.take<double>(n) : nullptr;
    s.cell_rks = m.n_kperm > 0 ? b.take<double>(n) : nullptr;
    s.ads_hist = m.ads_res > 0.0 ? b.take<double>(n) : nullptr;
    s.dx = b.take<double>(nv); s.rhs = b.take<double>(nv);
    const int mcap = s.restart_cap;
    // Krylov vectors: natural layout (nv) or, on the FP64 red-black ILU(0)
    // path, the colour-split one (nvc; longer by the pad slots when nx is odd)
    const bool fp64 = s.opts.precision != PF_PREC_MIXED;
    s.nvc = 6 * cs_ns(m) + m.nw;
    const int64_t kst = fp64 ? std::max(nv, s.nvc) : nv;
    s.kst = kst;
    s.nk = nv;
    s.V = b.take<double>((size_t)(mcap + 1) * kst);
    if (!fp64) {
        s.Z = nullptr;
        s.Z32 = b.take<float>((size_t)mcap * kst);
    } else {
        s.Z = b.take<double>((size_t)mcap * kst);
        s.Z32 = nullptr;
    }
    s.t1 = b.take<double>(kst); s.t2 = b.take<double>(kst);
    s.bcs = fp64 ? b.take<double>(s.nvc) : nullptr;
    s.xcs = fp64 ? b.take<double>(s.nvc) : nullptr;
    s.w = nullptr;
    s.kc = b.take<KrylovCtl>(1);
    s.part = b.take<double>((size_t)kPartSlots * kRedBlocks);
    s.red = b.take<double>(64);
    cpr_plan(s, b);
    return b.used + 256;
}

void upload(Sim& s, void* dst, const void* src, size_t bytes) { copy_h2d(s, dst, src, bytes); }

void sync(Sim& s) { stream_sync(s); }

// Active well controls to the device: control, target and the well row's
// scale (BHP rows by 1 bar, rate rows by |target|), also in the row scales
// of the convergence test.
void set_well_controls(Sim& s, const std::vector<int32_t>& ctrl, const std::vector<double>& target) {
    const int nw = s.m.nw;
    if (nw == 0) return;
    std::vector<double> scale(nw);
    for (int w = 0; w < nw; ++w) scale[w] = ctrl[w] == PF_CTRL_BHP ? 1.0 / kBar : 1.0 / std::fabs(target[w]);
    upload(s, s.w_ctrl, ctrl.data(), nw * 4);
    upload(s, s.w_target, target.data(), nw * 8);
    upload(s, s.w_scale, scale.data(), nw * 8);
    upload(s, s.rscale + 3 * s.m.n, scale.data(), nw * 8);
    sync(s);   // the host vectors must outlive the copies
    s.h_w_ctrl = ctrl;
    s.h_target = target;
}

// Surface water and oil rates of every well at the last assembled state.
void well_rates(Sim& s, std::vector<double>& qw, std::vector<double>& qo) {
    const int nw = s.m.nw;
    const int64_t np = s.m.np;
    qw.assign(nw, 0.0);
    qo.assign(nw, 0.0);
    if (np == 0) return;
    std::vector<double> q(2 * np);
    copy_d2h(s, q.data(), s.perf_q, 2 * np * 8);
    sync(s);
    // per well in perforation order (the order of the well equation's sum)
    for (int64_t k = 0; k < np; ++k) {
        qw[s.h_perf_well[k]] += q[2 * k];
        qo[s.h_perf_well[k]] += q[2 * k + 1];
    }
}

// The controlled surface stream of a rate control.
double controlled_rate(int ctrl, double qw, double qo) {
    return ctrl == PF_CTRL_WRATE ? qw : ctrl == PF_CTRL_ORATE ? qo : qw + qo;
}

// Between sub-steps (well operations are fixed within one): a rate-
// controlled well beyond its BHP limit continues at the limit; a well held
// at its limit whose rate there exceeds its target returns to the target.
// Returns the number of switches.
int apply_well_limits(Sim& s) {
    const int nw = s.m.nw;
    bool any = false;
    for (int w = 0; w < nw; ++w) any = any || (s.h_limit[w] > 0.0 && s.h_ctrl0[w] != PF_CTRL_BHP);
    if (!any) return 0;
    std::vector<double> pb(nw), qw, qo;
    copy_d2h(s, pb.data(), s.x + 3 * s.m.n, nw * 8);
    sync(s);
    well_rates(s, qw, qo);
    std::vector<int32_t> ctrl = s.h_w_ctrl;
    std::vector<double> target = s.h_target;
    int switches = 0;
    for (int w = 0; w < nw; ++w) {
        const double lim = s.h_limit[w];
        if (!(lim > 0.0) || s.h_ctrl0[w] == PF_CTRL_BHP) continue;
        if (ctrl[w] != PF_CTRL_BHP) {
            const bool beyond = s.h_inj[w] ? pb[w] > lim : pb[w] < lim;
            if (beyond) { ctrl[w] = PF_CTRL_BHP; target[w] = lim; ++switches; }
        } else {
            const double q = controlled_rate(s.h_ctrl0[w], qw[w], qo[w]);
            if (std::fabs(q) > std::fabs(s.h_target0[w])) { ctrl[w] = s.h_ctrl0[w]; target[w] = s.h_target0[w]; ++switches; }
        }
    }
    if (switches) set_well_controls(s, ctrl, target);
    return switches;
}

void read_back(Sim& s, const void* src, size_t bytes) {
    if (s.fu) {
        // in a fusion group a kernel writes the pinned buffer (one merged launch for all members)
        launch_copy_words(s, src, s.hbuf, bytes);
        sync(s);
        return;
    }
    PF_HIP(hipMemcpyAsync(s.hbuf, src, bytes, hipMemcpyDeviceToHost, s.stream));
    sync(s);
}

// Whether fgmres works in the colour-split layout (FP64, PF order, red-black
// ILU(0)).
bool fgmres_cs(const Sim& s) { return s.Z && cpr_colour_split(s); }

// Restarted flexible GMRES, right preconditioned by CPR, x0 = 0.  Returns the
// iteration count; *rel receives the final relative residual estimate.  b and
// x are in natural order; on the colour-split path (fgmres_cs) the Krylov
// vectors are in the colour-split layout, b is brought into it once and x out
// of it once, unless in_cs: then b is s.bcs and x is s.xcs, both already in
// (and left in) that layout.
int fgmres(Sim& s, const double* b_nat, double tol, double* x_nat, double* rel, int max_it, bool in_cs = false) {
    const int m = std::min<int>(s.opts.restart, s.restart_cap);
    const bool cs = fgmres_cs(s);
    s.nk = cs ? s.nvc : s.nv;
    const double* b = b_nat;
    double* x = x_nat;
    if (cs) {
        if (!in_cs) launch_to_cs(s, b_nat, s.bcs);
        b = s.bcs;
        x = s.xcs;
    }
    // x0 = 0: the first correction is written rather than added (x_set),
    // and x is zeroed only if the solve stops before any Krylov step
    bool x_set = false;
    int total = 0;
    bool first = true;
    double r_est = 1.0;
    for (;;) {
        const double* r0 = b;
        if (!first) {
            if (cs) {
                // r = b - J x through the natural-order product (restarts are rare)
                launch_from_cs(s, x, s.t2);
                launch_spmv(s, s.t2, s.t1);
                launch_to_cs(s, s.t1, s.t2);
                launch_axpby(s, s.nk, 1.0, b, -1.0, s.t2);
                r0 = s.t2;
            } else {
                launch_spmv(s, x, s.t1);
                launch_axpby(s, s.nk, 1.0, b, -1.0, s.t1);
                r0 = s.t1;
            }
        }
        launch_norm_to_ctl(s, r0, first ? 1 : 0);
        launch_scale_by_ctl(s, r0, s.V, 0);
        read_back(s, &s.kc->rel, 2 * sizeof(double) + 2 * sizeof(int32_t));
        r_est = s.hbuf[0];
        const int32_t brk = reinterpret_cast<const int32_t*>(s.hbuf + 1)[1];
        if (brk || r_est <= tol || total >= max_it) break;
        int k = 0;
        bool stop = false;
        for (int j = 0; j < m; ++j) {
            double* vj = s.V + (int64_t)j * s.kst;
            double* w = s.V + (int64_t)(j + 1) * s.kst;
            if (s.Z32) {
                float* zj = s.Z32 + (int64_t)j * s.kst;
                cpr_apply(s, vj, zj);
                launch_spmv(s, zj, w);
            } else {
                cpr_apply_spmv(s, vj, s.Z + (int64_t)j * s.kst, w);
            }
            launch_arnoldi(s, j, w);
            ++total;
            read_back(s, &s.kc->rel, 2 * sizeof(double) + 2 * sizeof(int32_t));
            if (!s.opts.reorth && reinterpret_cast<const int32_t*>(s.hbuf + 1)[0]) {
                // the first pass cancelled most of w: second pass, then the final estimate
                launch_arnoldi_second(s, j, w);
                read_back(s, &s.kc->rel, 2 * sizeof(double) + 2 * sizeof(int32_t));
            }
            r_est = s.hbuf[0];
            const int32_t bk = reinterpret_cast<const int32_t*>(s.hbuf + 1)[1];
            k = j + 1;
            if (!std::isfinite(r_est)) throw InvalidArg{"non-finite Krylov residual"};
            if (bk || r_est <= tol || total >= max_it) { stop = true; break; }
            if (!reinterpret_cast<const int32_t*>(s.hbuf + 1)[2]) launch_normalise(s, w);
        }
        launch_solve_small(s, k);
        launch_zcomb(s, k, x, !x_set);
        x_set = true;
        if (stop) break;
        first = false;
    }
    if (!x_set) launch_fill(s, s.nk, 0.0, x);
    if (cs && !in_cs) launch_from_cs(s, x, x_nat);
    s.nk = s.nv;
    if (rel) *rel = r_est;
    return total;
}

enum class NewtonState { Converged, Continue, Failed };

NewtonState newton_iteration(Sim& s, double dt, pf_step_stats* st) {
    const double t0 = now_s();
    launch_assemble(s, dt, true);
    launch_norms(s, s.R, s.red);
    read_back(s, s.red, 6 * sizeof(double));
    const double rmax = s.hbuf[4], bnorm = s.hbuf[5];
    const double t1 = now_s();
    if (st) { st->t_assemble += t1 - t0; st->res_norm = rmax; }
    if (!std::isfinite(rmax) || !std::isfinite(bnorm)) return NewtonState::Failed;
    if (s.newton_it > 0 && rmax <= s.opts.tol_res && s.last_upd <= s.opts.tol_upd) {
        if (st) { st->converged = 1; st->upd_norm = s.last_upd; }
        return NewtonState::Converged;
    }
    if (s.newton_it >= s.opts.max_newton) return NewtonState::Failed;
    // forcing term: third choice of eq. fterm, gamma = 0.5, beta = (1+sqrt 5)/2,
    // kept in [0.01, 0.1]; the first iteration uses the upper bound
    double eta = s.opts.lin_tol;
    if (s.opts.inexact) {
        if (s.newton_it == 0 || !(s.last_bnorm > 0)) eta = 0.1;
        else eta = 0.5 * std::pow(bnorm / s.last_bnorm, 0.5 * (1.0 + std::sqrt(5.0)));
        eta = std::min(0.1, std::max(0.01, eta));
    }
    // the right-hand side -R, on the colour-split path formed straight in the
    // solver's layout, whose solution the update then reads in place
    const bool csl = fgmres_cs(s);
    if (csl) launch_to_cs(s, s.R, s.bcs, -1.0);
    else launch_axpby(s, s.nv, -1.0, s.R, 0.0, s.rhs);
    cpr_setup(s);
    const double t2 = now_s();
    double rel = 0.0;
    int its = 0;
    try {
        its = fgmres(s, csl ? s.bcs : s.rhs, eta, csl ? s.xcs : s.dx, &rel, s.opts.max_lin_it, csl);
    } catch (const InvalidArg&) {
        return NewtonState::Failed;
    }
    launch_update(s, csl ? s.xcs : s.dx, s.red + 8, csl);
    read_back(s, s.red + 8, 5 * sizeof(double));
    const double t3 = now_s();
    s.last_upd = s.hbuf[4];
    s.last_bnorm = bnorm;
    s.newton_it++;
    if (st) {
        st->t_setup += t2 - t1;
        st->t_solve += t3 - t2;
        st->lin_its += its;
        st->newton_its += 1;
        st->lin_rel = rel;
        st->upd_norm = s.last_upd;
    }
    if (!std::isfinite(s.last_upd)) return NewtonState::Failed;
    return NewtonState::Continue;
}

void begin_step(Sim& s) {
    if (s.ads_hist) launch_ads_hist(s);     // retention: the converged state x^n is taken in first
    launch_copy(s, s.nv, s.x, s.xn);
    launch_accum(s, s.x, s.Mn);
    s.newton_it = 0;
    s.last_upd = INFINITY;
    s.last_bnorm = 0.0;
}

// the side stream and its events (after the last use: synchronised first)
void side_release(Sim& s) {
    if (s.aux) {
        (void)hipStreamSynchronize(s.aux);
        (void)hipStreamDestroy(s.aux);
        s.aux = nullptr;
    }
    if (s.ev_fork) (void)hipEventDestroy(s.ev_fork);
    if (s.ev_join) (void)hipEventDestroy(s.ev_join);
    s.ev_fork = s.ev_join = nullptr;
}

}  // namespace
}  // namespace pf

// ---- the static workspace of pf_create_static ----------------------------
// A fixed array in the library's device image, one copy on every GPU the
// library runs on, held until the process ends.  In host code the name
// 'scratch' is only a host-side stand-in: its device address on the current
// GPU comes from hipGetSymbolAddress, and only that address is used.
static constexpr size_t kStaticWorkspaceBytes = PF_STATIC_WORKSPACE_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

namespace {
constexpr int kMaxStaticDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxStaticDevices];                  // device address of scratch, per device
bool g_static_busy[kMaxStaticDevices];                  // held by a live simulator
double g_static_hbuf[kMaxStaticDevices][64];            // host read-back buffer of that simulator

// The device address of this device's array (looked up once per device,
// with the device current) if no live simulator holds it; marks it held.
void* static_workspace_acquire(int dev) {
    if (dev < 0 || dev >= kMaxStaticDevices) throw pf::InvalidArg{"device index beyond the static workspace table"};
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[dev]) {
        void* ptr = nullptr;
        PF_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr || ((uintptr_t)ptr & 255)) throw pf::HipError{"hipGetSymbolAddress returned an unusable address"};
        g_static_ptr[dev] = ptr;
    }
    if (g_static_busy[dev]) return nullptr;
    g_static_busy[dev] = true;
    return g_static_ptr[dev];
}

void static_workspace_release(int dev) {
    std::lock_guard<std::mutex> lk(g_static_mu);
    g_static_busy[dev] = false;
}

double* static_hbuf(int dev) { return g_static_hbuf[dev]; }
}  // namespace

using namespace pf;

struct pf_sim {
    Sim s;
};

pf::Sim& pf_sim_state(pf_sim* h) { return h->s; }

#define PF_API_BEGIN try {
#define PF_API_END                                             \
    }                                                          \
    catch (const pf::HipError& e) {                            \
        set_error(e.msg);                                      \
        return PF_EHIP;                                        \
    }                                                          \
    catch (const pf::InvalidArg& e) {                          \
        set_error(e.msg);                                      \
        return PF_EINVAL;                                      \
    }                                                          \
    catch (const std::exception& e) {                          \
        set_error(e.what());                                   \
        return PF_EINVAL;                                      \
    }

extern "C" {

const char* pf_last_error(void) { return g_error.c_str(); }

void pf_default_opts(pf_solver_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->precision = PF_PREC_FP64;
    o->cpr_order = PF_CPR_PF;
    o->smoother = PF_SMOOTH_RBILU0;
    o->restart = 30;
    o->max_lin_it = 200;
    o->max_newton = 12;
    o->max_cuts = 5;
    o->inexact = 1;
    o->tol_res = 1e-6;
    o->tol_upd = 1e-3;
    o->lin_tol = 1e-8;
    o->ds_max = 0.2;
    o->mg_pre = 1;
    o->mg_post = 0;
    o->mg_coarse = 96;
    o->mg_cycles = 2;
    o->mg_pre_small = 5;
    o->mg_small_cells = 50000;
    o->reorth = 0;
}

pf_status pf_workspace_size(const pf_model_desc* d, const pf_solver_opts* o, size_t* bytes) {
    PF_API_BEGIN
    validate(d, o);
    if (!bytes) throw InvalidArg{"null bytes"};
    Sim s;
    HostWells h = build_wells(d);
    s.m = make_devmodel(d, h);
    s.opts = *o;
    s.nv = 3 * s.m.n + s.m.nw;
    s.restart_cap = o->restart;
    cpr_choose_levels(s);
    *bytes = plan(s, nullptr);
    return PF_OK;
    PF_API_END
}

static pf_status create_sim(const pf_model_desc* d, const pf_solver_opts* o, void* dev_ws, size_t ws_bytes,
                            void* hip_stream, int static_dev, pf_sim** out) {
    PF_API_BEGIN
    validate(d, o);
    if (!out) throw InvalidArg{"null output handle"};
    if (((uintptr_t)dev_ws) & 255) throw InvalidArg{"workspace must be 256-byte aligned"};
    pf_sim* h = new pf_sim();
    Sim& s = h->s;
    try {
        HostWells hw = build_wells(d);
        s.m = make_devmodel(d, hw);
        s.opts = *o;
        s.stream = (hipStream_t)hip_stream;
        PF_HIP(hipGetDevice(&s.device));
        s.nv = 3 * s.m.n + s.m.nw;
        s.restart_cap = o->restart;
        cpr_choose_levels(s);
        const size_t need = plan(s, nullptr);
        if (ws_bytes < need) {
            delete h;
            set_error(static_dev >= 0
                          ? "model needs " + std::to_string(need) + " bytes of workspace; the static workspace holds " +
                                std::to_string(ws_bytes)
                          : "workspace too small: need " + std::to_string(need) + " bytes");
            return PF_ENOMEM;
        }
        s.ws = (char*)dev_ws;
        s.ws_bytes = ws_bytes;
        plan(s, s.ws);
        s.m.tab = s.tab;
        s.m.cell_cap = s.cell_cap;
        s.m.cell_rks = s.cell_rks;
        s.m.ads_hist = s.ads_hist;
        if (static_dev >= 0) {
            // no allocation of any kind: read-backs through the device's static
            // host buffer, the coarsest inverse in order on the caller's stream,
            // and the array cleared of the previous simulator's contents
            s.static_dev = static_dev;
            s.hbuf = static_hbuf(static_dev);
            launch_fill(s, (int64_t)(need / sizeof(double)), 0.0, (double*)s.ws);
        } else {
            // coherent: in a fusion group a kernel writes the read-backs here directly
            PF_HIP(hipHostMalloc((void**)&s.hbuf, 64 * sizeof(double), hipHostMallocCoherent));
            PF_HIP(hipStreamCreateWithFlags(&s.aux, hipStreamNonBlocking));
            PF_HIP(hipEventCreateWithFlags(&s.ev_fork, hipEventDisableTiming));
            PF_HIP(hipEventCreateWithFlags(&s.ev_join, hipEventDisableTiming));
        }
        {
            int dev = 0, lds = 0;
            PF_HIP(hipGetDevice(&dev));
            PF_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
            s.max_lds = lds;
        }
        const int64_t n = s.m.n;
        upload(s, s.poro, d->rock.poro, n * sizeof(double));
        upload(s, s.kx, d->rock.kx, n * sizeof(double));
        upload(s, s.ky, d->rock.ky, n * sizeof(double));
        upload(s, s.kz, d->rock.kz, n * sizeof(double));
        upload(s, s.perf_cell, hw.perf_cell.data(), hw.perf_cell.size() * 4);
        upload(s, s.perf_well, hw.perf_well.data(), hw.perf_well.size() * 4);
        upload(s, s.pc_cell, hw.pc_cell.data(), hw.pc_cell.size() * 4);
        upload(s, s.pc_first, hw.pc_first.data(), hw.pc_first.size() * 4);
        {
            std::vector<int32_t> pc_map((size_t)n, -1);
            for (size_t k = 0; k < hw.pc_cell.size(); ++k) pc_map[hw.pc_cell[k]] = (int32_t)k;
            upload(s, s.pc_map, pc_map.data(), n * 4);
            sync(s);
        }
        upload(s, s.wp_first, hw.wp_first.data(), hw.wp_first.size() * 4);
        upload(s, s.wp_idx, hw.wp_idx.data(), hw.wp_idx.size() * 4);
        upload(s, s.perf_depth, hw.perf_depth.data(), hw.perf_depth.size() * 8);
        upload(s, s.w_ctrl, hw.ctrl.data(), hw.ctrl.size() * 4);
        upload(s, s.w_inj, hw.inj.data(), hw.inj.size() * 4);
        upload(s, s.w_target, hw.target.data(), hw.target.size() * 8);
        upload(s, s.w_cinj, hw.cinj.data(), hw.cinj.size() * 8);
        upload(s, s.w_gamma, hw.gamma.data(), hw.gamma.size() * 8);
        upload(s, s.w_zref, hw.zref.data(), hw.zref.size() * 8);
        upload(s, s.w_scale, hw.scale.data(), hw.scale.size() * 8);
        upload(s, s.w_rw, hw.rw.data(), hw.rw.size() * 8);
        upload(s, s.w_skin, hw.skin.data(), hw.skin.size() * 8);
        upload(s, s.w_dir, hw.dir.data(), hw.dir.size() * 4);
        {
            static_assert(kTabSlots == 9, "table layout");
            std::vector<double> tab(kTabSlots * PF_TABLE_MAX, 0.0);
            const pf_polymer& pp = d->polymer;
            const pf_fluid& ff = d->fluid;
            for (int k = 0; k < PF_TABLE_MAX; ++k) {
                tab[kTabAdsC * PF_TABLE_MAX + k] = pp.ads_c[k];
                tab[kTabAdsA * PF_TABLE_MAX + k] = pp.ads_a[k];
                tab[kTabViscC * PF_TABLE_MAX + k] = pp.visc_c[k];
                tab[kTabViscM * PF_TABLE_MAX + k] = pp.visc_m[k];
                tab[kTabPcS * PF_TABLE_MAX + k] = ff.pc_s[k];
                tab[kTabPcV * PF_TABLE_MAX + k] = ff.pc_v[k];
                // the rock table is interpolated in log10 of permeability
                tab[kTabKpK * PF_TABLE_MAX + k] = k < pp.n_kperm ? std::log10(pp.kperm_k[k]) : 0.0;
                tab[kTabKpRrf * PF_TABLE_MAX + k] = pp.kperm_rrf[k];
                tab[kTabKpAdm * PF_TABLE_MAX + k] = pp.kperm_admax[k];
            }
            upload(s, s.tab, tab.data(), tab.size() * 8);
            sync(s);
        }
        if (s.m.nw > 0) upload(s, s.rscale + 3 * n, hw.scale.data(), hw.scale.size() * 8);
        launch_fill(s, s.nv, 0.0, s.x);
        // the (oil, C) entry of every Jacobian block is zero: its seven planes
        // are cleared once here and never written again (the assembly skips them)
        for (int f = 0; f < 7; ++f) launch_fill(s, n, 0.0, s.J + (int64_t)(f * 9 + 5) * n);
        launch_static(s);
        if (s.m.n_kperm > 0) launch_kperm(s);
        if (s.ads_hist) launch_fill(s, n, 0.0, s.ads_hist);
        sync(s);   // host vectors above must outlive the copies
        for (int w = 0; w < d->n_wells; ++w) s.h_wktop.push_back(d->wells[w].k_top);
        s.h_perf_cell = hw.perf_cell;
        s.h_perf_well = hw.perf_well;
        s.h_ctrl0 = hw.ctrl;
        s.h_w_ctrl = hw.ctrl;
        s.h_inj = hw.inj;
        s.h_wp_first = hw.wp_first;
        s.h_target0 = hw.target;
        s.h_target = hw.target;
        s.h_limit = hw.limit;
        s.newton_it = 0;
        s.last_upd = INFINITY;
        s.last_bnorm = 0.0;
        *out = h;
        return PF_OK;
    } catch (...) {
        side_release(s);
        if (s.hbuf && s.static_dev < 0) (void)hipHostFree(s.hbuf);
        delete h;
        throw;
    }
    PF_API_END
}

pf_status pf_create(const pf_model_desc* d, const pf_solver_opts* o, void* dev_ws, size_t ws_bytes,
                    void* hip_stream, pf_sim** out) {
    if (!dev_ws) {
        set_error("null workspace");
        return PF_EINVAL;
    }
    return create_sim(d, o, dev_ws, ws_bytes, hip_stream, -1, out);
}

pf_status pf_create_static(const pf_model_desc* d, const pf_solver_opts* o, void* hip_stream, pf_sim** out) {
    PF_API_BEGIN
    if (!out) throw InvalidArg{"null output handle"};
    int dev = 0;
    PF_HIP(hipGetDevice(&dev));
    if (hip_stream) {
        int sdev = -1;
        PF_HIP(hipStreamGetDevice((hipStream_t)hip_stream, &sdev));
        if (sdev != dev) throw InvalidArg{"the stream belongs to another device than the current one"};
    }
    void* ws = static_workspace_acquire(dev);
    if (!ws) {
        set_error("the static workspace of this device is held by another simulator (destroy it first)");
        return PF_EBUSY;
    }
    const pf_status st = create_sim(d, o, ws, kStaticWorkspaceBytes, hip_stream, dev, out);
    if (st != PF_OK) static_workspace_release(dev);
    return st;
    PF_API_END
}


static void prof_release(Sim& s) {
    for (hipEvent_t e : s.prof_ev) (void)hipEventDestroy(e);
    s.prof_ev.clear();
    s.prof_id = 0;
    s.prof_used = 0;
}

void pf_destroy(pf_sim* h) {
    if (!h) return;
    if (h->s.fu) (void)pf_fusion_leave(h);
    prof_release(h->s);
    side_release(h->s);
    if (h->s.static_dev >= 0) {
        (void)hipStreamSynchronize(h->s.stream);     // its kernels are done with the array
        static_workspace_release(h->s.static_dev);
    } else if (h->s.hbuf) {
        (void)hipHostFree(h->s.hbuf);
    }
    delete h;
}

pf_status pf_profile_begin(pf_sim* h, int32_t kernel_id, int32_t max_launches) {
    PF_API_BEGIN
    if (!h || kernel_id < PF_K_ASSEMBLE || kernel_id > PF_K_BLACK_SPMV || max_launches < 1 || max_launches > 100000)
        throw InvalidArg{"bad profiling request"};
    Sim& s = h->s;
    prof_release(s);
    s.prof_ev.resize(2 * (size_t)max_launches);
    for (auto& e : s.prof_ev) PF_HIP(hipEventCreate(&e));
    s.prof_used = 0;
    s.prof_id = kernel_id;
    return PF_OK;
    PF_API_END
}

pf_status pf_profile_end(pf_sim* h, int32_t* launches, double* total_ms) {
    PF_API_BEGIN
    if (!h) throw InvalidArg{"null argument"};
    Sim& s = h->s;
    sync(s);
    double tot = 0.0;
    for (int k = 0; k < s.prof_used; ++k) {
        float ms = 0.0f;
        PF_HIP(hipEventElapsedTime(&ms, s.prof_ev[2 * k], s.prof_ev[2 * k + 1]));
        tot += ms;
    }
    if (launches) *launches = s.prof_used;
    if (total_ms) *total_ms = tot;
    prof_release(s);
    return PF_OK;
    PF_API_END
}

pf_status pf_set_opts(pf_sim* h, const pf_solver_opts* o) {
    PF_API_BEGIN
    if (!h || !o) throw InvalidArg{"null argument"};
    Sim& s = h->s;
    if (o->restart < 1 || o->restart > s.restart_cap) throw InvalidArg{"restart exceeds the workspace plan"};
    if (o->precision != s.opts.precision) throw InvalidArg{"precision is fixed at creation"};
    if (o->max_lin_it < 1 || o->max_newton < 1 || o->max_cuts < 0) throw InvalidArg{"bad iteration limits"};
    if (o->smoother != PF_SMOOTH_BJAC && o->smoother != PF_SMOOTH_RBILU0) throw InvalidArg{"bad smoother"};
    if (o->cpr_order != PF_CPR_PF && o->cpr_order != PF_CPR_FP) throw InvalidArg{"bad CPR order"};
    s.opts = *o;
    return PF_OK;
    PF_API_END
}

pf_status pf_set_state(pf_sim* h, const double* P, const double* S, const double* C, const double* Pb) {
    PF_API_BEGIN
    if (!h || !P || !S || !C || (h->s.m.nw > 0 && !Pb)) throw InvalidArg{"null argument"};
    Sim& s = h->s;
    const int64_t n = s.m.n;
    upload(s, s.x, P, n * 8);
    upload(s, s.x + n, S, n * 8);
    upload(s, s.x + 2 * n, C, n * 8);
    if (s.m.nw > 0) upload(s, s.x + 3 * n, Pb, s.m.nw * 8);
    if (s.ads_hist) launch_fill(s, n, 0.0, s.ads_hist);
    sync(s);
    s.dt_next = s.opts.dt_init;
    set_well_controls(s, s.h_ctrl0, s.h_target0);
    return PF_OK;
    PF_API_END
}

pf_status pf_set_equilibrium_state(pf_sim* h, double datum_depth, double datum_pressure, double fwl_depth) {
    PF_API_BEGIN
    if (!h) throw InvalidArg{"null argument"};
    if (!std::isfinite(datum_depth) || !std::isfinite(datum_pressure) || !std::isfinite(fwl_depth))
        throw InvalidArg{"non-finite datum or free-water level"};
    Sim& s = h->s;
    {
        // the capillary-pressure table must decrease strictly to be inverted
        std::vector<double> tab(kTabSlots * PF_TABLE_MAX);
        PF_HIP(hipMemcpyAsync(tab.data(), s.tab, tab.size() * 8, hipMemcpyDeviceToHost, s.stream));
        sync(s);
        for (int k = 1; k < s.m.n_pc; ++k)
            if (!(tab[kTabPcV * PF_TABLE_MAX + k] < tab[kTabPcV * PF_TABLE_MAX + k - 1]))
                throw InvalidArg{"equilibrium initialisation needs a strictly decreasing capillary-pressure table"};
    }
    launch_equilibrium(s, datum_depth, datum_pressure, fwl_depth);
    if (s.ads_hist) launch_fill(s, s.m.n, 0.0, s.ads_hist);
    sync(s);
    s.dt_next = s.opts.dt_init;
    set_well_controls(s, s.h_ctrl0, s.h_target0);
    return PF_OK;
    PF_API_END
}

pf_status pf_get_state(pf_sim* h, double* P, double* S, double* C, double* Pb) {
    PF_API_BEGIN
    if (!h) throw InvalidArg{"null argument"};
    Sim& s = h->s;
    const int64_t n = s.m.n;
    if (P) PF_HIP(hipMemcpyAsync(P, s.x, n * 8, hipMemcpyDeviceToHost, s.stream));
    if (S) PF_HIP(hipMemcpyAsync(S, s.x + n, n * 8, hipMemcpyDeviceToHost, s.stream));
    if (C) PF_HIP(hipMemcpyAsync(C, s.x + 2 * n, n * 8, hipMemcpyDeviceToHost, s.stream));
    if (Pb && s.m.nw > 0) PF_HIP(hipMemcpyAsync(Pb, s.x + 3 * n, s.m.nw * 8, hipMemcpyDeviceToHost, s.stream));
    sync(s);
    return PF_OK;
    PF_API_END
}

pf_status pf_well_status(pf_sim* h, int32_t* ctrl, double* target, double* qw, double* qo) {
    PF_API_BEGIN
    if (!h) throw InvalidArg{"null argument"};
    Sim& s = h->s;
    const int nw = s.m.nw;
    std::vector<double> rw, ro;
    well_rates(s, rw, ro);
    for (int w = 0; w < nw; ++w) {
        if (ctrl) ctrl[w] = s.h_w_ctrl[w];
        if (target) target[w] = s.h_target[w];
        if (qw) qw[w] = rw[w];
        if (qo) qo[w] = ro[w];
    }
    return PF_OK;
    PF_API_END
}

pf_status pf_set_well_operation(pf_sim* h, int32_t w, int32_t control, double target, double c_inj,
                                double bhp_limit) {
    PF_API_BEGIN
    if (!h) throw InvalidArg{"null argument"};
    Sim& s = h->s;
    if (w < 0 || w >= s.m.nw) throw InvalidArg{"bad well index"};
    if (control < PF_CTRL_BHP || control > PF_CTRL_LRATE) throw InvalidArg{"bad well control"};
    if (control != PF_CTRL_BHP && target == 0.0) throw InvalidArg{"rate target must be non-zero"};
    if (!(c_inj >= 0.0) || !(bhp_limit >= 0.0) || !std::isfinite(bhp_limit)) throw InvalidArg{"bad c_inj or bhp_limit"};
    s.h_ctrl0[w] = control;
    s.h_target0[w] = target;
    s.h_limit[w] = bhp_limit;
    std::vector<int32_t> ctrl = s.h_w_ctrl;
    std::vector<double> tgt = s.h_target;
    ctrl[w] = control;
    tgt[w] = target;
    const double ci = c_inj;
    upload(s, s.w_cinj + w, &ci, 8);
    set_well_controls(s, ctrl, tgt);     // synchronises: ci outlives its copy
    return PF_OK;
    PF_API_END
}

pf_status pf_begin_step(pf_sim* h) {
    PF_API_BEGIN
    if (!h) throw InvalidArg{"null argument"};
    begin_step(h->s);
    return PF_OK;
    PF_API_END
}

pf_status pf_newton_iteration(pf_sim* h, double dt, pf_step_stats* st) {
    PF_API_BEGIN
    if (!h || !(dt > 0)) throw InvalidArg{"bad argument"};
    if (st) std::memset(st, 0, sizeof(*st));
    const NewtonState r = newton_iteration(h->s, dt, st);
    if (r == NewtonState::Failed) {
        set_error("Newton iteration failed (non-finite values or iteration limit)");
        return PF_ENONCONV;
    }
    return PF_OK;
    PF_API_END
}

pf_status pf_step(pf_sim* h, double dt, pf_step_stats* st) {
    PF_API_BEGIN
    if (!h || !(dt > 0)) throw InvalidArg{"bad argument"};
    Sim& s = h->s;
    pf_step_stats local;
    std::memset(&local, 0, sizeof(local));
    const double t0 = now_s();
    double remaining = dt;
    double dt_try = (s.dt_next > 0.0) ? std::min(s.dt_next, dt) : dt;
    int cuts = 0;
    while (remaining > 1e-9 * dt) {
        dt_try = std::min(dt_try, remaining);
        begin_step(s);
        NewtonState r = NewtonState::Continue;
        local.converged = 0;
        while (r == NewtonState::Continue) r = newton_iteration(s, dt_try, &local);
        if (r == NewtonState::Failed) {
            launch_copy(s, s.nv, s.xn, s.x);
            ++cuts;
            if (cuts > s.opts.max_cuts) {
                sync(s);
                local.cuts = cuts;
                local.t_total = now_s() - t0;
                if (st) *st = local;
                set_error("Newton failed after the maximum number of timestep cuts");
                return PF_ENONCONV;
            }
            dt_try *= 0.5;
            continue;
        }
        remaining -= dt_try;
        local.dt_taken += dt_try;
        dt_try = std::min(2.0 * dt_try, dt);
        local.well_switches += apply_well_limits(s);
    }
    s.dt_next = dt_try;
    sync(s);
    local.cuts = cuts;
    local.converged = 1;
    local.t_total = now_s() - t0;
    if (st) *st = local;
    return PF_OK;
    PF_API_END
}

pf_status pf_assemble(pf_sim* h, double dt, double* R, double* J, double* border) {
    PF_API_BEGIN
    if (!h || !R || !(dt > 0)) throw InvalidArg{"bad argument"};
    Sim& s = h->s;
    launch_assemble(s, dt, true);
    const int64_t n = s.m.n, np = s.m.np;
    PF_HIP(hipMemcpyAsync(R, s.R, s.nv * 8, hipMemcpyDeviceToHost, s.stream));
    if (J) {
        ensure_j_natural(s);
        PF_HIP(hipMemcpyAsync(J, s.J, 63 * n * 8, hipMemcpyDeviceToHost, s.stream));
    }
    if (border && np > 0) {
        std::vector<double> Bh(3 * np), Ch(3 * np), Dh(std::max(s.m.nw, 1));
        PF_HIP(hipMemcpyAsync(Bh.data(), s.B, 3 * np * 8, hipMemcpyDeviceToHost, s.stream));
        PF_HIP(hipMemcpyAsync(Ch.data(), s.Cw, 3 * np * 8, hipMemcpyDeviceToHost, s.stream));
        PF_HIP(hipMemcpyAsync(Dh.data(), s.Dw, s.m.nw * 8, hipMemcpyDeviceToHost, s.stream));
        sync(s);
        for (int64_t k = 0; k < np; ++k) {
            for (int e = 0; e < 3; ++e) border[7 * k + e] = Bh[3 * k + e];
            for (int e = 0; e < 3; ++e) border[7 * k + 3 + e] = Ch[3 * k + e];
            border[7 * k + 6] = Dh[s.h_perf_well[k]];
        }
    }
    sync(s);
    return PF_OK;
    PF_API_END
}

pf_status pf_spmv(pf_sim* h, const double* x, double* y) {
    PF_API_BEGIN
    if (!h || !x || !y) throw InvalidArg{"null argument"};
    Sim& s = h->s;
    upload(s, s.t1, x, s.nv * 8);
    launch_spmv(s, s.t1, s.t2);
    PF_HIP(hipMemcpyAsync(y, s.t2, s.nv * 8, hipMemcpyDeviceToHost, s.stream));
    sync(s);
    return PF_OK;
    PF_API_END
}

pf_status pf_linear_solve(pf_sim* h, const double* b, double rtol, double* dx, int32_t* iters, double* rel) {
    PF_API_BEGIN
    if (!h || !b || !dx) throw InvalidArg{"null argument"};
    Sim& s = h->s;
    upload(s, s.rhs, b, s.nv * 8);
    cpr_setup(s);
    double r = 0.0;
    const int its = fgmres(s, s.rhs, rtol, s.dx, &r, s.opts.max_lin_it);
    PF_HIP(hipMemcpyAsync(dx, s.dx, s.nv * 8, hipMemcpyDeviceToHost, s.stream));
    sync(s);
    if (iters) *iters = its;
    if (rel) *rel = r;
    return PF_OK;
    PF_API_END
}

pf_status pf_get_static(pf_sim* h, double* row_scale, double* Tx, double* Ty, double* Tz, double* PVr,
                        int32_t* perf_well, int32_t* perf_cell, double* perf_wi) {
    PF_API_BEGIN
    if (!h) throw InvalidArg{"null argument"};
    Sim& s = h->s;
    const int64_t n = s.m.n, np = s.m.np;
    if (row_scale) PF_HIP(hipMemcpyAsync(row_scale, s.rscale, s.nv * 8, hipMemcpyDeviceToHost, s.stream));
    if (Tx) PF_HIP(hipMemcpyAsync(Tx, s.Tx, n * 8, hipMemcpyDeviceToHost, s.stream));
    if (Ty) PF_HIP(hipMemcpyAsync(Ty, s.Ty, n * 8, hipMemcpyDeviceToHost, s.stream));
    if (Tz) PF_HIP(hipMemcpyAsync(Tz, s.Tz, n * 8, hipMemcpyDeviceToHost, s.stream));
    if (PVr) PF_HIP(hipMemcpyAsync(PVr, s.pvr, n * 8, hipMemcpyDeviceToHost, s.stream));
    if (perf_wi && np > 0) PF_HIP(hipMemcpyAsync(perf_wi, s.perf_wi, np * 8, hipMemcpyDeviceToHost, s.stream));
    sync(s);
    if (perf_well) std::copy(s.h_perf_well.begin(), s.h_perf_well.end(), perf_well);
    if (perf_cell) std::copy(s.h_perf_cell.begin(), s.h_perf_cell.end(), perf_cell);
    return PF_OK;
    PF_API_END
}

int64_t pf_n_perf(const pf_sim* h) { return h ? h->s.m.np : 0; }

int32_t pf_pressure_level(pf_sim* h, int32_t level, int32_t* dims, double* A) {
    if (!h) return 0;
    Sim& s = h->s;
    const int nl = (int)s.mg.size();
    if (level < 0 || level >= nl) return nl;
    const MGLevel& L = s.mg[level];
    if (dims) { dims[0] = L.nx; dims[1] = L.ny; dims[2] = L.nz; }
    if (A) {
        try {
            std::vector<double> slots((size_t)(7 * L.ns));
            if (hipMemcpyAsync(slots.data(), L.A, 7 * L.ns * 8, hipMemcpyDeviceToHost, s.stream) != hipSuccess ||
                hipStreamSynchronize(s.stream) != hipSuccess)
                return -1;
            for_level_cells(L, [&](int64_t i, int64_t j) {
                for (int d = 0; d < 7; ++d) A[d * L.n + i] = slots[d * L.ns + j];
            });
        } catch (...) {
            return -1;
        }
    }
    return nl;
}

pf_status pf_pressure_smooth(pf_sim* h, int32_t level, int32_t colour, int32_t zero_init, const double* b,
                             double* x) {
    PF_API_BEGIN
    if (!h || !b || !x) throw InvalidArg{"null argument"};
    Sim& s = h->s;
    if (level < 0 || level + 1 >= (int)s.mg.size() || (colour != 0 && colour != 1))
        throw InvalidArg{"level must be a smoothed level and colour 0 or 1"};
    MGLevel& L = s.mg[level];
    // natural order <-> the level's slots (absent-cell slots are zero)
    std::vector<double> bs((size_t)L.ns, 0.0), xs((size_t)L.ns, 0.0);
    for_level_cells(L, [&](int64_t i, int64_t j) { bs[j] = b[i]; xs[j] = x[i]; });
    upload(s, L.b, bs.data(), L.ns * 8);
    upload(s, L.x, xs.data(), L.ns * 8);
    mg_smooth_once(s, level, colour, zero_init);
    PF_HIP(hipMemcpyAsync(xs.data(), L.x, L.ns * 8, hipMemcpyDeviceToHost, s.stream));
    sync(s);
    for_level_cells(L, [&](int64_t i, int64_t j) { x[i] = xs[j]; });
    return PF_OK;
    PF_API_END
}

pf_status pf_smoother_apply(pf_sim* h, const double* f, double* z) {
    PF_API_BEGIN
    if (!h || !f || !z) throw InvalidArg{"null argument"};
    Sim& s = h->s;
    if (s.mg.empty()) throw InvalidArg{"no preconditioner set up"};
    upload(s, s.t2, f, s.nv * 8);
    smoother_once(s, s.t2);
    if (s.opts.precision == PF_PREC_MIXED) {
        std::vector<float> z32((size_t)s.nv);
        PF_HIP(hipMemcpyAsync(z32.data(), s.Z32, s.nv * 4, hipMemcpyDeviceToHost, s.stream));
        sync(s);
        for (int64_t i = 0; i < s.nv; ++i) z[i] = z32[i];
    } else {
        PF_HIP(hipMemcpyAsync(z, s.t1, s.nv * 8, hipMemcpyDeviceToHost, s.stream));
        sync(s);
    }
    return PF_OK;
    PF_API_END
}

pf_status pf_precond_apply(pf_sim* h, const double* v, double* z, double* w) {
    PF_API_BEGIN
    if (!h || !v || !z) throw InvalidArg{"null argument"};
    Sim& s = h->s;
    if (s.mg.empty()) throw InvalidArg{"no preconditioner set up"};
    // the first two Krylov columns serve as v and w
    double* vd = s.V;
    double* wd = s.V + s.kst;
    if (s.Z32) {
        upload(s, vd, v, s.nv * 8);
        cpr_apply(s, vd, s.Z32);
        launch_spmv(s, s.Z32, wd);
        std::vector<float> z32((size_t)s.nv);
        PF_HIP(hipMemcpyAsync(z32.data(), s.Z32, s.nv * 4, hipMemcpyDeviceToHost, s.stream));
        sync(s);
        for (int64_t i = 0; i < s.nv; ++i) z[i] = z32[i];
        if (w) PF_HIP(hipMemcpyAsync(w, wd, s.nv * 8, hipMemcpyDeviceToHost, s.stream));
    } else if (cpr_colour_split(s)) {
        // the solver's layout: v in, z and w out through the colour-split one
        upload(s, s.t1, v, s.nv * 8);
        launch_to_cs(s, s.t1, vd);
        cpr_apply_spmv(s, vd, s.Z, wd);
        launch_from_cs(s, s.Z, s.t1);
        launch_from_cs(s, wd, s.t2);
        PF_HIP(hipMemcpyAsync(z, s.t1, s.nv * 8, hipMemcpyDeviceToHost, s.stream));
        if (w) PF_HIP(hipMemcpyAsync(w, s.t2, s.nv * 8, hipMemcpyDeviceToHost, s.stream));
    } else {
        upload(s, vd, v, s.nv * 8);
        cpr_apply_spmv(s, vd, s.Z, wd);
        PF_HIP(hipMemcpyAsync(z, s.Z, s.nv * 8, hipMemcpyDeviceToHost, s.stream));
        if (w) PF_HIP(hipMemcpyAsync(w, wd, s.nv * 8, hipMemcpyDeviceToHost, s.stream));
    }
    sync(s);
    return PF_OK;
    PF_API_END
}

pf_status pf_pressure_vcycle(pf_sim* h, const double* b, double* x) {
    PF_API_BEGIN
    if (!h || !b || !x) throw InvalidArg{"null argument"};
    Sim& s = h->s;
    if (s.mg.empty()) throw InvalidArg{"no multigrid hierarchy"};
    const int64_t n = s.m.n;
    // v = (b, 0, ...): Pi_r v = b on the cells
    std::vector<double> v((size_t)s.nv, 0.0);
    std::copy(b, b + n, v.begin());
    upload(s, s.t2, v.data(), s.nv * 8);
    mg_cycles_once(s, s.t2);
    if (s.opts.precision == PF_PREC_MIXED) {
        std::vector<float> p32((size_t)n);
        PF_HIP(hipMemcpyAsync(p32.data(), s.pnat32, n * 4, hipMemcpyDeviceToHost, s.stream));
        sync(s);
        for (int64_t i = 0; i < n; ++i) x[i] = p32[i];
    } else {
        PF_HIP(hipMemcpyAsync(x, s.pnat, n * 8, hipMemcpyDeviceToHost, s.stream));
        sync(s);
    }
    return PF_OK;
    PF_API_END
}

}  // extern "C"
