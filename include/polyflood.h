/*
 * polyflood.h - C ABI of the MI355X (gfx950) HIP library for the Newton
 * iteration of a fully implicit water / oil / polymer reservoir simulator
 * (after Zhong et al., "Numerical simulations of polymer flooding process in
 * porous media on distributed-memory parallel computers", arXiv 1807.05298).
 *
 * One Newton iteration (Sec. 3.3, Algorithm 1) = assemble the backward-Euler
 * residual (Sec. 3.1) of water, oil and polymer mass conservation (Sec. 2)
 * with upstream-weighted finite-volume fluxes (Sec. 3.2) and Peaceman wells
 * (Sec. 2.4), plus its 3x3-block Jacobian (7-point stencil + well border,
 * block-wise ordering of Sec. 3.4); then solve J dx = -R with restarted
 * flexible GMRES under the two-stage CPR preconditioner (Sec. 3.4,
 * Algorithm 2: a pressure-block stage solved by multigrid and a full-system
 * block smoother); then update the state.
 *
 * Conventions (every entry point):
 *   - Units are SI: m, m^2, Pa, Pa*s, kg/m^3, s.  Well rate targets are
 *     surface volume rates (mass / reference density, m^3/s), positive into
 *     the reservoir.
 *   - Cells are in natural order i = ix + nx*(iy + ny*iz), x fastest,
 *     iz = 0 at the top; depth grows with iz.
 *   - Host arrays passed in are read during the call and never retained.
 *   - Device memory: exactly one caller-owned workspace of
 *     pf_workspace_size() bytes (any device allocation, 256-byte aligned),
 *     which must outlive the simulator.  A simulator allocates no device
 *     memory of its own, only a few KB of pinned host memory for scalar
 *     read-backs; a fusion group (pf_fusion_*) allocates its merged
 *     launches' argument tables (device and pinned host memory, grown as
 *     needed: tens to hundreds of KB).
 *   - All device work is ordered on the caller's HIP stream (a hipStream_t
 *     passed as void*, e.g. torch.cuda.current_stream().cuda_stream).  Calls
 *     that return host data synchronise that stream.  Internally a simulator
 *     also owns one side stream (default priority) for the coarsest-level
 *     inversion of the preconditioner set-up, forked from and joined back
 *     into the caller's stream by events within each set-up, so the
 *     caller's stream still orders everything the simulator does (a member
 *     of a fusion group uses the group's stream alone).
 *   - A pf_sim is not thread-safe; distinct sims are independent.
 *   - Errors are returned as pf_status; pf_last_error() gives a message
 *     (thread-local).  No C++ exception crosses the ABI.
 *
 * Residual scaling.  The library works on the row-scaled system
 *   R~ = D R,  J~ = D J,
 * where for cell i the water row is divided by rho_w0*PVr_i, the oil row by
 * rho_o0*PVr_i and the polymer row by C_ref*PVr_i (PVr_i = phi_r,i * V_i,
 * C_ref = max(largest injection concentration, 1 kg/m^3)), a rate-controlled
 * well row by |target| and a BHP row by 1e5 Pa.  Row scaling changes neither
 * the root nor the Newton step; it makes the residual dimensionless (pore
 * volumes per step), which is what the convergence test and the Krylov
 * norms measure.  pf_get_static() returns D.
 */
#ifndef POLYFLOOD_H
#define POLYFLOOD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PF_OK = 0,
    PF_EINVAL = 1,      /* bad argument or model description */
    PF_ENOMEM = 2,      /* workspace smaller than pf_workspace_size() */
    PF_ENONCONV = 3,    /* Newton failed after the maximum number of cuts; state rolled back */
    PF_ELINEAR = 4,     /* linear solver breakdown (non-finite values) */
    PF_EHIP = 5,        /* a HIP runtime call failed */
    PF_EBUSY = 6        /* serving: no free slot / budget */
} pf_status;

enum { PF_CTRL_BHP = 0, PF_CTRL_WRATE = 1, PF_CTRL_ORATE = 2, PF_CTRL_LRATE = 3 };
/* Well direction: vertical (z) or horizontal along x. */
enum { PF_WELL_Z = 0, PF_WELL_X = 1 };
enum { PF_PREC_FP64 = 0, PF_PREC_MIXED = 1 };
enum { PF_CPR_PF = 0, PF_CPR_FP = 1 };
enum { PF_SMOOTH_BJAC = 0, PF_SMOOTH_RBILU0 = 1 };

/* Grid (Sec. 3 item 2): structured, uniform block sizes; top_depth is the
 * depth of the top face of layer 0. */
typedef struct { int32_t nx, ny, nz; double dx, dy, dz, top_depth; } pf_grid;

/* Rock (Sec. 2.1): reference porosity and diagonal permeability per cell
 * (host arrays of N values, m^2); phi(P) = phi_r + cr*(P - p_ref). */
typedef struct { const double *poro, *kx, *ky, *kz; double cr, p_ref; } pf_rock;

/* Tables (PF_TABLE_MAX points, abscissae strictly increasing) are
 * interpolated linearly between points and held constant outside them. */
#define PF_TABLE_MAX 16

/* Fluids (Sec. 2.2): reference densities, compressibilities (1/Pa) with
 * rho = rho0*exp(c*(P - p_ref)); constant viscosities; Corey relative
 * permeabilities krw = krw0*Sn^n_w, kro = kro0*(1-Sn)^n_o with
 * Sn = (S - swc)/(1 - swc - sor) clamped to [0,1]; gravity (m/s^2).
 * Capillary pressure P_c(S) = P_o - P_w (Sec. 2.2) from the table
 * (pc_s[k], pc_v[k] in Pa) of n_pc points, 0 when n_pc = 0; it enters the
 * water potential of every face flux (the unknown P is the oil pressure). */
typedef struct {
    double rho_w0, rho_o0, c_w, c_o, mu_w, mu_o, swc, sor, n_w, n_o, krw0, kro0, gravity;
    int32_t n_pc, reserved;
    double pc_s[PF_TABLE_MAX], pc_v[PF_TABLE_MAX];
} pf_fluid;

/* Polymer (Sec. 2.3).  Fully mixed viscosity mu_m(C) by mix_rule:
 * PF_MIX_POLY mu_w*(1 + a1*C + a2*C^2); PF_MIX_LINEAR beta*mu_p_ref +
 * (1 - beta)*mu_w and PF_MIX_EXP mu_p_ref^beta * mu_w^(1 - beta), beta =
 * C/c_max (the paper's linear and nonlinear mixing rules); PF_MIX_TABLE
 * mu_w times the multiplier table (visc_c, visc_m) of n_visc points.
 * mu_p_ref (Pa s) is the viscosity at c_max (0: mu_m(c_max)).
 * Todd-Longstaff omega with mu_p^ref and alpha = C/c_max.  Adsorption
 * (kg per m^3 rock): Langmuir ads_max*ads_b*C/(1 + ads_b*C) when n_ads = 0,
 * else the table (ads_c, ads_a) of n_ads points; R_k = 1 + (rrf - 1)*A/
 * ads_max; inaccessible pore-volume fraction ipv.
 * Retention (Sec. 2.3: desorption only above a residual sorption level):
 * a cell keeps ads_res (in [0, 1]) times the largest equilibrium adsorption
 * of its converged states, A = max(A_eq(C), ads_res * A_hist); 0 is
 * equilibrium sorption, 1 no desorption.  A_hist is taken in at the start of
 * every timestep (pf_begin_step) and cleared by pf_set_state.
 * RRF and A_d,max against rock permeability (Sec. 2.3): with n_kperm > 0
 * points (kperm_k in m^2, increasing; kperm_rrf >= 1; kperm_admax > 0 in kg
 * per m^3 rock), each cell's values are the table interpolated linearly in
 * log10 of its kx (end values held outside); its equilibrium isotherm is
 * scaled by A_d,max / ads_max and R_k = 1 + (RRF - 1)*A/A_d,max. */
enum { PF_MIX_POLY = 0, PF_MIX_LINEAR = 1, PF_MIX_EXP = 2, PF_MIX_TABLE = 3 };
typedef struct {
    double a1, a2, omega, c_max, ads_max, ads_b, rrf, ipv;
    int32_t mix_rule, n_ads;
    double mu_p_ref;
    int32_t n_visc, reserved;
    double ads_c[PF_TABLE_MAX], ads_a[PF_TABLE_MAX], visc_c[PF_TABLE_MAX], visc_m[PF_TABLE_MAX];
    double ads_res;
    int32_t n_kperm, reserved2;
    double kperm_k[PF_TABLE_MAX], kperm_rrf[PF_TABLE_MAX], kperm_admax[PF_TABLE_MAX];
} pf_polymer;

/* A well (Sec. 2.4).  direction PF_WELL_Z: vertical at column (ix, iy),
 * perforated in layers k_top..k_bot.  PF_WELL_X: horizontal along x in row
 * iy of layer k_top (= k_bot), perforated in cells ix..ix_last; its Peaceman
 * index is eq:wi:re:k as printed (permeabilities ky, kz and block sizes dy,
 * dz across the well, h = dx along it), a vertical well's the same formula
 * with (y, z) replaced by (x, y) and h = dz.  control is PF_CTRL_*; target
 * in Pa (BHP) or m^3/s (rates,
 * positive into the reservoir); c_inj the injected polymer concentration
 * (kg/m^3); rw the wellbore radius; skin the skin factor.  The bottom-hole
 * pressure refers to the depth of the top perforation; the wellbore unit
 * weight is rho_w0*g for injectors and rho_o0*g for producers.
 * bhp_limit (Pa, 0: none) bounds a rate-controlled well's bottom-hole
 * pressure: at most bhp_limit for an injector, at least bhp_limit for a
 * producer (the multi-constraint injector of Sec. 4.1.2).  Well operations are
 * fixed within a timestep (Sec. 3 item 4): after each converged sub-step a
 * rate-controlled well beyond its limit continues at the limiting BHP, and
 * a well held at its limit returns to its rate target once it could
 * deliver more than that target at the limit. */
typedef struct {
    int32_t ix, iy, k_top, k_bot, is_injector, control;
    double target, c_inj, rw, skin;
    double bhp_limit;
    int32_t direction, ix_last;
} pf_well;

typedef struct {
    pf_grid grid;
    pf_rock rock;
    pf_fluid fluid;
    pf_polymer polymer;
    int32_t n_wells;
    const pf_well* wells;
} pf_model_desc;

/* Solver options (Sec. 3 items 4-6).  pf_default_opts() fills them. */
typedef struct {
    int32_t precision;     /* PF_PREC_FP64 | PF_PREC_MIXED (FP32/BF16 preconditioner) */
    int32_t cpr_order;     /* PF_CPR_PF (pressure stage first) | PF_CPR_FP (Algorithm 2 order) */
    int32_t smoother;      /* PF_SMOOTH_BJAC | PF_SMOOTH_RBILU0 (second CPR stage) */
    int32_t restart;       /* FGMRES restart length m (1..64) */
    int32_t max_lin_it;    /* total FGMRES iterations per Newton iteration */
    int32_t max_newton;    /* Newton iterations before a timestep cut */
    int32_t max_cuts;      /* cuts per scheduled step before PF_ENONCONV */
    int32_t inexact;       /* 1: forcing term of eq. fterm (third choice); 0: fixed lin_tol */
    double tol_res;        /* converged when max|R~| <= tol_res ... */
    double tol_upd;        /* ... and the last scaled update max-norm <= tol_upd */
    double lin_tol;        /* relative FGMRES tolerance when inexact == 0 */
    double ds_max;         /* Newton chop: |dS| <= ds_max per cell */
    int32_t mg_pre;        /* multigrid pre-smoothing sweeps (z-line GS, colour 0 then 1; >= 1) */
    int32_t mg_post;       /* multigrid post-smoothing sweeps (colour 1 then 0; 0: prolongation only) */
    int32_t mg_coarse;     /* coarsest-level cell limit */
    int32_t reorth;        /* 1: always re-orthogonalise (CGS2); 0: when a CGS pass removed more than
                              90 % of the vector's norm */
    int32_t mg_cycles;     /* V-cycles per pressure-stage application (1..8) */
    int32_t zline_len;     /* layers per z-line smoother segment (0: by level size; at most 64 segments) */
    int32_t mg_pre_small;  /* pre-smoothing sweeps on levels of at most max(mg_small_cells, n0 / 32)
                              cells (n0: cells of the finest level), when n0 is at least
                              10 mg_small_cells (0: 5) */
    int32_t mg_small_cells;/* (0: 50000) */
    double dt_init;        /* first sub-step length (s) after pf_set_state; 0: the scheduled step */
} pf_solver_opts;

typedef struct {
    int32_t newton_its;    /* Newton iterations taken (this step / iteration) */
    int32_t lin_its;       /* FGMRES iterations summed over them */
    int32_t cuts;          /* timestep cuts */
    int32_t converged;     /* 1 when the Newton loop met both tolerances */
    double dt_taken;       /* sum of the sub-steps actually taken (s) */
    double res_norm;       /* final max|R~| */
    double upd_norm;       /* final scaled update max-norm */
    double lin_rel;        /* last achieved relative linear residual */
    double t_assemble, t_setup, t_solve, t_total;   /* host wall seconds */
    int32_t well_switches; /* control switches at BHP limits after this step's sub-steps */
    int32_t reserved;
} pf_step_stats;

struct pf_sim;
typedef struct pf_sim pf_sim;

/* Defaults: FP64; PF order; red-black block ILU(0) second stage; FGMRES(30),
 * at most 200 iterations per Newton iteration, forcing term on; 12 Newton
 * iterations and 5 cuts per step; tol_res 1e-6, tol_upd 1e-3; chop 0.2;
 * pressure multigrid of 2 V-cycles, each with 1 pre-smoothing sweep (5 on
 * levels of at most max(50,000, n0 / 32) cells of grids of n0 >= 500,000
 * cells) and none
 * after, coarsest level <= 96 cells, z-line segments chosen by level size;
 * re-orthogonalisation only on cancellation; dt_init 0. */
void pf_default_opts(pf_solver_opts* opts);

/* Bytes of device workspace a simulator of this model needs (its HBM
 * footprint). */
pf_status pf_workspace_size(const pf_model_desc* model, const pf_solver_opts* opts, size_t* bytes);

/* Create a simulator: copies the model into the workspace, runs the static
 * set-up kernels (transmissibilities, pore volumes, Peaceman indices; Sec.
 * 2.4 eq:wi, Sec. 3.2 interface averaging).  The state is undefined until
 * pf_set_state(). */
pf_status pf_create(const pf_model_desc* model, const pf_solver_opts* opts,
                    void* dev_workspace, size_t workspace_bytes, void* hip_stream, pf_sim** out);
void pf_destroy(pf_sim* sim);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc: tight serving loops, harnesses that forbid allocation, set-up
 * ahead of HIP graph capture): pf_create with the workspace taken from a
 * fixed 64 MiB array that the library holds on every GPU it runs on until
 * the process ends (PF_STATIC_WORKSPACE_BYTES; about 20,000 cells in FP64
 * with restart 30 - pf_workspace_size tells).  It allocates no device or
 * pinned host memory and creates no stream or event: read-backs go through
 * a static host buffer of the device and the coarsest-level inversion runs
 * in order on the caller's stream (the same arithmetic, so the results are
 * those of pf_create).  The array is cleared of the previous simulator's
 * contents at creation.  One simulator per GPU may hold the array at a time:
 * a second call while one lives returns PF_EBUSY (pf_destroy frees it); calls
 * that overlap on one GPU from other threads race for it.  hip_stream must
 * belong to the current device (NULL: its null stream).  Errors: PF_ENOMEM
 * when the model's footprint exceeds the array, PF_EBUSY, PF_EINVAL and
 * PF_EHIP as for pf_create. */
#define PF_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
pf_status pf_create_static(const pf_model_desc* model, const pf_solver_opts* opts, void* hip_stream,
                           pf_sim** out);

/* Replace the solver options (same workspace; precision/smoother/restart
 * may not grow beyond what the workspace was sized for). */
pf_status pf_set_opts(pf_sim* sim, const pf_solver_opts* opts);

/* Initial state (Sec. 3, solution flowchart item 3: the simulator starts
 * from the given pressure, saturation and concentration of every block) and
 * the current state, as host arrays: P (oil pressure, Pa), S (water
 * saturation), C (polymer concentration, kg/m^3) of N cells in natural
 * order and Pb (bottom-hole pressure at each well's datum, Pa) of n_wells
 * wells.  pf_set_state copies them in, resets the well controls to those of
 * the model and the next sub-step length to opts.dt_init; pf_get_state
 * synchronises the stream and copies the state out (any pointer may be
 * NULL).  Errors: PF_EINVAL for a null simulator or (set) a missing array. */
pf_status pf_set_state(pf_sim* sim, const double* P, const double* S, const double* C, const double* Pb);
pf_status pf_get_state(pf_sim* sim, double* P, double* S, double* C, double* Pb);

/* Initial state in capillary-gravity equilibrium (Sec. 4.1.3), computed on
 * the device: the oil pressure is marched from the datum (datum_depth, m;
 * datum_pressure, Pa, the oil pressure there) to every layer centre and to
 * the free-water level fwl_depth (m), where the water pressure equals it;
 * the water pressure is marched from there with its density taken at the
 * cell pressure unknown, as the fluxes take it.  Marching: classical
 * fourth-order Runge-Kutta in equal steps of at most 0.25 m, the density
 * recomputed at every stage.  The saturation balances P_o - P_w on the
 * capillary-pressure table, which must then decrease strictly (without a
 * table: S_wc above the free-water level, 1 - S_or below); the cell pressure
 * is P_o where the oil phase is continuous (P_o - P_w above the table's last
 * value) and P_w + P_c(S) below; C = 0; wells start at their BHP target or,
 * rate-controlled, at the pressure of their datum layer.  Then as
 * pf_set_state.  Errors: PF_EINVAL for a table that does not decrease. */
pf_status pf_set_equilibrium_state(pf_sim* sim, double datum_depth, double datum_pressure, double fwl_depth);

/* Start a timestep: snapshot the current state as x^n and its accumulation
 * M^n (Sec. 3.1).  pf_step() calls it itself. */
pf_status pf_begin_step(pf_sim* sim);

/* One Newton iteration of the step begun by pf_begin_step with step length
 * dt: assemble, test convergence, and (if not converged) CPR-FGMRES solve and
 * update.  st->converged reports whether the state already met the
 * tolerances (then nothing was updated). */
pf_status pf_newton_iteration(pf_sim* sim, double dt, pf_step_stats* st);

/* Advance one scheduled step of length dt (s) with Newton and the timestep
 * rules of Sec. 3 item 4: sub-steps start from the length remembered from
 * the previous step (or opts.dt_init after pf_set_state), are halved and
 * retried on Newton failure (rolling back; at most max_cuts times per
 * scheduled step) and doubled after each success, never beyond dt.  On
 * PF_ENONCONV the state is x^n of the failing sub-step. */
pf_status pf_step(pf_sim* sim, double dt, pf_step_stats* st);

/* Test hooks.  pf_assemble evaluates R~ and J~ at the current state against
 * the M^n of the last pf_begin_step.  R: 3N + n_wells values (P-, S-, C-
 * equation planes of N, then wells).  J (nullable): 63*N values, J[(d*9 +
 * e)*N + i] with d in {0: own cell, 1: -x, 2: +x, 3: -y, 4: +y, 5: -z, 6: +z}
 * and e = 3*row + col, rows (water, oil, polymer), cols (P, S, C); blocks of
 * missing neighbours are zero.  border (nullable): 7*n_perf values: per
 * perforation (in the order of pf_get_static's perf arrays) B[3] =
 * dR~_cell/dPb, C[3] = dW~/dx_cell, then dW~/dPb of its well. */
pf_status pf_assemble(pf_sim* sim, double dt, double* R, double* J, double* border);

/* y = J~ x for the last assembled system (x, y host vectors of 3N+n_wells
 * in the plane layout above). */
pf_status pf_spmv(pf_sim* sim, const double* x, double* y);

/* Solve J~ dx = b for the last assembled system with CPR-FGMRES to relative
 * tolerance rtol (b, dx host; plane layout).  *iters receives the FGMRES
 * iteration count, *rel the achieved relative residual. */
pf_status pf_linear_solve(pf_sim* sim, const double* b, double rtol, double* dx,
                          int32_t* iters, double* rel);

/* Pressure multigrid test hooks (valid after pf_linear_solve or a Newton
 * iteration has set the preconditioner up).  pf_pressure_level returns the
 * number of levels; for level < levels it writes dims[3] = (nx, ny, nz) and,
 * if A is non-NULL, the 7 coefficient planes of that level's operator
 * (diag, -x, +x, -y, +y, -z, +z; n_level values each).
 * pf_pressure_smooth applies one z-line Gauss-Seidel half-sweep on a level
 * (not the coarsest) to the columns of one colour ((ix + iy) % 2 == colour):
 * x (in/out, n_level) against right-hand side b; zero_init treats the
 * neighbours as zero.  pf_pressure_vcycle applies the pressure stage's
 * multigrid (mg_cycles V-cycles from x = 0, in the simulator's precision) to
 * a right-hand side b on the cells of level 0 and writes the result x; both
 * are host arrays of N in natural cell order. */
int32_t pf_pressure_level(pf_sim* sim, int32_t level, int32_t* dims, double* A);
pf_status pf_pressure_smooth(pf_sim* sim, int32_t level, int32_t colour, int32_t zero_init,
                             const double* b, double* x);
pf_status pf_pressure_vcycle(pf_sim* sim, const double* b, double* x);

/* Second-stage smoother test hook (Sec. 3.4, the block smoother of the CPR
 * preconditioner; valid after the preconditioner has been set up):
 * z = S^{-1} f for the last set-up system, S the red-black block ILU(0) or
 * block-Jacobi factors in the simulator's precision (well rows: f_w / D_w).
 * f, z: host vectors of 3N + n_wells in the plane layout above. */
pf_status pf_smoother_apply(pf_sim* sim, const double* f, double* z);

/* One step of flexible GMRES's inner loop (Sec. 3.4, Algorithm 2 and the
 * PF order of the two stages; valid after the preconditioner has been set
 * up): z = M^{-1} v, the whole two-stage CPR preconditioner in the
 * simulator's precision, and, if w is non-NULL, w = J~ z (FP64) computed as
 * the solver computes it (in FP64 PF order with the ILU(0) smoother, along
 * with the last smoother phase; there the red rows of w are those of v,
 * which J~ z equals on red rows since red-black ILU(0) keeps the red
 * diagonal blocks, up to the rounding of the block solves).  v, z, w: host
 * vectors of 3N + n_wells in
 * the plane layout above; z is returned in FP64 (widened in mixed
 * precision).  Uses the first two Krylov vectors as device storage. */
pf_status pf_precond_apply(pf_sim* sim, const double* v, double* z, double* w);

/* Static data: row scales D (3N + n_wells), transmissibilities to the
 * +x/+y/+z neighbours (N each, 0 at the boundary), reference pore volumes
 * (N), and per perforation (sorted by cell) its well, cell and Peaceman
 * index.  Any pointer may be NULL. */
pf_status pf_get_static(pf_sim* sim, double* row_scale, double* Tx, double* Ty, double* Tz,
                        double* PVr, int32_t* perf_well, int32_t* perf_cell, double* perf_wi);
int64_t pf_n_perf(const pf_sim* sim);

/* Kernel timing for roofline measurements: between pf_profile_begin and
 * pf_profile_end, every launch of the chosen kernel (PF_K_*) is bracketed
 * by HIP events on the simulator's stream (at most max_launches launches).
 * pf_profile_end synchronises the stream and returns the number of timed
 * launches and their summed duration in milliseconds.  Timing adds event
 * records between kernels and is off by default. */
enum { PF_K_ASSEMBLE = 1, PF_K_SPMV = 2, PF_K_ZLINE = 3, PF_K_MDOT = 4, PF_K_MUPDATE = 5,
       PF_K_ILU = 6, PF_K_STAGE_RESID = 7, PF_K_RED_SPMV = 8, PF_K_BLACK_SPMV = 9 };
pf_status pf_profile_begin(pf_sim* sim, int32_t kernel_id, int32_t max_launches);
pf_status pf_profile_end(pf_sim* sim, int32_t* launches, double* total_ms);

/* ---- Fused launches across simulators ------------------------------------
 * A fusion group merges the device work of its member simulators into
 * shared launches, for many small realisations whose own launches are too
 * short to fill the GPU (one FGMRES iteration issues about 80).  A member
 * records its kernel launches and copies instead of issuing them.  Each
 * member is driven by its own host thread: a call that synchronises (every
 * call that returns host data, and the convergence tests inside pf_step)
 * blocks until every member has reached such a point; the last thread to
 * arrive then issues all the recorded work on the group's stream: one
 * launch per kernel over a table of (member, block range) entries for the
 * operations of the same kernel and block size at the heads of the
 * members' queues, the rest one by one, each member's operations in its
 * own order.  A member computes exactly what it computes alone: the same
 * kernels with the same arguments, block counts and reductions.
 * pf_fusion_create: hip_stream is the group's stream, on the current device
 * (PF_EINVAL for a stream of another device).
 * pf_fusion_join: add a simulator created on the group's device (its own
 * stream is synchronised first; PF_EINVAL for a simulator of another
 * device, one already in a group, on the static workspace or with kernel
 * timing on).  pf_fusion_leave: issue its remaining work and remove it
 * (pf_destroy of a member does this first).  pf_fusion_step: the n
 * simulators join the group (all before any steps), then one pf_step of
 * each (dts[i], stats[i] may be NULL) on a thread of its own, then each
 * leaves; the first failure is returned (a failed join: none steps).
 * pf_fusion_stats: issues, recorded operations and launches so far.
 * pf_fusion_destroy: the group must have no members. */
struct pf_fusion;
typedef struct pf_fusion pf_fusion;
pf_status pf_fusion_create(void* hip_stream, pf_fusion** out);
pf_status pf_fusion_join(pf_fusion* group, pf_sim* sim);
pf_status pf_fusion_leave(pf_sim* sim);
pf_status pf_fusion_step(pf_fusion* group, int32_t n, pf_sim* const* sims, const double* dts,
                         pf_step_stats* stats);
pf_status pf_fusion_stats(pf_fusion* group, int64_t* issues, int64_t* ops, int64_t* launches);
void pf_fusion_destroy(pf_fusion* group);

/* ---- Serving: continuous batching of many realisations on one GPU -------
 * The server owns no device memory: the caller passes one device arena
 * (256-byte aligned) of arena_bytes.  pf_server_submit deep-copies a
 * request (model, options, initial state P0/S0/C0 of N and Pb0 of n_wells,
 * n_steps step lengths in s) into a queue and returns a ticket.  Each of
 * max_slots worker threads owns a HIP stream (default priority); a free
 * worker admits the first queued request, in arrival order, whose footprint
 * (pf_workspace_size) fits the arena's free memory (first fit; a request
 * that does not fit yet lets at most 8 later ones pass before admissions
 * wait for it), runs its schedule with pf_step on its own
 * stream, records each step's wall latency, then frees the memory.
 * Requests arriving while others run are admitted as slots and memory free
 * up, and the active realisations' kernels overlap on the device.  With
 * fused = G > 0 (at most max_slots) the slots are spread over G fusion
 * groups (pf_fusion_*; slot i in group i % G), each on a stream of the
 * server's own: the active realisations of a group are its members for
 * their steps, their launches merged into shared ones, and the G streams
 * overlap on the device.
 * pf_server_poll: state 0 queued, 1 running, 2 done (outputs filled: final
 * P, S, C, Pb; per-step latency (s) and Newton iterations; times[3] =
 * submit, start, end on the host steady clock, s), 3 failed
 * (pf_last_error has the reason).  pf_server_wait blocks until the ticket
 * (0: every request) is finished.  The server keeps a finished request's
 * results until pf_server_release frees them (PF_EINVAL for an unknown
 * ticket or one still queued or running; the ticket is unknown afterwards).
 * pf_server_destroy stops the workers after their current request; queued
 * requests are dropped. */
struct pf_server;
typedef struct pf_server pf_server;
pf_status pf_server_create(void* dev_arena, size_t arena_bytes, int32_t max_slots, int32_t fused, pf_server** out);
pf_status pf_server_submit(pf_server* sv, const pf_model_desc* model, const pf_solver_opts* opts,
                           const double* P0, const double* S0, const double* C0, const double* Pb0,
                           int32_t n_steps, const double* dts, uint64_t* ticket);
pf_status pf_server_poll(pf_server* sv, uint64_t ticket, int32_t* state, double* P, double* S, double* C,
                         double* Pb, double* step_latency_s, int32_t* newton_its, double* times);
pf_status pf_server_wait(pf_server* sv, uint64_t ticket);
pf_status pf_server_release(pf_server* sv, uint64_t ticket);
pf_status pf_server_info(pf_server* sv, int32_t* queued, int32_t* running, int32_t* peak_running,
                         size_t* peak_bytes, size_t* free_bytes);
void pf_server_destroy(pf_server* sv);

/* Wells at the last assembled state (after pf_step: the end of the step),
 * arrays of n_wells, any may be NULL: ctrl the active control (PF_CTRL_*),
 * target its target, qw and qo the surface water and oil rates (m^3/s,
 * positive into the reservoir).  pf_set_state restores the controls given
 * in the model. */
pf_status pf_well_status(pf_sim* sim, int32_t* ctrl, double* target, double* qw, double* qo);

/* Change well w's operation between timesteps (Sec. 3 item 4; e.g. the
 * start or end of polymer injection, Sec. 4.1): control, target, injected
 * concentration and BHP limit as in pf_well.  They become the well's given
 * operation (pf_set_state restores these) and its active one. */
pf_status pf_set_well_operation(pf_sim* sim, int32_t well, int32_t control, double target, double c_inj,
                                double bhp_limit);

/* Message for the last failing call on this thread ("" if none). */
const char* pf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* POLYFLOOD_H */
