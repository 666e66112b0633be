// Internal declarations of the polyflood HIP library (gfx950).
//
// Device data layout (all in the caller's workspace, 256-byte aligned):
//   state vectors   x, xn: 3N + nw doubles: planes P[N], S[N], C[N], then Pb[nw]
//   accumulation    Mn: 3N (water, oil, polymer planes)
//   residual        R: 3N + nw (row-scaled, see polyflood.h)
//   Jacobian        J: 63 planes of N: J[(d*9 + e)*N + i], d = 0 own block,
//                   1..6 = -x,+x,-y,+y,-z,+z neighbour blocks, e = 3*row + col
//   well border     B[3*np] (dR~_cell/dPb), Cw[3*np] (dW~/dx_cell), Dw[nw]
//   static          PVr[N], Tx/Ty/Tz[N] (to the + neighbour, 0 on the boundary)
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>
#include <functional>
#include <string>
#include <vector>

#include "../../include/polyflood.h"

namespace pf {

constexpr double kBar = 1.0e5;
constexpr int kBlock = 256;          // threads per block for cell sweeps
constexpr int kMaxRestart = 64;
constexpr int kRedBlocks = 1024;     // fixed partial-sum grid of the reductions
constexpr int kDotChunk = 16;        // dot products per multi-dot launch
constexpr int kPartSlots = kMaxRestart + 2;   // partial-sum slots: restart + 2 dot products

// Everything a kernel needs to evaluate cell properties; passed by value.
struct DevModel {
    int32_t nx, ny, nz, nw;
    int64_t n, nxy;
    int64_t np;                      // perforations
    int64_t npc;                     // perforated cells
    double dx, dy, dz, top, vol;
    double cr, pref;
    double rho_w0, rho_o0, c_w, c_o, mu_w, mu_o, swc, sor, n_w, n_o, krw0, kro0, grav;
    double a1, a2, omega, cmax, mup_ref, ads_max, ads_b, rrf, ipv;
    double inv_den;                  // 1/(1 - swc - sor)
    double tl_pref;                  // mu_p^ref^(1-omega)  (Todd-Longstaff)
    double tl_pw;                    // mu_w^(1-omega)
    double c_ref;                    // polymer row scale concentration
    double inv_mu_o, inv_rho_w0, inv_vol, rk_slope;   // 1/mu_o, 1/rho_w0, 1/V, (RRF - 1)/A_max
    double inv_rho_o0, inv_c_ref;    // 1/rho_o0, 1/C_ref (row scales)
    int32_t corey2_w, corey2_o, omega1, pad;
    // property variants: mixing rule, tables (adsorption, viscosity multiplier, capillary pressure)
    int32_t mix_rule, n_ads, n_visc, n_pc;
    double mix_ln;                   // ln(mu_p^ref / mu_w) (PF_MIX_EXP)
    // device copy of the tables, kTabSlots x PF_TABLE_MAX doubles:
    // ads_c, ads_a, visc_c, visc_m, pc_s, pc_v, log10 of kperm_k, kperm_rrf, kperm_admax
    const double* tab;
    // retention and the rock table (null when not used): per cell the rock's
    // capacity A_d,max / ads_max, its (RRF - 1) / A_d,max, and the largest
    // past equilibrium adsorption
    int32_t n_kperm, pad2;
    double ads_res;
    const double* cell_cap;
    const double* cell_rks;
    const double* ads_hist;
};
enum { kTabAdsC = 0, kTabAdsA = 1, kTabViscC = 2, kTabViscM = 3, kTabPcS = 4, kTabPcV = 5, kTabKpK = 6,
       kTabKpRrf = 7, kTabKpAdm = 8, kTabSlots = 9 };


// ---- kernel launches: direct, or recorded for a fusion group --------------
// Every kernel is a __device__ body that takes the block index of its launch
// (Blk), with a __global__ wrapper for a direct launch and a functor
// F_<kernel> through which k_multi runs the same body for each simulator's
// share of a merged launch.  A simulator in a fusion group (pf_fusion_*)
// records its launches instead of issuing them; when every member has
// reached a synchronisation point the group issues the recorded work, one
// launch for the ops of the same kernel at the heads of the members' queues.
struct Blk {
    uint32_t x, n;                   // block index within this simulator's launch, its block count
};
#define PF_BLK (::pf::Blk{blockIdx.x, gridDim.x})

// Kernel arguments as a flat aggregate (host and device see one layout).
template <class... T> struct Pack {};
template <class H, class... T> struct Pack<H, T...> {
    H h;
    Pack<T...> t;
};
template <class... T> struct PackOf;
template <> struct PackOf<> {
    static Pack<> make() { return Pack<>{}; }
};
template <class H, class... T> struct PackOf<H, T...> {
    static Pack<H, T...> make(const H& h, const T&... t) { return Pack<H, T...>{h, PackOf<T...>::make(t...)}; }
};
template <class F, class... D>
__device__ __forceinline__ void pack_apply(const F& f, const Blk& wg, const Pack<>&, const D&... d) {
    f(wg, d...);
}
template <class F, class H, class... T, class... D>
__device__ __forceinline__ void pack_apply(const F& f, const Blk& wg, const Pack<H, T...>& p, const D&... d) {
    pack_apply(f, wg, p.t, d..., p.h);
}

// One simulator's share of a merged launch: nb blocks, from a first block
// that is a multiple of 8 (so that every block runs on the XCD it would run
// on alone), and the kernel's arguments.
template <class... P> struct MEntry {
    uint32_t nb, pad;
    Pack<P...> a;
};

// The table of a merged launch: the first blocks of its ns entries as one
// compact array (the block's search touches one or two cache lines), then
// the entries from byte multi_entries(ns).
__host__ __device__ inline size_t multi_entries(int ns) { return ((size_t)ns * 4 + 15) & ~(size_t)15; }

template <class F, class... P>
__global__ __launch_bounds__(F::kLB) void k_multi(const uint8_t* __restrict__ tab, int ns) {
    const uint32_t* __restrict__ b0 = reinterpret_cast<const uint32_t*>(tab);
    const MEntry<P...>* __restrict__ e = reinterpret_cast<const MEntry<P...>*>(tab + multi_entries(ns));
    const uint32_t b = blockIdx.x;
    int lo = 0, hi = ns - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (b0[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    const uint32_t lb = b - b0[lo];
    if (lb >= e[lo].nb) return;          // padding up to the next simulator's range
    pack_apply(F{}, Blk{lb, e[lo].nb}, e[lo].a);
}

using MultiFn = void (*)(const void* table, int n, unsigned blocks, unsigned threads, size_t shm, hipStream_t st);

template <class F, class... P>
void run_multi(const void* table, int n, unsigned blocks, unsigned threads, size_t shm, hipStream_t st) {
    hipLaunchKernelGGL((k_multi<F, P...>), dim3(blocks), dim3(threads), shm, st, static_cast<const uint8_t*>(table),
                       n);
}

// A recorded stream operation of a fusion-group member.
struct Op {
    MultiFn multi = nullptr;         // merged kernel launch, or null: a host-issued operation
    uint32_t nb = 0, threads = 0;    // this simulator's blocks, threads per block
    size_t shm = 0;                  // dynamic LDS bytes
    size_t off = 0, len = 0;         // its MEntry in the member's byte buffer
    std::function<void(hipStream_t)> host;
};

struct Fusion;                       // pf_fuse.hip

// Small device-side control block of FGMRES (Hessenberg, Givens, norms).
struct KrylovCtl {
    double H[(kMaxRestart + 1) * kMaxRestart];   // column-major, ld = kMaxRestart+1
    double cs[kMaxRestart], sn[kMaxRestart];
    double g[kMaxRestart + 1];
    double y[kMaxRestart];
    double h[kMaxRestart + 2];       // scratch column of dot products
    double beta0;                    // initial residual norm of this solve
    double beta;                     // residual norm at the start of this cycle
    double wnorm0;                   // |w| before orthogonalisation
    double wnorm;                    // |w| after
    double inv_h;                    // 1 / h(j+1, j)
    double rel;                      // |g(j+1)| / beta0
    int32_t reorth;                  // second CGS pass requested
    int32_t breakdown;
    int32_t normalised;              // w was scaled to unit norm by the update itself
    int32_t pad;
};

// Grid dimensions of a multigrid level; split: colour-split slot order.
struct Dims { int nx, ny, nz, split; };

struct MGLevel {
    int32_t nx, ny, nz;
    int32_t split;                   // colour-split storage (every level but the coarsest)
    int64_t ns;                      // slots per plane (>= n)
    int32_t cx, cy, cz;              // aggregation factors to the next coarser level
    int64_t n;
    double* A;                       // 7 planes: diag, -x, +x, -y, +y, -z, +z
    double* aux;                     // smoother set-up data (inverse diagonal / line factors)
    double* x;
    double* b;
    double* r;
    float* A32;                      // mixed precision copies
    float* aux32;
    float* x32;
    float* b32;
    float* r32;
};

struct Sim {
    DevModel m;
    pf_solver_opts opts;
    hipStream_t stream;
    hipStream_t aux = nullptr;       // side stream: the coarsest inverse overlaps the ILU set-up
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    char* ws;
    size_t ws_bytes;
    int64_t nv;                      // 3N + nw

    // static
    double *poro, *kx, *ky, *kz;
    double *pvr, *Tx, *Ty, *Tz, *rscale;
    int32_t *perf_cell, *perf_well, *pc_cell, *pc_first, *wp_first, *wp_idx;
    int32_t *pc_map;                 // cell -> index into pc_cell, or -1
    double *perf_wi, *perf_depth;
    int32_t *w_ctrl, *w_inj, *w_dir;
    double *w_target, *w_cinj, *w_gamma, *w_zref, *w_scale, *w_rw, *w_skin;

    // state / system
    double *x, *xn, *Mn, *R, *J, *B, *Cw, *Dw, *wv, *wdp;
    double *perf_q;                  // surface water and oil rate of each perforation (2 per perforation)
    double *cell_cap, *cell_rks;     // rock table per cell (n_kperm > 0)
    double *ads_hist;                // largest past equilibrium adsorption (ads_res > 0)
    double *tab;                     // property tables (kTabSlots x PF_TABLE_MAX)
    double *dx;                      // Newton update
    double *rhs;                     // linear right-hand side

    // solver
    double *V, *Z, *w, *t1, *t2;
    // Krylov vectors: current length nk (nv, or nvc in the colour-split layout)
    // and the stride kst of the columns of V and Z (max(nv, nvc))
    int64_t nk = 0, kst = 0, nvc = 0;
    double *bcs = nullptr, *xcs = nullptr;   // right-hand side and solution in the colour-split layout
    KrylovCtl* kc;
    double *part;                    // reduction partials
    double *red;                     // reduction results (64 doubles)
    double *Dinv;                    // block Jacobi: 9N natural; ILU(0): 2 x 9 colour-split planes
    double *Ap;                      // pressure operator (7N) = level 0 of MG
    double *coarse_aug;              // coarsest-level [A | I] -> [I | A^-1]
    double *coarse_inv;              // compact coarsest inverse (n x n)
    float *coarse_inv32;
    float *Jp32;                     // mixed: FP32 P-columns of J (21 planes)
    double *Lc;                      // FP64 ILU: colour-split off-diagonal blocks (2 x 54 planes)
    double *Jdc;                     // FP64 ILU: colour-split diagonal blocks of J (2 x 9 planes)
    uint16_t *Joff16;                // mixed ILU: colour-split BF16 off-diagonal blocks (2 x 54 planes)
    float *Dinv32;                   // mixed: FP32 smoother inverse diagonals
    float *t32;                      // mixed: FP32 stage residual
    float *Z32;                      // mixed: FP32 preconditioned Krylov vectors
    double *pb;                      // well bottom-hole pressures of the pressure stage
    double *pnat;                    // pressure-stage correction in natural cell order
    float *pnat32;                   // the same, mixed precision
    std::vector<MGLevel> mg;
    int restart_cap;
    int max_lds = 65536;             // bytes of LDS a workgroup may allocate

    // host
    double* hbuf;                    // read-back buffer (64 doubles): pinned, or static (static_dev >= 0)
    int static_dev = -1;             // device whose static workspace this simulator holds (-1: caller's)
    int device = 0;                  // device current at creation (its workspace and stream)
    bool coarse_pending = false;     // the coarsest inverse may still run on the side stream
    bool j_cs = false;               // the last Jacobian is in the colour-split copies (Jdc, Lc) only
    bool j_nat = true;               // the natural-order planes of J hold the last Jacobian
    int newton_it;                   // Newton iterations in the current step
    double dt_next = 0.0;            // next sub-step length (0: the scheduled step)
    double last_upd;
    double last_bnorm;               // ||R~||_2 of the previous Newton iteration
    int prec_ready;
    std::vector<int32_t> h_perf_cell, h_perf_well, h_w_ctrl;
    // well controls: as given in the model (primary) and active (after BHP-limit switches)
    std::vector<int32_t> h_ctrl0, h_inj, h_wp_first;
    std::vector<double> h_target0, h_limit, h_target;
    std::vector<double> h_perf_wi;
    std::vector<int32_t> h_wktop;    // datum (top perforated) layer of every well

    // fusion group membership (pf_fusion_join): recorded operations
    Fusion* fu = nullptr;
    std::vector<Op> ops;
    std::vector<uint8_t> op_bytes;

    // kernel timing (pf_profile_begin/end)
    int prof_id = 0;
    int prof_used = 0;
    std::vector<hipEvent_t> prof_ev;     // start/stop pairs
};

// Brackets one launch with events when the simulator times this kernel.
struct ProfScope {
    Sim& s;
    bool on;
    ProfScope(Sim& sim, int id)
        : s(sim), on(!sim.fu && sim.prof_id == id && 2 * (sim.prof_used + 1) <= (int)sim.prof_ev.size()) {
        if (on) (void)hipEventRecord(s.prof_ev[2 * s.prof_used], s.stream);
    }
    ~ProfScope() {
        if (on) {
            (void)hipEventRecord(s.prof_ev[2 * s.prof_used + 1], s.stream);
            ++s.prof_used;
        }
    }
};

// Bump allocator over the workspace; with base == nullptr it only measures.
struct Bump {
    char* base;
    size_t used = 0;
    template <class T>
    T* take(size_t count) {
        used = (used + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + used) : nullptr;
        used += (count > 0 ? count : 1) * sizeof(T);
        return p;
    }
};

// ---- kernels launchers (k_physics.hip) ----------------------------------
void launch_static(Sim& s);
void launch_accum(Sim& s, const double* x, double* M);
void launch_assemble(Sim& s, double dt, bool with_jacobian);
void launch_norms(Sim& s, const double* v, double* out);          // out[0..5]
void launch_update(Sim& s, const double* dx, double* out, bool cs = false);   // out[0..4]; cs: dx colour-split
void launch_kperm(Sim& s);                                          // per-cell RRF, A_d,max
void launch_ads_hist(Sim& s);                                       // take in the current state
void launch_equilibrium(Sim& s, double datum_depth, double datum_p, double fwl_depth);

// ---- linear algebra (k_linalg.hip) ----------------------------------------
void launch_spmv(Sim& s, const double* x, double* y);
void launch_spmv(Sim& s, const float* x, double* y);
// the well border of y = J x alone; cs: 0 natural layout, 1 colour-split, 2 colour-split black cell rows and wells
void launch_spmv_border(Sim& s, const double* x, double* y, int cs = 0);
void launch_to_cs(Sim& s, const double* x, double* y, double scale = 1.0);   // natural -> colour-split, times scale
void launch_from_cs(Sim& s, const double* x, double* y);          // colour-split -> natural layout
void launch_axpby(Sim& s, int64_t n, double a, const double* x, double b, double* y);
void launch_copy(Sim& s, int64_t n, const double* x, double* y);
void launch_fill(Sim& s, int64_t n, double v, double* y);
// J in the colour-split layout only (FP64 red-black ILU(0), PF order), and
// the natural-order planes formed from it when a kernel needs them
bool j_colour_split_mode(const Sim& s);
void ensure_j_natural(Sim& s);
void launch_copy_words(Sim& s, const void* src, void* dst, size_t bytes);   // bytes: a multiple of 4
void launch_bjac_setup(Sim& s);
void launch_bjac_apply(Sim& s, const double* r, double* z);
// Krylov helpers
void launch_norm_to_ctl(Sim& s, const double* v, int which);      // which 0: beta0+beta, 1: beta
void launch_scale_by_ctl(Sim& s, const double* v, double* out, int which);  // which 0: 1/beta, 1: inv_h
void launch_arnoldi(Sim& s, int j, double* w);                     // first CGS pass of w against V[0..j]
void launch_arnoldi_second(Sim& s, int j, double* w);              // second pass (when requested)
void launch_normalise(Sim& s, double* w);                          // w /= h(j+1, j)
void launch_solve_small(Sim& s, int k);                             // y = H(0:k,0:k)^{-1} g
void launch_zcomb(Sim& s, int k, double* dx, bool first = false);   // dx += Z y (first: dx = Z y)
void launch_init_cycle(Sim& s, int first);

// ---- CPR (k_cpr.hip) ---------------------------------------------------------
void cpr_choose_levels(Sim& s);     // host: multigrid hierarchy shape
void cpr_plan(Sim& s, Bump& b);      // workspace of the preconditioner
void cpr_setup(Sim& s);
void cpr_apply(Sim& s, const double* v, double* z);
void cpr_apply(Sim& s, const double* v, float* z);      // mixed precision
void cpr_apply_spmv(Sim& s, const double* v, double* z, double* w);   // z = M^{-1} v, w = J z
bool cpr_colour_split(const Sim& s);  // cpr_apply_spmv takes and gives the colour-split layout
void mg_smooth_once(Sim& s, int level, int colour, int zero_init);   // test hook
int64_t mg_slot(const MGLevel& L, int ix, int iy, int iz);             // cell -> slot of a level
void mg_cycles_once(Sim& s, const double* v);   // test hook: s.pnat(32) = V-cycles(Pi_r v)
void smoother_once(Sim& s, const double* f);    // test hook: s.t1 (FP64) / s.Z32 (mixed) = S f

// ---- errors -----------------------------------------------------------------
void set_error(const std::string& msg);
struct HipError { std::string msg; };
#define PF_HIP(call)                                                              \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess)                                                     \
            throw ::pf::HipError{std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)
#define PF_LAUNCH_CHECK() PF_HIP(hipGetLastError())

// ---- fusion group hooks (pf_fuse.hip) -----------------------------------------
void fusion_record(Sim& s, MultiFn f, uint32_t nb, uint32_t threads, size_t shm, const void* entry, size_t len);
void fusion_host(Sim& s, std::function<void(hipStream_t)> op);
void fusion_sync(Sim& s);            // every member at a synchronisation point: the group's work is issued

// Launch of kernel k (functor F) on stream st, or its record in s's fusion group.
template <class F, class... P, class... A>
void launch(Sim& s, hipStream_t st, void (*k)(P...), dim3 grid, dim3 block, size_t shm, const A&... a) {
    static_assert(sizeof...(P) == sizeof...(A), "argument count");
    if (!s.fu) {
        hipLaunchKernelGGL(k, grid, block, shm, st, a...);
        PF_LAUNCH_CHECK();
        return;
    }
    if (grid.y != 1 || grid.z != 1 || block.y != 1 || block.z != 1) {
        fusion_host(s, [=](hipStream_t q) { hipLaunchKernelGGL(k, grid, block, shm, q, a...); });
        return;
    }
    using E = MEntry<P...>;
    static_assert(sizeof(E) % alignof(E) == 0 && alignof(E) <= 16, "entries of one launch are an array");
    const E e{grid.x, 0u, PackOf<P...>::make(static_cast<P>(a)...)};
    fusion_record(s, &run_multi<F, P...>, grid.x, block.x, shm, &e, sizeof(e));
}

// Host <-> device copies and stream synchronisation of a simulator's stream
// (recorded in a fusion group: host sources are copied at record time).
void copy_h2d(Sim& s, void* dst, const void* src, size_t bytes);
void copy_d2h(Sim& s, void* dst, const void* src, size_t bytes);
void stream_sync(Sim& s);

// Colour-split vector layout of the FP64 red-black ILU(0) path (PF order):
// each of the three planes holds 2 ns entries, the red cells ((ix+iy+iz) even)
// in slots [0, ns) and the black ones in [ns, 2 ns), both in the slot order
// of the smoother's colour-split factors (x-lines of ceil(nx/2) slots, lines
// in natural order; where nx is odd every other line has a pad slot, which
// holds zero); the wells follow the three planes.  A kernel over the cells
// of one colour then writes whole cache lines.
__host__ __device__ __forceinline__ int64_t cs_ns(const DevModel& m) {
    return (int64_t)((m.nx + 1) / 2) * m.ny * m.nz;
}
// plane offset of the cell with natural index i
__device__ __forceinline__ int64_t cs_index(const DevModel& m, int64_t i) {
    const int64_t iz = i / m.nxy;
    const int64_t rem = i - iz * m.nxy;
    const int64_t iy = rem / m.nx;
    const int64_t ix = rem - iy * m.nx;
    return ((ix + iy + iz) & 1) * cs_ns(m) + (iy + m.ny * iz) * ((m.nx + 1) >> 1) + (ix >> 1);
}

// XCD-aware block order: workgroups are dispatched round-robin over the 8
// XCDs (each with its own L2); renumbering them so that XCD x processes one
// contiguous range of blocks keeps stencil neighbours in the same L2.
__device__ __forceinline__ int64_t xcd_block(const Blk& wg) {
    const int64_t nb = wg.n, b = wg.x;
    const int64_t q = nb >> 3, r = nb & 7, x = b & 7, j = b >> 3;
    return x * q + (x < r ? x : r) + j;
}

// y-strip order of a grid of lines of w entries (line = iy + ny*iz): strips
// of kStripLines lines in y, each taken layer by layer, a strip-layer being
// one contiguous run of entries.  Maps a thread index v to an entry (a
// bijection on [0, w*ny*nz)); the last strip may hold fewer lines.  Kernels
// whose threads read neighbours one layer up or down use it on grids with
// large layers, so that those neighbours were read a strip-layer earlier
// (within the reach of the L2 cache) rather than a whole layer earlier.
constexpr int64_t kStripLines = 16;
__device__ __forceinline__ int64_t strip_order(int64_t v, int64_t w, int64_t ny, int64_t nz) {
    if (ny <= kStripLines) return v;
    const int64_t full = kStripLines * w * nz;          // entries of a strip of kStripLines lines
    const int64_t st = v / full;
    const int64_t y0 = st * kStripLines;
    const int64_t lines = min(kStripLines, ny - y0);
    const int64_t r = v - st * full;
    const int64_t per_layer = lines * w;
    const int64_t iz = r / per_layer;
    const int64_t r2 = r - iz * per_layer;
    return (y0 + ny * iz) * w + r2;                     // line (y0 + r2 / w, iz), entry r2 % w
}

// The cell a natural-order kernel's thread v takes: y-strips on grids whose
// layers hold at least kStripCells cells, natural order otherwise.
constexpr int64_t kStripCells = 65536;
__device__ __forceinline__ int64_t strip_cell(const DevModel& m, int64_t v) {
    if (m.nxy < kStripCells) return v;
    return strip_order(v, m.nx, m.ny, m.nz);
}

inline unsigned grid_for(int64_t n, int block = kBlock) {
    int64_t g = (n + block - 1) / block;
    return (unsigned)(g > 0 ? g : 1);
}

}  // namespace pf

// the simulator behind a handle of the C interface
pf::Sim& pf_sim_state(pf_sim* h);
