// Two-stage CPR preconditioner (Sec. 3.4, Algorithm 2).
//
// Stage "P": the pressure block.  Its operator A_p is the P-column of the sum
// of the (row-scaled) water and oil equations - a total-volume combination
// of the two phase equations, which stays non-singular where the water
// relative permeability vanishes - and the restriction sums the water and
// oil residuals of a cell.  A_p is solved approximately by mg_cycles
// multigrid V-cycles on the structured grid (pre-smoothing only; the
// upward pass is one prolongation chain):
//   * smoother: z-line Gauss-Seidel, columns coloured as a checkerboard in
//     (x, y); each column's tridiagonal system is solved exactly with
//     factors precomputed at set-up (the vertical couplings of thin layers
//     are the strongest, so they are relaxed implicitly); every smoothed
//     level is stored colour-split by column;
//   * coarsening: unsmoothed box aggregation with a Galerkin coarse operator,
//     which stays a 7-point stencil; only x and y are aggregated while a
//     level keeps >= 4096 columns, then 2x2x2;
//   * coarsest level (<= mg_coarse cells): dense inverse by Gauss-Jordan,
//     computed on a side stream during the smoother set-up.
// The well bottom-hole pressures of the pressure stage follow from the well
// rows once the cell pressures are known.
//
// Stage "F": a full-system block smoother on the 3x3 blocks: block Jacobi
// or red-black block ILU(0).
//
// Order: PF (pressure first, then the smoother on the stage residual) or FP
// (the order of Algorithm 2: smoother, residual, pressure correction).
#include "pf_internal.h"

#include <algorithm>
#include <cfloat>

namespace pf {
namespace {

constexpr int kColsForXY = 4096;
constexpr int64_t kZlineSmallThreads = 65536;
constexpr int64_t kPreSmallCells = 50000;   // default mg_small_cells
constexpr int kPreSmall = 5;                // default mg_pre_small
constexpr int64_t kPreSmallFrac = 32;       // levels of at most 1/32 of the finest level count as small

}  // namespace

// Level storage.  A smoothed level is split by column colour c = (ix+iy)&1:
// cell (ix, iy, iz) has slot c*half + (iz*ny + iy)*hx + (ix>>1), hx =
// ceil(nx/2), half = hx*ny*nz, so the columns one z-line half-sweep visits
// are contiguous and their neighbours (the other colour) are too.  The
// coarsest level (solved directly, never swept) is in natural order.  Planes
// of a level are lv_slots() apart; slots of absent cells (ix = nx when nx is
// odd) are never read.
__host__ __device__ __forceinline__ int64_t lv_half(const Dims& g) {
    return (int64_t)((g.nx + 1) >> 1) * g.ny * g.nz;
}
__host__ __device__ __forceinline__ int64_t lv_slots(const Dims& g) {
    return g.split ? 2 * lv_half(g) : (int64_t)g.nx * g.ny * g.nz;
}
__host__ __device__ __forceinline__ int64_t lv_index(const Dims& g, int ix, int iy, int iz) {
    if (!g.split) return ix + (int64_t)g.nx * (iy + (int64_t)g.ny * iz);
    return ((ix + iy) & 1) * lv_half(g) + ((int64_t)iz * g.ny + iy) * ((g.nx + 1) >> 1) + (ix >> 1);
}

Dims dims_of(const MGLevel& L) { return Dims{L.nx, L.ny, L.nz, L.split}; }
int64_t mg_slot(const MGLevel& L, int ix, int iy, int iz) { return lv_index(dims_of(L), ix, iy, iz); }

namespace {

// natural cell index -> coordinates
__device__ __forceinline__ void cell_coords(const Dims& g, int64_t i, int& ix, int& iy, int& iz) {
    const int64_t nxy = (int64_t)g.nx * g.ny;
    iz = (int)(i / nxy);
    const int64_t rem = i - (int64_t)iz * nxy;
    iy = (int)(rem / g.nx);
    ix = (int)(rem - (int64_t)iy * g.nx);
}

// Level-0 pressure operator: the P-column of the (water + oil) rows of J.
__device__ __forceinline__ void k_extract_ap_d(const Blk& wg, Dims g, const double* __restrict__ J,
                                               double* __restrict__ A) {
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int64_t i = (int64_t)wg.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int ix, iy, iz;
    cell_coords(g, i, ix, iy, iz);
    const int64_t j = lv_index(g, ix, iy, iz), ns = lv_slots(g);
    for (int d = 0; d < 7; ++d) {
        const double* Jd = J + (int64_t)d * 9 * n;
        A[(int64_t)d * ns + j] = Jd[0 * n + i] + Jd[3 * n + i];   // (water + oil) rows, P column
    }
}
__global__ void k_extract_ap(Dims g, const double* __restrict__ J, double* __restrict__ A) {
    k_extract_ap_d(PF_BLK, g, J, A);
}
struct F_k_extract_ap {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_extract_ap_d(wg, a...);
    }
};

// The same from the colour-split storage of J (diagonal blocks Jdc, face
// blocks Lc; cell colour (ix+iy+iz)&1, slot (iy + ny*iz)*ceil(nx/2) + ix/2).
__device__ __forceinline__ void k_extract_ap_cs_d(const Blk& wg, Dims g, const double* __restrict__ Lc,
                                                  const double* __restrict__ Jdc, double* __restrict__ A) {
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int64_t i = (int64_t)wg.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int ix, iy, iz;
    cell_coords(g, i, ix, iy, iz);
    const int64_t j = lv_index(g, ix, iy, iz), ns = lv_slots(g);
    const int64_t nsl = (int64_t)((g.nx + 1) >> 1) * g.ny * g.nz, cl = (ix + iy + iz) & 1;
    const int64_t sl = ((int64_t)iy + (int64_t)g.ny * iz) * ((g.nx + 1) >> 1) + (ix >> 1);
    for (int d = 0; d < 7; ++d) {
        const double* Jd = d == 0 ? Jdc + cl * 9 * nsl + sl : Lc + (cl * 54 + (d - 1) * 9) * nsl + sl;
        A[(int64_t)d * ns + j] = Jd[0 * nsl] + Jd[3 * nsl];   // (water + oil) rows, P column
    }
}
__global__ void k_extract_ap_cs(Dims g, const double* __restrict__ Lc, const double* __restrict__ Jdc,
                                double* __restrict__ A) {
    k_extract_ap_cs_d(PF_BLK, g, Lc, Jdc, A);
}
struct F_k_extract_ap_cs {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_extract_ap_cs_d(wg, a...);
    }
};

// Galerkin coarse operator of box aggregation (piecewise-constant
// prolongation): couplings inside an aggregate fold into the coarse
// diagonal; couplings across its face in direction d become coarse
// coefficient d.
__device__ __forceinline__ void k_galerkin_d(const Blk& wg, Dims f, Dims c, int cx, int cy, int cz,
                                             const double* __restrict__ Af, double* __restrict__ Ac) {
    const int64_t nc = (int64_t)c.nx * c.ny * c.nz;
    const int64_t I = (int64_t)wg.x * blockDim.x + threadIdx.x;
    if (I >= nc) return;
    const int64_t nf = lv_slots(f);
    const int64_t cxy = (int64_t)c.nx * c.ny;
    const int IZ = (int)(I / cxy);
    const int64_t rem = I - IZ * cxy;
    const int IY = (int)(rem / c.nx);
    const int IX = (int)(rem - (int64_t)IY * c.nx);
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int dz = 0; dz < cz; ++dz) {
        const int iz = IZ * cz + dz;
        if (iz >= f.nz) continue;
        for (int dy = 0; dy < cy; ++dy) {
            const int iy = IY * cy + dy;
            if (iy >= f.ny) continue;
            for (int dx = 0; dx < cx; ++dx) {
                const int ix = IX * cx + dx;
                if (ix >= f.nx) continue;
                const int64_t i = lv_index(f, ix, iy, iz);
                acc[0] += Af[i];
                // -x, +x, -y, +y, -z, +z: internal iff the neighbour stays in the box
                const bool in[6] = {dx > 0, dx + 1 < cx && ix + 1 < f.nx, dy > 0, dy + 1 < cy && iy + 1 < f.ny,
                                    dz > 0, dz + 1 < cz && iz + 1 < f.nz};
                for (int d = 0; d < 6; ++d) {
                    const double a = Af[(int64_t)(d + 1) * nf + i];
                    if (in[d]) acc[0] += a;
                    else acc[d + 1] += a;
                }
            }
        }
    }
    const int64_t nsc = lv_slots(c), Ic = lv_index(c, IX, IY, IZ);
    for (int d = 0; d < 7; ++d) Ac[(int64_t)d * nsc + Ic] = acc[d];
}
__global__ void k_galerkin(Dims f, Dims c, int cx, int cy, int cz, const double* __restrict__ Af,
                           double* __restrict__ Ac) {
    k_galerkin_d(PF_BLK, f, c, cx, cy, cz, Af, Ac);
}
struct F_k_galerkin {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_galerkin_d(wg, a...);
    }
};

// Thomas factors of every z-column: aux[0..n) = c'_k, aux[n..2n) = 1/den_k,
// aux[2n..3n) = -a_k/den_k (the forward recurrence d'_k = alpha_k d'_{k-1} +
// r_k/den_k).
__device__ __forceinline__ void k_zline_setup_d(const Blk& wg, Dims g, const double* __restrict__ A,
                                                double* __restrict__ aux) {
    const int64_t nxy = (int64_t)g.nx * g.ny;
    const int64_t t = (int64_t)wg.x * blockDim.x + threadIdx.x;
    if (t >= nxy) return;
    const int64_t n = lv_slots(g);
    const int iy = (int)(t / g.nx), ix = (int)(t - (int64_t)iy * g.nx);
    const int64_t lstride = lv_index(g, ix, iy, 1) - lv_index(g, ix, iy, 0);
    double cprev = 0.0;
    int64_t i = lv_index(g, ix, iy, 0);
    for (int k = 0; k < g.nz; ++k, i += lstride) {
        const double den = A[i] - A[5 * n + i] * cprev;
        const double id = 1.0 / den;
        const double cp = A[6 * n + i] * id;
        aux[i] = cp;
        aux[n + i] = id;
        aux[2 * n + i] = -A[5 * n + i] * id;
        cprev = cp;
    }
}
__global__ void k_zline_setup(Dims g, const double* __restrict__ A, double* __restrict__ aux) {
    k_zline_setup_d(PF_BLK, g, A, aux);
}
struct F_k_zline_setup {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_zline_setup_d(wg, a...);
    }
};

// One half-sweep of z-line Gauss-Seidel over the columns of one colour
// ((ix + iy) % 2 == colour), each column's tridiagonal system solved by the
// Thomas algorithm with the factors of k_zline_setup.  With zero_init the
// neighbours are taken as 0 (first half-sweep from a zero initial guess).
//
// Segmented: a block holds cpb consecutive columns of the active colour and
// nseg segments per column; segment s owns layers [s*L, (s+1)*L).  Both
// Thomas recurrences are affine in the carried value, so each segment first
// folds its cells into one affine map; the maps of the segments below
// (forward) or above (backward) are composed through LDS; then every segment
// finishes its own cells.  Consecutive threads take consecutive columns, so
// loads are coalesced along x, and the column work is spread over nseg
// times more threads than a thread-per-column sweep.  This variant keeps a
// segment's layers in registers (L <= LMAX <= 8).
//
// zline_seg_body is one block's share: columns col0 .. col0+cpb-1, thread t
// (t >= cpb*nseg idle; every thread reaches the three barriers).  With BIN
// the right-hand side of the segment's layers comes in registers (bin[j],
// layer seg*L + j) instead of from b.
template <int LMAX, class T, bool ZERO_INIT, bool BIN = false>
__device__ __forceinline__ void zline_seg_body(const Dims& g, const T* __restrict__ A, const T* __restrict__ aux,
                                               const T* __restrict__ b, T* __restrict__ x, int colour, int L,
                                               int nseg, int cpb, int64_t col0, int t, T* sA, T* sB,
                                               const T* bin = nullptr) {
    static_assert(LMAX <= 8, "long segments use k_zline_seg_mem");
    static_assert(!BIN || ZERO_INIT, "a right-hand side in registers is for a first half-sweep");
    // thread t -> segment t / cpb, column t % cpb
    const int seg = t / cpb, c = t - seg * cpb;
    const int hx = (g.nx + 1) >> 1;
    const int64_t tcol = col0 + c;
    bool active = seg < nseg && tcol < (int64_t)hx * g.ny;
    int iy = 0, ix = 0;
    if (active) {
        // a column index of one colour fits 32 bits (hx * ny < 2^31)
        const int tc = (int)tcol;
        iy = tc / hx;
        ix = 2 * (tc - iy * hx) + ((iy + colour) & 1);
        active = ix < g.nx;
    }
    // colour-split level: this colour's columns are contiguous (slot
    // colour*half + tcol + k*lstr), the x and y neighbours lie at fixed
    // offsets in the other colour's half
    const int64_t half = (int64_t)hx * g.ny * g.nz, n = 2 * half, lstr = (int64_t)hx * g.ny;
    const int k0 = seg * L;
    const int len = active ? max(0, min(L, g.nz - k0)) : 0;
    // every load below is unconditional from a valid cell (the segment's
    // last layer past its end, the cell itself for a missing neighbour) and
    // masked afterwards, so all layers' loads issue together instead of one
    // memory round trip per layer
    const int64_t i0 = len > 0 ? colour * half + tcol + (int64_t)k0 * lstr : 0;
    const bool xm = len > 0 && ix > 0, xp = len > 0 && ix + 1 < g.nx;
    const bool ym = len > 0 && iy > 0, yp = len > 0 && iy + 1 < g.ny;
    const int64_t dother = (1 - 2 * colour) * half;
    const int64_t oxm = xm ? dother + (((ix - 1) >> 1) - (ix >> 1)) : 0;
    const int64_t oxp = xp ? dother + (((ix + 1) >> 1) - (ix >> 1)) : 0;
    const int64_t oym = ym ? dother - hx : 0, oyp = yp ? dother + hx : 0;
    T al[LMAX], be[LMAX], cp[LMAX];
#pragma unroll
    for (int j = 0; j < LMAX; ++j) {
        cp[j] = 0;
        al[j] = 1;
        be[j] = 0;
    }
    // idle threads keep the identity steps; a wave of idle threads skips the loads
    if (len > 0) {
#pragma unroll
        for (int j = 0; j < LMAX; ++j) {
            const bool v = j < len;
            const int64_t i = i0 + (int64_t)(v ? j : len - 1) * lstr;
            T r;
            if constexpr (BIN) r = bin[j];
            else r = b[i];
            if (!ZERO_INIT) {
                // selects, not products with 0: x may hold anything where masked
                const T a1 = A[n + i], a2 = A[2 * n + i], a3 = A[3 * n + i], a4 = A[4 * n + i];
                const T x1 = x[i + oxm], x2 = x[i + oxp], x3 = x[i + oym], x4 = x[i + oyp];
                r -= (xm ? a1 * x1 : (T)0) + (xp ? a2 * x2 : (T)0) + (ym ? a3 * x3 : (T)0) +
                     (yp ? a4 * x4 : (T)0);
            }
            const T c0 = aux[i], c1 = aux[n + i], c2 = aux[2 * n + i];
            cp[j] = v ? c0 : (T)0;
            al[j] = v ? c2 : (T)1;
            be[j] = v ? r * c1 : (T)0;
        }
    }
    T Fa = 1, Fb = 0;
#pragma unroll
    for (int j = 0; j < LMAX; ++j) {
        Fb = al[j] * Fb + be[j];
        Fa = al[j] * Fa;
    }
    sA[t] = Fa;
    sB[t] = Fb;
    __syncthreads();
    T y = 0;
    // the maps' loads do not depend on the carried value: unrolled, they issue together
#pragma unroll 8
    for (int q = 0; q < seg; ++q) y = sA[q * cpb + c] * y + sB[q * cpb + c];
    // forward values d'_k (kept in be); then this segment's backward map.
    // Positions past the segment's end are identity steps in both passes
    // (forward: al = 1, be = 0; backward: factor 1, be = 0).
#pragma unroll
    for (int j = 0; j < LMAX; ++j) {
        y = al[j] * y + be[j];
        be[j] = j < len ? y : (T)0;
    }
    T Ga = 1, Gb = 0;
#pragma unroll
    for (int j = LMAX - 1; j >= 0; --j) {
        const T gm = j < len ? -cp[j] : (T)1;
        al[j] = gm;
        Gb = gm * Gb + be[j];
        Ga = gm * Ga;
    }
    __syncthreads();
    sA[t] = Ga;
    sB[t] = Gb;
    __syncthreads();
    T xin = 0;
#pragma unroll 8
    for (int q = nseg - 1; q > seg; --q) xin = sA[q * cpb + c] * xin + sB[q * cpb + c];
#pragma unroll
    for (int j = LMAX - 1; j >= 0; --j) {
        xin = al[j] * xin + be[j];
        if (j < len) x[i0 + (int64_t)j * lstr] = xin;
    }
}

template <int LMAX, class T, bool ZERO_INIT>
__device__ __forceinline__ void k_zline_seg_d(const Blk& wg, Dims g, const T* __restrict__ A,
                                              const T* __restrict__ aux, const T* __restrict__ b, T* __restrict__ x,
                                              int colour, int L, int nseg, int cpb) {
    __shared__ T sA[1024];
    __shared__ T sB[1024];
    zline_seg_body<LMAX, T, ZERO_INIT>(g, A, aux, b, x, colour, L, nseg, cpb, xcd_block(wg) * cpb, (int)threadIdx.x,
                                       sA, sB);
}
template <int LMAX, class T, bool ZERO_INIT>
__global__ __launch_bounds__(1024) void k_zline_seg(Dims g, const T* __restrict__ A, const T* __restrict__ aux,
                                                    const T* __restrict__ b, T* __restrict__ x, int colour, int L,
                                                    int nseg, int cpb) {
    k_zline_seg_d<LMAX, T, ZERO_INIT>(PF_BLK, g, A, aux, b, x, colour, L, nseg, cpb);
}
template <int LMAX, class T, bool ZERO_INIT>
struct F_k_zline_seg {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_zline_seg_d<LMAX, T, ZERO_INIT>(wg, a...);
    }
};

// Whole sweeps (colour 0, then colour 1, sweeps times) of a level small
// enough for one workgroup to hold every column of a colour: each half reads
// the other colour's values of the same launch after a workgroup barrier, so
// all the level's pre-sweeps cost one launch instead of two per sweep, with
// the same arithmetic.
template <int LMAX, class T, bool ZERO_FIRST>
__device__ __forceinline__ void k_zline_full_d(const Blk& wg, Dims g, const T* __restrict__ A,
                                               const T* __restrict__ aux, const T* __restrict__ b, T* __restrict__ x,
                                               int L, int nseg, int cpb, int sweeps) {
    __shared__ T sA[1024];
    __shared__ T sB[1024];
    const int t = (int)threadIdx.x;
    zline_seg_body<LMAX, T, ZERO_FIRST>(g, A, aux, b, x, 0, L, nseg, cpb, 0, t, sA, sB);
    __syncthreads();
    zline_seg_body<LMAX, T, false>(g, A, aux, b, x, 1, L, nseg, cpb, 0, t, sA, sB);
    for (int k = 1; k < sweeps; ++k) {
        __syncthreads();
        zline_seg_body<LMAX, T, false>(g, A, aux, b, x, 0, L, nseg, cpb, 0, t, sA, sB);
        __syncthreads();
        zline_seg_body<LMAX, T, false>(g, A, aux, b, x, 1, L, nseg, cpb, 0, t, sA, sB);
    }
}
template <int LMAX, class T, bool ZERO_FIRST>
__global__ __launch_bounds__(1024) void k_zline_full(Dims g, const T* __restrict__ A, const T* __restrict__ aux,
                                                     const T* __restrict__ b, T* __restrict__ x, int L, int nseg,
                                                     int cpb, int sweeps) {
    k_zline_full_d<LMAX, T, ZERO_FIRST>(PF_BLK, g, A, aux, b, x, L, nseg, cpb, sweeps);
}
template <int LMAX, class T, bool ZERO_FIRST>
struct F_k_zline_full {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_zline_full_d<LMAX, T, ZERO_FIRST>(wg, a...);
    }
};

// The same half-sweep for segments of any length: no per-layer register
// arrays; the forward terms are staged in the column's own x entries, which
// no other thread reads during a half-sweep of this colour (the x and y
// neighbours of a column have the other colour).
template <class T>
__device__ __forceinline__ void k_zline_seg_mem_d(const Blk& wg, Dims g, const T* __restrict__ A,
                                                  const T* __restrict__ aux, const T* __restrict__ b,
                                                  T* __restrict__ x, int colour, int zero_init, int L, int nseg,
                                                  int cpb) {
    __shared__ T sA[256];
    __shared__ T sB[256];
    const int t = threadIdx.x;
    const int seg = t / cpb, c = t - seg * cpb;
    const int hx = (g.nx + 1) >> 1;
    const int64_t tcol = xcd_block(wg) * cpb + c;
    bool active = seg < nseg && tcol < (int64_t)hx * g.ny;
    int iy = 0, ix = 0;
    if (active) {
        iy = (int)(tcol / hx);
        ix = 2 * (int)(tcol - (int64_t)iy * hx) + ((iy + colour) & 1);
        active = ix < g.nx;
    }
    // colour-split level (see k_zline_seg)
    const int64_t half = (int64_t)hx * g.ny * g.nz, n = 2 * half, lstr = (int64_t)hx * g.ny;
    const int k0 = seg * L;
    const int len = active ? max(0, min(L, g.nz - k0)) : 0;
    const int64_t i0 = colour * half + tcol + (int64_t)k0 * lstr;
    const bool xm = ix > 0, xp = ix + 1 < g.nx, ym = iy > 0, yp = iy + 1 < g.ny;
    const int64_t dother = (1 - 2 * colour) * half;
    const int64_t oxm = dother + (((ix - 1) >> 1) - (ix >> 1)), oxp = dother + (((ix + 1) >> 1) - (ix >> 1));
    const int64_t oym = dother - hx, oyp = dother + hx;
    T Fa = 1, Fb = 0;
#pragma unroll 4
    for (int j = 0; j < len; ++j) {
        const int64_t i = i0 + (int64_t)j * lstr;
        T r = b[i];
        if (!zero_init) {
            if (xm) r -= A[n + i] * x[i + oxm];
            if (xp) r -= A[2 * n + i] * x[i + oxp];
            if (ym) r -= A[3 * n + i] * x[i + oym];
            if (yp) r -= A[4 * n + i] * x[i + oyp];
        }
        const T a = aux[2 * n + i];
        const T be = r * aux[n + i];
        x[i] = be;
        Fb = a * Fb + be;
        Fa = a * Fa;
    }
    sA[t] = Fa;
    sB[t] = Fb;
    __syncthreads();
    T y = 0;
    // the maps' loads do not depend on the carried value: unrolled, they issue together
#pragma unroll 8
    for (int q = 0; q < seg; ++q) y = sA[q * cpb + c] * y + sB[q * cpb + c];
    for (int j = 0; j < len; ++j) {
        const int64_t i = i0 + (int64_t)j * lstr;
        y = aux[2 * n + i] * y + x[i];
        x[i] = y;
    }
    T Ga = 1, Gb = 0;
    for (int j = len - 1; j >= 0; --j) {
        const int64_t i = i0 + (int64_t)j * lstr;
        const T gm = -aux[i];
        Gb = gm * Gb + x[i];
        Ga = gm * Ga;
    }
    __syncthreads();
    sA[t] = Ga;
    sB[t] = Gb;
    __syncthreads();
    T xin = 0;
#pragma unroll 8
    for (int q = nseg - 1; q > seg; --q) xin = sA[q * cpb + c] * xin + sB[q * cpb + c];
    for (int j = len - 1; j >= 0; --j) {
        const int64_t i = i0 + (int64_t)j * lstr;
        xin = -aux[i] * xin + x[i];
        x[i] = xin;
    }
}
template <class T>
__global__ __launch_bounds__(256) void k_zline_seg_mem(Dims g, const T* __restrict__ A, const T* __restrict__ aux,
                                                       const T* __restrict__ b, T* __restrict__ x, int colour,
                                                       int zero_init, int L, int nseg, int cpb) {
    k_zline_seg_mem_d<T>(PF_BLK, g, A, aux, b, x, colour, zero_init, L, nseg, cpb);
}
template <class T>
struct F_k_zline_seg_mem {
    static constexpr int kLB = 256;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_zline_seg_mem_d<T>(wg, a...);
    }
};

// b_i - (A x)_i of one cell of a colour-split level, or 0 when !v (slot
// arithmetic of the split layout: x/y neighbours in the other colour's
// half, z neighbours one layer of hx*ny slots away).  Branch-free: the
// loads come from a valid cell (ifb when !v, the cell itself for a missing
// neighbour) and are masked by selects, so a caller's unrolled loop over
// cells issues all of them together.
template <class T>
__device__ __forceinline__ T cell_residual(const Dims& f, int64_t half, int hx, const T* __restrict__ A,
                                           const T* __restrict__ x, const T* __restrict__ b, bool v, int c, int ix,
                                           int iy, int iz, int64_t ifb) {
    const int64_t nf = 2 * half, lstr = (int64_t)hx * f.ny;
    const int64_t i = v ? c * half + ((int64_t)iz * f.ny + iy) * hx + (ix >> 1) : ifb;
    const int64_t dother = c ? -half : half;
    const bool xm = v && ix > 0, xp = v && ix + 1 < f.nx, ym = v && iy > 0, yp = v && iy + 1 < f.ny;
    const bool zm = v && iz > 0, zp = v && iz + 1 < f.nz;
    const int odd = ix & 1;
    const int64_t jxm = xm ? i + dother - (1 - odd) : i, jxp = xp ? i + dother + odd : i;
    const int64_t jym = ym ? i + dother - hx : i, jyp = yp ? i + dother + hx : i;
    const int64_t jzm = zm ? i - lstr : i, jzp = zp ? i + lstr : i;
    const T a0 = A[i], a1 = A[nf + i], a2 = A[2 * nf + i], a3 = A[3 * nf + i], a4 = A[4 * nf + i];
    const T a5 = A[5 * nf + i], a6 = A[6 * nf + i];
    const T x0 = x[i], x1 = x[jxm], x2 = x[jxp], x3 = x[jym], x4 = x[jyp], x5 = x[jzm], x6 = x[jzp];
    T r = b[i] - a0 * x0;
    r -= (xm ? a1 * x1 : (T)0) + (xp ? a2 * x2 : (T)0) + (ym ? a3 * x3 : (T)0) + (yp ? a4 * x4 : (T)0);
    r -= (zm ? a5 * x5 : (T)0) + (zp ? a6 * x6 : (T)0);
    return v ? r : (T)0;
}

// The residual of a cell of the column colour c after one z-line sweep from
// x = 0 (colour c ^ 1's half-sweep being the last): colour c's half-sweep
// solved its rows with zero lateral neighbours, so b - A x there is minus the
// lateral couplings times the other colour's new values alone (lateral
// neighbours of a column are of the other colour; the column's own rows were
// solved exactly, up to rounding).  Four coefficients and four neighbour
// values instead of seven, b and the column's values.
template <class T>
__device__ __forceinline__ T cell_residual_lateral(const Dims& f, int64_t half, int hx, const T* __restrict__ A,
                                                   const T* __restrict__ x, bool v, int c, int ix, int iy, int iz,
                                                   int64_t ifb) {
    const int64_t nf = 2 * half;
    const int64_t i = v ? c * half + ((int64_t)iz * f.ny + iy) * hx + (ix >> 1) : ifb;
    const int64_t dother = c ? -half : half;
    const bool xm = v && ix > 0, xp = v && ix + 1 < f.nx, ym = v && iy > 0, yp = v && iy + 1 < f.ny;
    const int odd = ix & 1;
    const int64_t jxm = xm ? i + dother - (1 - odd) : i, jxp = xp ? i + dother + odd : i;
    const int64_t jym = ym ? i + dother - hx : i, jyp = yp ? i + dother + hx : i;
    const T a1 = A[nf + i], a2 = A[2 * nf + i], a3 = A[3 * nf + i], a4 = A[4 * nf + i];
    const T x1 = x[jxm], x2 = x[jxp], x3 = x[jym], x4 = x[jyp];
    const T r = -((xm ? a1 * x1 : (T)0) + (xp ? a2 * x2 : (T)0) + (ym ? a3 * x3 : (T)0) + (yp ? a4 * x4 : (T)0));
    return v ? r : (T)0;
}
template <class T, bool LAT>
__device__ __forceinline__ T kept_residual(const Dims& f, int64_t half, int hx, const T* __restrict__ A,
                                           const T* __restrict__ x, const T* __restrict__ b, bool v, int c, int ix,
                                           int iy, int iz, int64_t ifb) {
    if constexpr (LAT) return cell_residual_lateral(f, half, hx, A, x, v, c, ix, iy, iz, ifb);
    else return cell_residual(f, half, hx, A, x, b, v, c, ix, iy, iz, ifb);
}

// Fine residual b - A x summed over each aggregate (restriction = P^T).
// Cells of the column colour zero_colour ((ix+iy)&1) are taken as zero: a
// z-line half-sweep of that colour has just solved their rows exactly (-1:
// every cell computed).  With 2x2 lateral aggregates (even origins) the
// kept colour is the diagonal pair (dx, dy) = (p, p ^ zero_colour ^ 1); RB
// selects that form (instantiated apart so each keeps its own registers).
// LAT: the pre-smoothing was one sweep from x = 0, and the kept cells'
// residuals are their lateral terms alone (cell_residual_lateral).
template <class T, bool RB, bool LAT>
__device__ __forceinline__ T resid_restrict_one(const Dims& f, const Dims& c, int cx, int cy, int cz,
                                                const T* __restrict__ A, const T* __restrict__ x,
                                                const T* __restrict__ b, int64_t I, int zero_colour,
                                                int64_t& Ic) {
    // f is colour-split (a smoothed level)
    const int hx = (f.nx + 1) >> 1;
    const int64_t half = lv_half(f);
    const int64_t cxy = (int64_t)c.nx * c.ny;
    const int IZ = (int)(I / cxy);
    const int64_t rem = I - IZ * cxy;
    const int IY = (int)(rem / c.nx);
    const int IX = (int)(rem - (int64_t)IY * c.nx);
    const int64_t ifb = lv_index(f, IX * cx, IY * cy, IZ * cz);
    T s = 0;
    if constexpr (RB) {
        // cz is 1 or 2: the dz = 1 cells only when the aggregate has them
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int p = q;
            const int iz = IZ * cz, iy = IY * 2 + (p ^ zero_colour ^ 1), ix = IX * 2 + p;
            const bool v = iz < f.nz && iy < f.ny && ix < f.nx;
            s += kept_residual<T, LAT>(f, half, hx, A, x, b, v, zero_colour ^ 1, ix, iy, iz, ifb);
        }
        if (cz == 2) {
#pragma unroll
            for (int q = 2; q < 4; ++q) {
                const int p = q & 1;
                const int iz = IZ * cz + 1, iy = IY * 2 + (p ^ zero_colour ^ 1), ix = IX * 2 + p;
                const bool v = iz < f.nz && iy < f.ny && ix < f.nx;
                s += kept_residual<T, LAT>(f, half, hx, A, x, b, v, zero_colour ^ 1, ix, iy, iz, ifb);
            }
        }
    } else {
        // any factors: the 8 candidate cells one at a time (few registers)
#pragma unroll 1
        for (int q = 0; q < 8; ++q) {
            const int dz = q >> 2, dy = (q >> 1) & 1, dx = q & 1;
            const int iz = IZ * cz + dz, iy = IY * cy + dy, ix = IX * cx + dx;
            const bool v = dz < cz && dy < cy && dx < cx && iz < f.nz && iy < f.ny && ix < f.nx &&
                           ((ix + iy) & 1) != zero_colour;
            if (v) s += kept_residual<T, LAT>(f, half, hx, A, x, b, v, (ix + iy) & 1, ix, iy, iz, ifb);
        }
    }
    Ic = lv_index(c, IX, IY, IZ);
    return s;
}

template <class T, bool RB, bool LAT>
__device__ __forceinline__ void k_resid_restrict_d(const Blk& wg, Dims f, Dims c, int cx, int cy, int cz,
                                                   const T* __restrict__ A, const T* __restrict__ x,
                                                   const T* __restrict__ b, T* __restrict__ bc, int zero_colour) {
    const int64_t nc = (int64_t)c.nx * c.ny * c.nz;
    const int64_t I = xcd_block(wg) * blockDim.x + threadIdx.x;
    if (I >= nc) return;
    int64_t Ic;
    const T s = resid_restrict_one<T, RB, LAT>(f, c, cx, cy, cz, A, x, b, I, zero_colour, Ic);
    bc[Ic] = s;
}
template <class T, bool RB, bool LAT>
__global__ __launch_bounds__(256) void k_resid_restrict(Dims f, Dims c, int cx, int cy, int cz,
                                                        const T* __restrict__ A, const T* __restrict__ x,
                                                        const T* __restrict__ b, T* __restrict__ bc,
                                                        int zero_colour) {
    k_resid_restrict_d<T, RB, LAT>(PF_BLK, f, c, cx, cy, cz, A, x, b, bc, zero_colour);
}
template <class T, bool RB, bool LAT>
struct F_k_resid_restrict {
    static constexpr int kLB = 256;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_resid_restrict_d<T, RB, LAT>(wg, a...);
    }
};

template <class T>
__device__ __forceinline__ void k_prolong_add_d(const Blk& wg, Dims f, Dims c, int cx, int cy, int cz,
                                                const T* __restrict__ xc, T* __restrict__ x) {
    const int64_t nf = (int64_t)f.nx * f.ny * f.nz;
    const int64_t i = (int64_t)wg.x * blockDim.x + threadIdx.x;
    if (i >= nf) return;
    int ix, iy, iz;
    cell_coords(f, i, ix, iy, iz);
    x[lv_index(f, ix, iy, iz)] += xc[lv_index(c, ix / cx, iy / cy, iz / cz)];
}
template <class T>
__global__ void k_prolong_add(Dims f, Dims c, int cx, int cy, int cz, const T* __restrict__ xc, T* __restrict__ x) {
    k_prolong_add_d<T>(PF_BLK, f, c, cx, cy, cz, xc, x);
}
template <class T>
struct F_k_prolong_add {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_prolong_add_d<T>(wg, a...);
    }
};

// Level-0 pressure in natural cell order from the level's slots.
template <class T>
__device__ __forceinline__ void k_gather_p_d(const Blk& wg, Dims g, const T* __restrict__ x, T* __restrict__ p) {
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int64_t i = xcd_block(wg) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int ix, iy, iz;
    cell_coords(g, i, ix, iy, iz);
    p[i] = x[lv_index(g, ix, iy, iz)];
}
template <class T>
__global__ void k_gather_p(Dims g, const T* __restrict__ x, T* __restrict__ p) {
    k_gather_p_d<T>(PF_BLK, g, x, p);
}
template <class T>
struct F_k_gather_p {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_gather_p_d<T>(wg, a...);
    }
};

// Prolongation through every level at once, for V-cycles without
// post-smoothing: x_0 += P_0 (x_1 + P_1 (x_2 + ...)).  Box aggregation with
// factors 1 or 2 per direction composes to shifts (floor(floor(i/2)/2) =
// i >> 2), so a level-0 cell reads its aggregate on every coarser level.
// Summed from the coarsest level down, as the nested form associates.  With
// p given, the sum goes to p in natural cell order instead of back into x_0
// (the last cycle).
constexpr int kMaxChain = 32;
struct ProlongChain {
    int nl;
    int sx[kMaxChain], sy[kMaxChain], sz[kMaxChain];
    Dims d[kMaxChain];
    const void* x[kMaxChain];
};

// NL > 0: exactly NL levels, the level loop unrolled so that every level's
// load issues at once; NL == 0: pc.nl levels.
template <class T, int NL>
__device__ __forceinline__ void k_prolong_chain_d(const Blk& wg, Dims f, ProlongChain pc, T* __restrict__ x,
                                                  T* __restrict__ p) {
    const int64_t nf = (int64_t)f.nx * f.ny * f.nz;
    const int64_t i = xcd_block(wg) * blockDim.x + threadIdx.x;
    if (i >= nf) return;
    int ix, iy, iz;
    cell_coords(f, i, ix, iy, iz);
    T sum = 0;
    if constexpr (NL > 0) {
        T v[NL > 0 ? NL : 1];
#pragma unroll
        for (int l = 1; l < NL; ++l)
            v[l] = static_cast<const T*>(pc.x[l])[lv_index(pc.d[l], ix >> pc.sx[l], iy >> pc.sy[l], iz >> pc.sz[l])];
#pragma unroll
        for (int l = NL - 1; l >= 1; --l) sum = v[l] + sum;
    } else {
        for (int l = pc.nl - 1; l >= 1; --l) {
            const int64_t I = lv_index(pc.d[l], ix >> pc.sx[l], iy >> pc.sy[l], iz >> pc.sz[l]);
            sum = static_cast<const T*>(pc.x[l])[I] + sum;
        }
    }
    const int64_t j = lv_index(f, ix, iy, iz);
    if (p) p[i] = x[j] + sum;
    else x[j] += sum;
}
template <class T, int NL>
__global__ void k_prolong_chain(Dims f, ProlongChain pc, T* __restrict__ x, T* __restrict__ p) {
    k_prolong_chain_d<T, NL>(PF_BLK, f, pc, x, p);
}
template <class T, int NL>
struct F_k_prolong_chain {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_prolong_chain_d<T, NL>(wg, a...);
    }
};

// Dense coarsest matrix (row-major, augmented with the identity: n x 2n).
__device__ __forceinline__ void k_coarse_build_d(const Blk& wg, Dims g, const double* __restrict__ A,
                                                 double* __restrict__ M) {
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int64_t r = (int64_t)wg.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int64_t W = 2 * n;
    double* row = M + r * W;
    for (int64_t c = 0; c < W; ++c) row[c] = 0.0;
    row[n + r] = 1.0;
    const int64_t gxy = (int64_t)g.nx * g.ny;
    const int iz = (int)(r / gxy);
    const int64_t rem = r - iz * gxy;
    const int iy = (int)(rem / g.nx);
    const int ix = (int)(rem - (int64_t)iy * g.nx);
    row[r] = A[r];
    if (ix > 0) row[r - 1] += A[n + r];
    if (ix + 1 < g.nx) row[r + 1] += A[2 * n + r];
    if (iy > 0) row[r - g.nx] += A[3 * n + r];
    if (iy + 1 < g.ny) row[r + g.nx] += A[4 * n + r];
    if (iz > 0) row[r - gxy] += A[5 * n + r];
    if (iz + 1 < g.nz) row[r + gxy] += A[6 * n + r];
}
__global__ void k_coarse_build(Dims g, const double* __restrict__ A, double* __restrict__ M) {
    k_coarse_build_d(PF_BLK, g, A, M);
}
struct F_k_coarse_build {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_coarse_build_d(wg, a...);
    }
};

// Gauss-Jordan with partial pivoting on the augmented matrix, one block.
__device__ __forceinline__ void k_gauss_jordan_d(const Blk& wg, int n, double* __restrict__ M) {
    __shared__ double fcol[1024];
    __shared__ double rv[16];
    __shared__ int ri[16];
    __shared__ int piv;
    const int W = 2 * n;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int k = 0; k < n; ++k) {
        double best = -1.0;
        int bi = k;
        for (int r = k + tid; r < n; r += nt) {
            const double v = fabs(M[(int64_t)r * W + k]);
            if (v > best) { best = v; bi = r; }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double ob = __shfl_down(best, o, 64);
            const int oi = __shfl_down(bi, o, 64);
            if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        if ((tid & 63) == 0) { rv[tid >> 6] = best; ri[tid >> 6] = bi; }
        __syncthreads();
        if (tid == 0) {
            double b = rv[0];
            int p = ri[0];
            for (int q = 1; q < (nt >> 6); ++q)
                if (rv[q] > b || (rv[q] == b && ri[q] < p)) { b = rv[q]; p = ri[q]; }
            piv = p;
        }
        __syncthreads();
        const int p = piv;
        if (p != k)
            for (int c = tid; c < W; c += nt) {
                const double a = M[(int64_t)k * W + c];
                M[(int64_t)k * W + c] = M[(int64_t)p * W + c];
                M[(int64_t)p * W + c] = a;
            }
        __syncthreads();
        const double inv = 1.0 / M[(int64_t)k * W + k];
        __syncthreads();
        for (int c = tid; c < W; c += nt) M[(int64_t)k * W + c] *= inv;
        for (int r = tid; r < n; r += nt) fcol[r] = (r == k) ? 0.0 : M[(int64_t)r * W + k];
        __syncthreads();
        for (int64_t idx = tid; idx < (int64_t)n * W; idx += nt) {
            const int r = (int)(idx / W);
            const int c = (int)(idx - (int64_t)r * W);
            const double f = fcol[r];
            if (f != 0.0) M[idx] -= f * M[(int64_t)k * W + c];
        }
        __syncthreads();
    }
}
__global__ __launch_bounds__(1024) void k_gauss_jordan(int n, double* __restrict__ M) {
    k_gauss_jordan_d(PF_BLK, n, M);
}
struct F_k_gauss_jordan {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_gauss_jordan_d(wg, a...);
    }
};


// Gauss-Jordan with partial pivoting in LDS for n <= kGJLds (augmented n x 2n
// matrix held in shared memory), result written back to M.
constexpr int kGJLds = 96;
__device__ __forceinline__ void k_gauss_jordan_lds_d(const Blk& wg, int n, double* __restrict__ M) {
    extern __shared__ double sm[];
    double* S = sm;                       // n x 2n
    double* fcol = sm + 2 * n * n;        // n
    __shared__ int piv;
    const int W = 2 * n;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wv = tid >> 6, nwv = nt >> 6;
    for (int idx = tid; idx < n * W; idx += nt) S[idx] = M[idx];
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        // pivot: largest |S[r][k]|, r >= k, by the first wavefront (ties to the lower row)
        if (wv == 0) {
            double best = -1.0;
            int p = k;
            for (int r = k + lane; r < n; r += 64) {
                const double v = fabs(S[r * W + k]);
                if (v > best) { best = v; p = r; }
            }
            for (int o = 32; o > 0; o >>= 1) {
                const double ob = __shfl_down(best, o, 64);
                const int op = __shfl_down(p, o, 64);
                if (lane + o < 64 && (ob > best || (ob == best && op < p))) { best = ob; p = op; }
            }
            if (lane == 0) piv = p;
        }
        __syncthreads();
        const int p = piv;
        // Rows k and p (>= k) are zero left of column k, so every row
        // operation of this step touches columns k .. W-1 only.
        // read phase: rows k and p (thread per column) and column k (thread per row)
        const double akk = S[k * W + k];
        const double inv = 1.0 / S[p * W + k];
        const int c0 = k + tid;
        double ak = 0.0, ap = 0.0, fr = 0.0;
        if (c0 < W) {
            ak = S[k * W + c0];
            ap = S[p * W + c0];
        }
        if (tid < n) fr = S[tid * W + k];
        __syncthreads();
        // write phase: swap rows k and p, scale the new pivot row, multipliers
        if (c0 < W) {
            S[p * W + c0] = ak;
            S[k * W + c0] = ap * inv;
        }
        if (tid < n) fcol[tid] = tid == k ? 0.0 : (tid == p ? akk : fr);
        __syncthreads();
        // eliminate column k from every other row: wavefront per row, lanes
        // over columns, the pivot row held in registers
        double pk[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int c = k + lane + 64 * q;
            pk[q] = c < W ? S[k * W + c] : 0.0;
        }
        for (int r = wv; r < n; r += nwv) {
            const double f = fcol[r];
            if (f != 0.0) {
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    const int c = k + lane + 64 * q;
                    if (c < W) S[r * W + c] -= f * pk[q];
                }
            }
        }
        __syncthreads();
    }
    for (int idx = tid; idx < n * W; idx += nt) M[idx] = S[idx];
}
__global__ __launch_bounds__(1024) void k_gauss_jordan_lds(int n, double* __restrict__ M) {
    k_gauss_jordan_lds_d(PF_BLK, n, M);
}
struct F_k_gauss_jordan_lds {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_gauss_jordan_lds_d(wg, a...);
    }
};

// The inverse (right half of the reduced augmented matrix) in compact n x n
// form, in FP64 and FP32.
__device__ __forceinline__ void k_compact_inv_d(const Blk& wg, int n, const double* __restrict__ M,
                                                double* __restrict__ inv, float* __restrict__ inv32) {
    const int64_t idx = (int64_t)wg.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * n) return;
    const int64_t r = idx / n, c = idx - r * n;
    const double v = M[r * 2 * n + n + c];
    inv[idx] = v;
    if (inv32) inv32[idx] = (float)v;
}
__global__ void k_compact_inv(int n, const double* __restrict__ M, double* __restrict__ inv,
                              float* __restrict__ inv32) {
    k_compact_inv_d(PF_BLK, n, M, inv, inv32);
}
struct F_k_compact_inv {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_compact_inv_d(wg, a...);
    }
};

// x = Minv b with the compact (n x n) coarsest inverse: one wavefront per
// row, lanes over the columns, fixed-order shuffle reduction.
template <class T>
__device__ __forceinline__ void k_coarse_apply_d(const Blk& wg, int n, const T* __restrict__ Minv,
                                                 const T* __restrict__ b, T* __restrict__ x) {
    const int r = wg.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= n) return;
    const T* row = Minv + (int64_t)r * n;
    T s = 0;
    for (int c = lane; c < n; c += 64) s += row[c] * b[c];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if (lane == 0) x[r] = s;
}
template <class T>
__global__ __launch_bounds__(256) void k_coarse_apply(int n, const T* __restrict__ Minv, const T* __restrict__ b,
                                                      T* __restrict__ x) {
    k_coarse_apply_d<T>(PF_BLK, n, Minv, b, x);
}
template <class T>
struct F_k_coarse_apply {
    static constexpr int kLB = 256;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_coarse_apply_d<T>(wg, a...);
    }
};

// Pressure restriction: water + oil residual of each cell, into the slots
// of level 0.
// The colour-split vector layout (pf_internal.h) on the finest grid's Dims:
// slots per colour and the plane offset of a cell.
__device__ __forceinline__ int64_t cs_half(const Dims& g) { return (int64_t)((g.nx + 1) >> 1) * g.ny * g.nz; }
__device__ __forceinline__ int64_t cs_offset(const Dims& g, int ix, int iy, int iz) {
    return ((ix + iy + iz) & 1) * cs_half(g) + ((int64_t)iy + (int64_t)g.ny * iz) * ((g.nx + 1) >> 1) + (ix >> 1);
}

template <class T>
__device__ __forceinline__ void k_restrict_p_d(const Blk& wg, Dims g, const double* __restrict__ v, T* __restrict__ b,
                                               int cs) {
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int64_t i = xcd_block(wg) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int ix, iy, iz;
    cell_coords(g, i, ix, iy, iz);
    const int64_t vi = cs ? cs_offset(g, ix, iy, iz) : i;
    const int64_t pl = cs ? 2 * cs_half(g) : n;
    b[lv_index(g, ix, iy, iz)] = (T)(v[vi] + v[pl + vi]);
}
template <class T>
__global__ void k_restrict_p(Dims g, const double* __restrict__ v, T* __restrict__ b, int cs) {
    k_restrict_p_d<T>(PF_BLK, g, v, b, cs);
}
template <class T>
struct F_k_restrict_p {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_restrict_p_d<T>(wg, a...);
    }
};

// The same restriction fused with the first half-sweep of the first V-cycle
// (colour 0 from x = 0), which needs only the right-hand side of its own
// columns.  The launch is that half-sweep's (level 0, colour 0); thread
// (segment, slot) forms b on the layers of its segment in both columns of
// its slot (one of each colour, so every cell is visited once), stores both
// and sweeps its colour-0 column from the values in its registers.
template <int LMAX, class T>
__device__ __forceinline__ void k_restrict_p_zline_d(const Blk& wg, Dims g, const double* __restrict__ v,
                                                     const T* __restrict__ A, const T* __restrict__ aux,
                                                     T* __restrict__ b, T* __restrict__ x, int L, int nseg, int cpb,
                                                     int cs) {
    __shared__ T sA[1024];
    __shared__ T sB[1024];
    const int t = threadIdx.x;
    const int seg = t / cpb, c = t - seg * cpb;
    const int hx = (g.nx + 1) >> 1;
    const int64_t col0 = xcd_block(wg) * cpb;
    const int64_t tcol = col0 + c;
    T bin[LMAX];
#pragma unroll
    for (int j = 0; j < LMAX; ++j) bin[j] = 0;
    if (seg < nseg && tcol < (int64_t)hx * g.ny) {
        const int tc = (int)tcol;
        const int iy = tc / hx;
        const int ixh = tc - iy * hx;
        const int64_t half = lv_half(g), lstr = (int64_t)hx * g.ny;
        const int64_t n = cs ? 2 * cs_half(g) : (int64_t)g.nx * g.ny * g.nz;
        const int k0 = seg * L;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int ix = 2 * ixh + ((iy + q) & 1);
            if (ix >= g.nx) continue;
#pragma unroll
            for (int j = 0; j < LMAX; ++j) {
                const int iz = k0 + j;
                if (j < L && iz < g.nz) {
                    const int64_t i = cs ? cs_offset(g, ix, iy, iz) : ix + (int64_t)g.nx * (iy + (int64_t)g.ny * iz);
                    const T r = (T)(v[i] + v[n + i]);
                    b[q * half + tcol + (int64_t)iz * lstr] = r;
                    if (q == 0) bin[j] = r;
                }
            }
        }
    }
    zline_seg_body<LMAX, T, true, true>(g, A, aux, b, x, 0, L, nseg, cpb, col0, t, sA, sB, bin);
}
template <int LMAX, class T>
__global__ __launch_bounds__(1024) void k_restrict_p_zline(Dims g, const double* __restrict__ v,
                                                           const T* __restrict__ A, const T* __restrict__ aux,
                                                           T* __restrict__ b, T* __restrict__ x, int L, int nseg,
                                                           int cpb, int cs) {
    k_restrict_p_zline_d<LMAX, T>(PF_BLK, g, v, A, aux, b, x, L, nseg, cpb, cs);
}
template <int LMAX, class T>
struct F_k_restrict_p_zline {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_restrict_p_zline_d<LMAX, T>(wg, a...);
    }
};

// Well bottom-hole pressures of the pressure stage from the well rows vw of
// v: pb_w = (v_w - sum_perf dW/dP * p_cell) / D_w.  One 64-lane block per well.
template <class T>
__device__ __forceinline__ void k_well_pb_d(const Blk& wg, DevModel m, const int32_t* __restrict__ wp_first,
                                            const int32_t* __restrict__ wp_idx, const int32_t* __restrict__ perf_cell,
                                            const double* __restrict__ Cw, const double* __restrict__ Dw,
                                            const double* __restrict__ vw, const T* __restrict__ p,
                                            double* __restrict__ pb) {
    const int w = wg.x;
    double s = 0.0;
    for (int k = wp_first[w] + (int)threadIdx.x; k < wp_first[w + 1]; k += 64) {
        const int q = wp_idx[k];
        s += Cw[3 * q] * (double)p[perf_cell[q]];
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if (threadIdx.x == 0) pb[w] = (vw[w] - s) / Dw[w];
}
template <class T>
__global__ __launch_bounds__(64) void k_well_pb(DevModel m, const int32_t* __restrict__ wp_first,
                                                const int32_t* __restrict__ wp_idx,
                                                const int32_t* __restrict__ perf_cell, const double* __restrict__ Cw,
                                                const double* __restrict__ Dw, const double* __restrict__ vw,
                                                const T* __restrict__ p, double* __restrict__ pb) {
    k_well_pb_d<T>(PF_BLK, m, wp_first, wp_idx, perf_cell, Cw, Dw, vw, p, pb);
}
template <class T>
struct F_k_well_pb {
    static constexpr int kLB = 64;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_well_pb_d<T>(wg, a...);
    }
};

// t = v - J * Pi_p(p, pb) on the cells: only the P-columns of the blocks.
// NT: stream the P-columns past the caches (where nothing after the stage
// reads J in natural order).
template <bool NT, class T> __device__ __forceinline__ T jp_ld(const T* q) {
    if constexpr (NT) return __builtin_nontemporal_load(q);
    else return *q;
}

// One cell, FP64 (J: 63 planes) ...
template <bool NT = false>
__device__ __forceinline__ void stage_resid_cell(const DevModel& m, const double* __restrict__ J,
                                                 const double* __restrict__ v, const double* __restrict__ p,
                                                 int64_t i, int64_t ix, int64_t iy, int64_t iz, double& t0,
                                                 double& t1, double& t2) {
    const int64_t n = m.n;
    const double pi = p[i];
    t0 = v[i] - jp_ld<NT>(J + 0 * n + i) * pi;
    t1 = v[n + i] - jp_ld<NT>(J + 3 * n + i) * pi;
    t2 = v[2 * n + i] - jp_ld<NT>(J + 6 * n + i) * pi;
    const bool ex[6] = {ix > 0, ix + 1 < m.nx, iy > 0, iy + 1 < m.ny, iz > 0, iz + 1 < m.nz};
    const int64_t off[6] = {-1, 1, -(int64_t)m.nx, (int64_t)m.nx, -m.nxy, m.nxy};
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        if (!ex[f]) continue;
        const double pj = p[i + off[f]];
        const double* B = J + (int64_t)(f + 1) * 9 * n + i;
        t0 -= jp_ld<NT>(B + 0 * n) * pj;
        t1 -= jp_ld<NT>(B + 3 * n) * pj;
        t2 -= jp_ld<NT>(B + 6 * n) * pj;
    }
}

// ... and FP32 (Jp: the 21 FP32 P-column planes, FP32 accumulation).
template <bool NT = false>
__device__ __forceinline__ void stage_resid_cell(const DevModel& m, const float* __restrict__ Jp,
                                                 const double* __restrict__ v, const float* __restrict__ p,
                                                 int64_t i, int64_t ix, int64_t iy, int64_t iz, float& t0,
                                                 float& t1, float& t2) {
    const int64_t n = m.n;
    const float pi = p[i];
    t0 = (float)v[i] - jp_ld<NT>(Jp + 0 * n + i) * pi;
    t1 = (float)v[n + i] - jp_ld<NT>(Jp + 1 * n + i) * pi;
    t2 = (float)v[2 * n + i] - jp_ld<NT>(Jp + 2 * n + i) * pi;
    const bool ex[6] = {ix > 0, ix + 1 < m.nx, iy > 0, iy + 1 < m.ny, iz > 0, iz + 1 < m.nz};
    const int64_t off[6] = {-1, 1, -(int64_t)m.nx, (int64_t)m.nx, -m.nxy, m.nxy};
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        if (!ex[f]) continue;
        const float pj = p[i + off[f]];
        const float* B = Jp + (int64_t)(f + 1) * 3 * n + i;
        t0 -= jp_ld<NT>(B + 0 * n) * pj;
        t1 -= jp_ld<NT>(B + 1 * n) * pj;
        t2 -= jp_ld<NT>(B + 2 * n) * pj;
    }
}

// The stage residual over the cells, FP64 (TJ = double, J) or FP32
// (TJ = float, Jp).
template <class TJ, class T>
__device__ __forceinline__ void k_stage_resid_d(const Blk& wg, DevModel m, const TJ* __restrict__ J,
                                                const double* __restrict__ v, const T* __restrict__ p,
                                                T* __restrict__ t) {
    const int64_t i = xcd_block(wg) * blockDim.x + threadIdx.x;
    if (i >= m.n) return;
    const int64_t n = m.n;
    const int64_t iz = i / m.nxy;
    const int64_t rem = i - iz * m.nxy;
    const int64_t iy = rem / m.nx;
    const int64_t ix = rem - iy * m.nx;
    T t0, t1, t2;
    stage_resid_cell(m, J, v, p, i, ix, iy, iz, t0, t1, t2);
    t[i] = t0;
    t[n + i] = t1;
    t[2 * n + i] = t2;
}
template <class TJ, class T>
__global__ __launch_bounds__(256) void k_stage_resid(DevModel m, const TJ* __restrict__ J,
                                                     const double* __restrict__ v, const T* __restrict__ p,
                                                     T* __restrict__ t) {
    k_stage_resid_d<TJ, T>(PF_BLK, m, J, v, p, t);
}
template <class TJ, class T>
struct F_k_stage_resid {
    static constexpr int kLB = 256;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_stage_resid_d<TJ, T>(wg, a...);
    }
};

// Border part of the stage residual: perforated cells subtract B * pb; the
// well rows are exactly satisfied by pb (their residual is 0).
template <class T>
__device__ __forceinline__ void k_stage_resid_border_d(const Blk& wg, DevModel m, const int32_t* __restrict__ pc_cell,
                                                       const int32_t* __restrict__ pc_first,
                                                       const int32_t* __restrict__ perf_well,
                                                       const double* __restrict__ B, const double* __restrict__ pb,
                                                       T* __restrict__ t) {
    const int64_t k = (int64_t)wg.x * blockDim.x + threadIdx.x;
    const int64_t n = m.n;
    if (k < m.npc) {
        const int64_t i = pc_cell[k];
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        for (int64_t q = pc_first[k]; q < pc_first[k + 1]; ++q) {
            const double v = pb[perf_well[q]];
            a0 += B[3 * q] * v;
            a1 += B[3 * q + 1] * v;
            a2 += B[3 * q + 2] * v;
        }
        t[i] = (T)(t[i] - a0);
        t[n + i] = (T)(t[n + i] - a1);
        t[2 * n + i] = (T)(t[2 * n + i] - a2);
    } else if (k < m.npc + m.nw) {
        t[3 * n + (k - m.npc)] = 0;
    }
}
template <class T>
__global__ void k_stage_resid_border(DevModel m, const int32_t* __restrict__ pc_cell,
                                     const int32_t* __restrict__ pc_first, const int32_t* __restrict__ perf_well,
                                     const double* __restrict__ B, const double* __restrict__ pb, T* __restrict__ t) {
    k_stage_resid_border_d<T>(PF_BLK, m, pc_cell, pc_first, perf_well, B, pb, t);
}
template <class T>
struct F_k_stage_resid_border {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_stage_resid_border_d<T>(wg, a...);
    }
};

// z = Dinv t (block Jacobi on cells, 1/D on wells) + Pi_p(p, pb)
__device__ __forceinline__ void k_bjac_apply_add_d(const Blk& wg, int64_t n, int nw, const double* __restrict__ Dinv,
                                                   const double* __restrict__ Dw, const double* __restrict__ t,
                                                   const double* __restrict__ p, const double* __restrict__ pb,
                                                   double* __restrict__ z) {
    const int64_t i = (int64_t)wg.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const double a = t[i], b = t[n + i], c = t[2 * n + i];
        z[i] = Dinv[0 * n + i] * a + Dinv[1 * n + i] * b + Dinv[2 * n + i] * c + (p ? p[i] : 0.0);
        z[n + i] = Dinv[3 * n + i] * a + Dinv[4 * n + i] * b + Dinv[5 * n + i] * c;
        z[2 * n + i] = Dinv[6 * n + i] * a + Dinv[7 * n + i] * b + Dinv[8 * n + i] * c;
    } else if (i < n + nw) {
        const int w = (int)(i - n);
        z[3 * n + w] = t[3 * n + w] / Dw[w] + (pb ? pb[w] : 0.0);
    }
}
__global__ void k_bjac_apply_add(int64_t n, int nw, const double* __restrict__ Dinv, const double* __restrict__ Dw,
                                 const double* __restrict__ t, const double* __restrict__ p,
                                 const double* __restrict__ pb, double* __restrict__ z) {
    k_bjac_apply_add_d(PF_BLK, n, nw, Dinv, Dw, t, p, pb, z);
}
struct F_k_bjac_apply_add {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_bjac_apply_add_d(wg, a...);
    }
};

// z += Pi_p(p, pb)
template <class T>
__device__ __forceinline__ void k_add_pressure_d(const Blk& wg, int64_t n, int nw, const T* __restrict__ p,
                                                 const double* __restrict__ pb, T* __restrict__ z) {
    const int64_t i = (int64_t)wg.x * blockDim.x + threadIdx.x;
    if (i < n) z[i] += p[i];
    else if (i < n + nw) z[3 * n + (i - n)] = (T)(z[3 * n + (i - n)] + pb[i - n]);
}
template <class T>
__global__ void k_add_pressure(int64_t n, int nw, const T* __restrict__ p, const double* __restrict__ pb,
                               T* __restrict__ z) {
    k_add_pressure_d<T>(PF_BLK, n, nw, p, pb, z);
}
template <class T>
struct F_k_add_pressure {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_add_pressure_d<T>(wg, a...);
    }
};

// ---- red-black block ILU(0) -------------------------------------------------
// Cells are coloured red ((ix+iy+iz) even) and black.  In red-black order
// the red-red and black-black blocks of J are block diagonal, so ILU(0)
// keeps D_r for red cells and the modified black diagonal
//   D~_b = D_b - sum_{r nb of b} J_br D_r^{-1} J_rb
// (fill between distinct black cells is dropped).  Apply:
//   y_r = D_r^{-1} f_r;  y_b = D~_b^{-1} (f_b - sum J_br y_r);
//   z_b = y_b;          z_r = y_r - D_r^{-1} sum J_rb z_b.
__device__ __forceinline__ void inv3(const double a[9], double r[9]) {
    const double c00 = a[4] * a[8] - a[5] * a[7];
    const double c01 = a[5] * a[6] - a[3] * a[8];
    const double c02 = a[3] * a[7] - a[4] * a[6];
    const double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
    const double id = 1.0 / det;
    r[0] = c00 * id;
    r[1] = (a[2] * a[7] - a[1] * a[8]) * id;
    r[2] = (a[1] * a[5] - a[2] * a[4]) * id;
    r[3] = c01 * id;
    r[4] = (a[0] * a[8] - a[2] * a[6]) * id;
    r[5] = (a[2] * a[3] - a[0] * a[5]) * id;
    r[6] = c02 * id;
    r[7] = (a[1] * a[6] - a[0] * a[7]) * id;
    r[8] = (a[0] * a[4] - a[1] * a[3]) * id;
}

__device__ __forceinline__ void decode(const DevModel& m, int64_t i, int64_t& ix, int64_t& iy, int64_t& iz) {
    iz = i / m.nxy;
    const int64_t rem = i - iz * m.nxy;
    iy = rem / m.nx;
    ix = rem - iy * m.nx;
}

// ---- red-black block ILU(0) on colour-split storage ---------------------
// Cell colour c = (ix+iy+iz)&1.  Each colour's cells of one x-line take the
// slots line*nxh + (ix>>1) with nxh = ceil(nx/2) (one pad slot on lines
// where the colour has floor(nx/2) cells), so a phase that works on one
// colour streams contiguous factor storage instead of every other element.
//   Dc[(c*9 + e)*ns + s]        inverse (modified) diagonal blocks, FP64
//   Lc[(c*54 + q*9 + e)*ns + s] off-diagonal blocks q = 0..5 (-x..+z)
//   Jdc[(c*9 + e)*ns + s]       diagonal blocks of J (FP64 ILU), so that the
//                               product w = J z can stream colour-split storage
// Entry e = 5 (oil row, C column) of every block of J is zero: the oil
// equation does not involve the polymer concentration (polymer is carried
// by the water phase, Sec. 2), and the assembly writes 0 there.  The kernels
// that stream J or its copies (Lc, Jdc, the BF16 copy) skip that plane.
__device__ __forceinline__ int64_t ilu_nxh(const DevModel& m) { return (m.nx + 1) >> 1; }
__device__ __forceinline__ int64_t ilu_slots(const DevModel& m) { return ilu_nxh(m) * m.ny * m.nz; }

// slot s of colour c -> cell coordinates; false for a pad slot
// Thread order of the one-colour kernels of the smoother and the product on
// grids with large layers (at least kStripLayer slots of a colour): y-strips
// (strip_order), so a slot's neighbours one layer up or down were read one
// strip-layer earlier rather than one whole layer of the grid earlier
// (300^3: +2 % end to end; on layers of 6,600 and 20,000 slots it was 1-2 %
// slower, so those keep the plain order).  Which thread takes a slot does
// not change what is computed for it.  v is the thread's index, the result
// its slot (a bijection on [0, ilu_slots)).
constexpr int64_t kStripLayer = 32768;
__device__ __forceinline__ int64_t strip_slot(const DevModel& m, int64_t v) {
    const int64_t hx = ilu_nxh(m);
    if (hx * m.ny < kStripLayer) return v;
    return strip_order(v, hx, m.ny, m.nz);
}

__device__ __forceinline__ bool ilu_slot_cell(const DevModel& m, int c, int64_t s, int64_t& ix, int64_t& iy,
                                              int64_t& iz) {
    const uint32_t nxh = (uint32_t)ilu_nxh(m);
    const uint32_t line = (uint32_t)s / nxh;
    const uint32_t t = (uint32_t)s - line * nxh;
    iz = line / (uint32_t)m.ny;
    iy = line - (uint32_t)iz * (uint32_t)m.ny;
    ix = 2 * (int64_t)t + ((c + iy + iz) & 1);
    return ix < m.nx;
}

template <class T>
__device__ __forceinline__ void k_well_diag_d(const Blk& wg, int64_t n, int nw, const double* __restrict__ Dw,
                                              const T* __restrict__ f, T* __restrict__ z) {
    const int w = wg.x * blockDim.x + threadIdx.x;
    if (w < nw) z[3 * n + w] = (T)(f[3 * n + w] / Dw[w]);
}
template <class T>
__global__ void k_well_diag(int64_t n, int nw, const double* __restrict__ Dw, const T* __restrict__ f,
                            T* __restrict__ z) {
    k_well_diag_d<T>(PF_BLK, n, nw, Dw, f, z);
}
template <class T>
struct F_k_well_diag {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_well_diag_d<T>(wg, a...);
    }
};


// ---- reduced-precision copies for the mixed-precision preconditioner --------
// BF16 storage with round-to-nearest-even (the upper 16 bits of an IEEE
// single); all arithmetic on them is FP32.
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ void k_cast_f32_d(const Blk& wg, int64_t n, const double* __restrict__ src,
                                             float* __restrict__ dst) {
    for (int64_t i = (int64_t)wg.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)wg.n * blockDim.x)
        dst[i] = (float)src[i];
}
__global__ void k_cast_f32(int64_t n, const double* __restrict__ src, float* __restrict__ dst) {
    k_cast_f32_d(PF_BLK, n, src, dst);
}
struct F_k_cast_f32 {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_cast_f32_d(wg, a...);
    }
};

// Jp32[(d*3 + row)*n + i]: FP32 P-columns of the 7 blocks (stage residual).
__device__ __forceinline__ void k_extract_lowp_d(const Blk& wg, int64_t n, const double* __restrict__ J,
                                                 float* __restrict__ Jp32) {
    const int64_t i = (int64_t)wg.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int d = 0; d < 7; ++d)
        for (int r = 0; r < 3; ++r) Jp32[(int64_t)(d * 3 + r) * n + i] = (float)J[(int64_t)(d * 9 + 3 * r) * n + i];
}
__global__ void k_extract_lowp(int64_t n, const double* __restrict__ J, float* __restrict__ Jp32) {
    k_extract_lowp_d(PF_BLK, n, J, Jp32);
}
struct F_k_extract_lowp {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_extract_lowp_d(wg, a...);
    }
};


// The same stage residual with its border part and the first phase of the
// red-black ILU(0) in one pass (PF order): perforated cells subtract B pb
// (found through pc_map, cell -> perforated-cell index or -1, in the order
// of k_stage_resid_border); red cells go straight to y_r = D_r^{-1} t_r,
// which is all the later phases need of them; black cells keep t_b for the
// second phase; the well rows get t_w = 0.  The arithmetic of each step is
// that of the separate kernels.
template <class TJ, class T, class TD>
__device__ __forceinline__ void k_stage_ilu0_d(const Blk& wg, DevModel m, const TJ* __restrict__ J,
                                               const double* __restrict__ v, const T* __restrict__ p,
                                               const double* __restrict__ pb, const double* __restrict__ B,
                                               const int32_t* __restrict__ pc_map,
                                               const int32_t* __restrict__ pc_first,
                                               const int32_t* __restrict__ perf_well, const TD* __restrict__ Dc,
                                               T* __restrict__ t, T* __restrict__ z) {
    const int64_t i = xcd_block(wg) * blockDim.x + threadIdx.x;
    const int64_t n = m.n;
    if (i >= n) {
        if (i < n + m.nw) t[3 * n + (i - n)] = 0;
        return;
    }
    const int64_t iz = i / m.nxy;
    const int64_t rem = i - iz * m.nxy;
    const int64_t iy = rem / m.nx;
    const int64_t ix = rem - iy * m.nx;
    T t0, t1, t2;
    stage_resid_cell<true>(m, J, v, p, i, ix, iy, iz, t0, t1, t2);
    const int32_t k = pc_map[i];
    if (k >= 0) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        for (int64_t q = pc_first[k]; q < pc_first[k + 1]; ++q) {
            const double w = pb[perf_well[q]];
            a0 += B[3 * q] * w;
            a1 += B[3 * q + 1] * w;
            a2 += B[3 * q + 2] * w;
        }
        t0 = (T)(t0 - a0);
        t1 = (T)(t1 - a1);
        t2 = (T)(t2 - a2);
    }
    if (((ix + iy + iz) & 1) == 0) {
        const int64_t ns = ilu_slots(m);
        const TD* D = Dc + (iy + m.ny * iz) * ilu_nxh(m) + (ix >> 1);
        z[i] = D[0 * ns] * t0 + D[1 * ns] * t1 + D[2 * ns] * t2;
        z[n + i] = D[3 * ns] * t0 + D[4 * ns] * t1 + D[5 * ns] * t2;
        z[2 * n + i] = D[6 * ns] * t0 + D[7 * ns] * t1 + D[8 * ns] * t2;
    } else {
        t[i] = t0;
        t[n + i] = t1;
        t[2 * n + i] = t2;
    }
}
template <class TJ, class T, class TD>
__global__ __launch_bounds__(256) void k_stage_ilu0(DevModel m, const TJ* __restrict__ J,
                                                    const double* __restrict__ v, const T* __restrict__ p,
                                                    const double* __restrict__ pb, const double* __restrict__ B,
                                                    const int32_t* __restrict__ pc_map,
                                                    const int32_t* __restrict__ pc_first,
                                                    const int32_t* __restrict__ perf_well, const TD* __restrict__ Dc,
                                                    T* __restrict__ t, T* __restrict__ z) {
    k_stage_ilu0_d<TJ, T, TD>(PF_BLK, m, J, v, p, pb, B, pc_map, pc_first, perf_well, Dc, t, z);
}
template <class TJ, class T, class TD>
struct F_k_stage_ilu0 {
    static constexpr int kLB = 256;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_stage_ilu0_d<TJ, T, TD>(wg, a...);
    }
};

// The factors in one pass over the cells in natural order (every load of J
// coalesced): red cells store D_r^{-1}; black cells store
// (D_b - sum_r J_br D_r^{-1} J_rb)^{-1} over their red neighbours r, each
// D_r^{-1} recomputed from r's diagonal block (the same inv3 as r's own
// thread) rather than read back, so no second pass has to wait for the red
// one.  Every cell copies its off-diagonal blocks into colour-split storage,
// FP64 (Lc, with the diagonal block in Jdc) or BF16 (L16); the zero plane
// (oil, C) is left unwritten, since no kernel reads it.
__device__ __forceinline__ void k_ilu_setup_d(const Blk& wg, DevModel m, const double* __restrict__ J,
                                              double* __restrict__ Dc, double* __restrict__ Lc,
                                              double* __restrict__ Jdc, uint16_t* __restrict__ L16) {
    const int64_t v = xcd_block(wg) * blockDim.x + threadIdx.x;
    const int64_t n = m.n;
    if (v >= n) return;
    const int64_t i = strip_cell(m, v);     // a black cell re-reads its red neighbours' blocks
    const int64_t ns = ilu_slots(m), nxh = ilu_nxh(m);
    const int64_t iz = i / m.nxy;
    const int64_t rem = i - iz * m.nxy;
    const int64_t iy = rem / m.nx;
    const int64_t ix = rem - iy * m.nx;
    const int colour = (int)((ix + iy + iz) & 1);
    const int64_t s = (iy + m.ny * iz) * nxh + (ix >> 1);
    // entry 5, (oil, C), of every block is zero: neither read nor copied
    double a[9];
    for (int e = 0; e < 9; ++e) a[e] = e == 5 ? 0.0 : J[e * n + i];
    if (Jdc)
        for (int e = 0; e < 9; ++e)
            if (e != 5) __builtin_nontemporal_store(a[e], &Jdc[((int64_t)colour * 9 + e) * ns + s]);
    const bool ex[6] = {ix > 0, ix + 1 < m.nx, iy > 0, iy + 1 < m.ny, iz > 0, iz + 1 < m.nz};
    const int64_t off[6] = {-1, 1, -(int64_t)m.nx, (int64_t)m.nx, -m.nxy, m.nxy};
    for (int f = 0; f < 6; ++f) {
        double Jbr[9];
        for (int e = 0; e < 9; ++e) Jbr[e] = e == 5 ? 0.0 : J[((int64_t)(f + 1) * 9 + e) * n + i];
        if (Lc)
            for (int e = 0; e < 9; ++e) {
                if (e != 5) __builtin_nontemporal_store(Jbr[e], &Lc[((int64_t)colour * 54 + f * 9 + e) * ns + s]);
            }
        else
            for (int e = 0; e < 9; ++e) {
                if (e != 5)
                    __builtin_nontemporal_store(f32_to_bf16((float)Jbr[e]),
                                                &L16[((int64_t)colour * 54 + f * 9 + e) * ns + s]);
            }
        if (colour == 0 || !ex[f]) continue;
        const int64_t r = i + off[f];
        const int fr = f ^ 1;       // direction from r back to i
        double Drr[9], Jrb[9], Dr[9], T[9];
        for (int e = 0; e < 9; ++e) {
            Drr[e] = e == 5 ? 0.0 : J[e * n + r];
            Jrb[e] = e == 5 ? 0.0 : J[((int64_t)(fr + 1) * 9 + e) * n + r];
        }
        inv3(Drr, Dr);
        // T = Dr * Jrb;  a -= Jbr * T
        for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q)
                T[3 * p + q] = Dr[3 * p] * Jrb[q] + Dr[3 * p + 1] * Jrb[3 + q] + Dr[3 * p + 2] * Jrb[6 + q];
        for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q)
                a[3 * p + q] -= Jbr[3 * p] * T[q] + Jbr[3 * p + 1] * T[3 + q] + Jbr[3 * p + 2] * T[6 + q];
    }
    double r[9];
    inv3(a, r);
    for (int e = 0; e < 9; ++e) Dc[((int64_t)colour * 9 + e) * ns + s] = r[e];
}
__global__ __launch_bounds__(256) void k_ilu_setup(DevModel m, const double* __restrict__ J, double* __restrict__ Dc,
                                                   double* __restrict__ Lc, double* __restrict__ Jdc,
                                                   uint16_t* __restrict__ L16) {
    k_ilu_setup_d(PF_BLK, m, J, Dc, Lc, Jdc, L16);
}
struct F_k_ilu_setup {
    static constexpr int kLB = 256;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_ilu_setup_d(wg, a...);
    }
};

// The inverse diagonal blocks of red-black ILU(0) from J in the colour-split
// storage (FP64): a cell reads its diagonal block from Jdc, a black cell its
// face blocks and its red neighbours' diagonal and back-pointing blocks from
// Jdc and Lc.  The arithmetic is k_ilu_setup's, in the same order.  Threads
// are colour-major: wavefront w takes 64 consecutive slots (in the order of
// the one-colour kernels) of colour w & 1, the next wavefront the same slots
// of the other colour, so the black cells' updates fill whole wavefronts
// instead of every other lane.  Grid: 2 ilu_slots threads, rounded up to
// whole blocks (a multiple of 128).
__device__ __forceinline__ void k_ilu_diag_d(const Blk& wg, DevModel m, const double* __restrict__ Lc,
                                             const double* __restrict__ Jdc, double* __restrict__ Dc) {
    const int64_t v = xcd_block(wg) * blockDim.x + threadIdx.x;
    const int64_t w = v >> 6;
    const int colour = (int)(w & 1);
    const int64_t u = (w >> 1) * 64 + (v & 63);
    const int64_t ns = ilu_slots(m), nxh = ilu_nxh(m);
    if (u >= ns) return;
    const int64_t s = strip_slot(m, u);     // a black cell re-reads its red neighbours' blocks
    int64_t ix, iy, iz;
    if (!ilu_slot_cell(m, colour, s, ix, iy, iz)) return;
    double a[9];
    for (int e = 0; e < 9; ++e) a[e] = e == 5 ? 0.0 : Jdc[((int64_t)colour * 9 + e) * ns + s];
    if (colour == 1) {
        const bool ex[6] = {ix > 0, ix + 1 < m.nx, iy > 0, iy + 1 < m.ny, iz > 0, iz + 1 < m.nz};
        for (int f = 0; f < 6; ++f) {
            if (!ex[f]) continue;
            // the red neighbour across face f, and its slot
            const int64_t rx = ix + (f == 0 ? -1 : f == 1 ? 1 : 0);
            const int64_t ry = iy + (f == 2 ? -1 : f == 3 ? 1 : 0);
            const int64_t rz = iz + (f == 4 ? -1 : f == 5 ? 1 : 0);
            const int64_t sr = (ry + m.ny * rz) * nxh + (rx >> 1);
            const int fr = f ^ 1;       // direction from r back to i
            double Jbr[9], Drr[9], Jrb[9], Dr[9], T[9];
            for (int e = 0; e < 9; ++e) {
                Jbr[e] = e == 5 ? 0.0 : Lc[((int64_t)54 + f * 9 + e) * ns + s];
                Drr[e] = e == 5 ? 0.0 : Jdc[(int64_t)e * ns + sr];
                Jrb[e] = e == 5 ? 0.0 : Lc[((int64_t)fr * 9 + e) * ns + sr];
            }
            inv3(Drr, Dr);
            // T = Dr * Jrb;  a -= Jbr * T
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q)
                    T[3 * p + q] = Dr[3 * p] * Jrb[q] + Dr[3 * p + 1] * Jrb[3 + q] + Dr[3 * p + 2] * Jrb[6 + q];
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q)
                    a[3 * p + q] -= Jbr[3 * p] * T[q] + Jbr[3 * p + 1] * T[3 + q] + Jbr[3 * p + 2] * T[6 + q];
        }
    }
    double r[9];
    inv3(a, r);
    for (int e = 0; e < 9; ++e) Dc[((int64_t)colour * 9 + e) * ns + s] = r[e];
}
__global__ __launch_bounds__(256) void k_ilu_diag(DevModel m, const double* __restrict__ Lc,
                                                  const double* __restrict__ Jdc, double* __restrict__ Dc) {
    k_ilu_diag_d(PF_BLK, m, Lc, Jdc, Dc);
}
struct F_k_ilu_diag {
    static constexpr int kLB = 256;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_ilu_diag_d(wg, a...);
    }
};

// Natural-order J from its colour-split storage (every entry but the zero
// (oil, C) one, whose planes stay cleared).
__device__ __forceinline__ void k_j_natural_d(const Blk& wg, DevModel m, const double* __restrict__ Lc,
                                              const double* __restrict__ Jdc, double* __restrict__ J) {
    const int64_t i = (int64_t)wg.x * blockDim.x + threadIdx.x;
    const int64_t n = m.n;
    if (i >= n) return;
    const int64_t ns = ilu_slots(m), nxh = ilu_nxh(m);
    const int64_t iz = i / m.nxy;
    const int64_t rem = i - iz * m.nxy;
    const int64_t iy = rem / m.nx;
    const int64_t ix = rem - iy * m.nx;
    const int64_t cl = (ix + iy + iz) & 1;
    const int64_t s = (iy + m.ny * iz) * nxh + (ix >> 1);
    for (int d = 0; d < 7; ++d) {
        const double* src = d == 0 ? Jdc + cl * 9 * ns + s : Lc + (cl * 54 + (d - 1) * 9) * ns + s;
        for (int e = 0; e < 9; ++e)
            if (e != 5) J[((int64_t)d * 9 + e) * n + i] = src[(int64_t)e * ns];
    }
}
__global__ __launch_bounds__(256) void k_j_natural(DevModel m, const double* __restrict__ Lc,
                                                   const double* __restrict__ Jdc, double* __restrict__ J) {
    k_j_natural_d(PF_BLK, m, Lc, Jdc, J);
}
struct F_k_j_natural {
    static constexpr int kLB = 256;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_j_natural_d(wg, a...);
    }
};

// Factor loads are streamed (each off-diagonal block is read once per
// application): non-temporal, so they do not evict the vectors and the
// P-columns of J that the stage residual has just brought into the caches.
__device__ __forceinline__ double ilu_ld(const double* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float ilu_ld(const float* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float ilu_ld(const uint16_t* p) { return bf16_to_f32(__builtin_nontemporal_load(p)); }

// Phase 0 (red, forward):   y_r = D_r^{-1} f_r
// phase 1 (black, forward): y_b = D~_b^{-1} (f_b - sum J_br y_r)
// phase 2 (red, backward):  z_r = y_r - D_r^{-1} sum J_rb z_b
// y and z share storage (natural cell order, 3 planes).  Launched over the
// slots of the phase's colour.  FP64: TL = TD = TV = double; mixed: BF16
// off-diagonals, FP32 inverse diagonals, FP32 vectors and arithmetic.
template <class TL, class TD, class TV>
__device__ __forceinline__ void k_ilu_apply_t_d(const Blk& wg, DevModel m, const TL* __restrict__ Lc,
                                                const TD* __restrict__ Dc, const TV* __restrict__ f,
                                                TV* __restrict__ z, int phase) {
    const int colour = phase == 1 ? 1 : 0;
    const int64_t s = xcd_block(wg) * blockDim.x + threadIdx.x;
    const int64_t ns = ilu_slots(m);
    if (s >= ns) return;
    int64_t ix, iy, iz;
    if (!ilu_slot_cell(m, colour, s, ix, iy, iz)) return;
    const int64_t n = m.n;
    const int64_t i = ix + m.nx * iy + m.nxy * iz;
    TV t0, t1, t2;
    if (phase == 2) { t0 = 0; t1 = 0; t2 = 0; }
    else { t0 = f[i]; t1 = f[n + i]; t2 = f[2 * n + i]; }
    if (phase >= 1) {
        const bool ex[6] = {ix > 0, ix + 1 < m.nx, iy > 0, iy + 1 < m.ny, iz > 0, iz + 1 < m.nz};
        const int64_t off[6] = {-1, 1, -(int64_t)m.nx, (int64_t)m.nx, -m.nxy, m.nxy};
        TV s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            if (!ex[q]) continue;
            const int64_t j = i + off[q];
            const TV a = z[j], b = z[n + j], c = z[2 * n + j];
            const TL* B = Lc + ((int64_t)colour * 54 + q * 9) * ns + s;
            s0 += ilu_ld(B + 0 * ns) * a + ilu_ld(B + 1 * ns) * b + ilu_ld(B + 2 * ns) * c;
            s1 += ilu_ld(B + 3 * ns) * a + ilu_ld(B + 4 * ns) * b;   // entry (oil, C) is zero
            s2 += ilu_ld(B + 6 * ns) * a + ilu_ld(B + 7 * ns) * b + ilu_ld(B + 8 * ns) * c;
        }
        t0 -= s0; t1 -= s1; t2 -= s2;
    }
    const TD* D = Dc + (int64_t)colour * 9 * ns + s;
    const TV u0 = D[0 * ns] * t0 + D[1 * ns] * t1 + D[2 * ns] * t2;
    const TV u1 = D[3 * ns] * t0 + D[4 * ns] * t1 + D[5 * ns] * t2;
    const TV u2 = D[6 * ns] * t0 + D[7 * ns] * t1 + D[8 * ns] * t2;
    if (phase == 2) {
        z[i] += u0; z[n + i] += u1; z[2 * n + i] += u2;
    } else {
        z[i] = u0; z[n + i] = u1; z[2 * n + i] = u2;
    }
}
template <class TL, class TD, class TV>
__global__ __launch_bounds__(256) void k_ilu_apply_t(DevModel m, const TL* __restrict__ Lc, const TD* __restrict__ Dc,
                                                     const TV* __restrict__ f, TV* __restrict__ z, int phase) {
    k_ilu_apply_t_d<TL, TD, TV>(PF_BLK, m, Lc, Dc, f, z, phase);
}
template <class TL, class TD, class TV>
struct F_k_ilu_apply_t {
    static constexpr int kLB = 256;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_ilu_apply_t_d<TL, TD, TV>(wg, a...);
    }
};

// FP64 stage residual and forward ILU phases from the colour-split copies of
// J.  The stage residual t = v - J (p, 0, 0) - B pb needs only the P-columns
// of a row's blocks, and the black rows' off-diagonal blocks are read by the
// forward black phase anyway: that phase forms its own rows' t from them, so
// no t is stored and the P-columns of black rows are read once.  Subtraction
// order as in stage_resid_cell and k_ilu_apply_t (all P-column terms in face
// order, then the border, then the ILU sum).
__device__ __forceinline__ void stage_border(const int32_t* __restrict__ pc_map, const int32_t* __restrict__ pc_first,
                                             const int32_t* __restrict__ perf_well, const double* __restrict__ B,
                                             const double* __restrict__ pb, int64_t i, double& t0, double& t1,
                                             double& t2) {
    const int32_t k = pc_map[i];
    if (k < 0) return;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int64_t q = pc_first[k]; q < pc_first[k + 1]; ++q) {
        const double w = pb[perf_well[q]];
        a0 += B[3 * q] * w;
        a1 += B[3 * q + 1] * w;
        a2 += B[3 * q + 2] * w;
    }
    t0 = t0 - a0;
    t1 = t1 - a1;
    t2 = t2 - a2;
}

// The kernels below work on v, z and w in the colour-split layout (the
// FP64 path in PF order; pf_internal.h): a cell of slot s and colour c has
// its entries at e*lp + c*ns + s, and its neighbours, all of the other
// colour, at the slots cs_nbr gives; p (the pressure-stage correction) stays
// in natural cell order.  Pad slots (odd nx) are written zero.
//
// Slot of the neighbour across face q (-x, +x, -y, +y, -z, +z) in the other
// colour's half: along x the neighbour shares the slot or the next/previous
// one, along y it is one line (nxh slots) away, along z one layer.
__device__ __forceinline__ int64_t cs_nbr(const DevModel& m, int64_t s, int64_t ix, int q) {
    const int64_t hx = ilu_nxh(m);
    switch (q) {
        case 0: return s - ((ix & 1) ? 0 : 1);
        case 1: return s + ((ix & 1) ? 1 : 0);
        case 2: return s - hx;
        case 3: return s + hx;
        case 4: return s - hx * m.ny;
        default: return s + hx * m.ny;
    }
}

// Red slots: t_r, then the first phase z_r = D_r^{-1} t_r.
__device__ __forceinline__ void k_stage_red_d(const Blk& wg, DevModel m, const double* __restrict__ Lc,
                                              const double* __restrict__ Jdc, const double* __restrict__ Dc,
                                              const double* __restrict__ v, const double* __restrict__ p,
                                              const double* __restrict__ pb, const double* __restrict__ B,
                                              const int32_t* __restrict__ pc_map,
                                              const int32_t* __restrict__ pc_first,
                                              const int32_t* __restrict__ perf_well, double* __restrict__ z) {
    const int64_t v0 = xcd_block(wg) * blockDim.x + threadIdx.x;
    const int64_t ns = ilu_slots(m);
    if (v0 >= ns) return;
    const int64_t s = strip_slot(m, v0);
    const int64_t lp = 2 * ns;
    int64_t ix, iy, iz;
    if (!ilu_slot_cell(m, 0, s, ix, iy, iz)) {
        z[s] = 0.0; z[lp + s] = 0.0; z[2 * lp + s] = 0.0;
        return;
    }
    const int64_t i = ix + m.nx * iy + m.nxy * iz;
    const double pi = p[i];
    const double* Jd = Jdc + s;
    double t0 = v[s] - ilu_ld(Jd + 0 * ns) * pi;
    double t1 = v[lp + s] - ilu_ld(Jd + 3 * ns) * pi;
    double t2 = v[2 * lp + s] - ilu_ld(Jd + 6 * ns) * pi;
    const bool ex[6] = {ix > 0, ix + 1 < m.nx, iy > 0, iy + 1 < m.ny, iz > 0, iz + 1 < m.nz};
    const int64_t off[6] = {-1, 1, -(int64_t)m.nx, (int64_t)m.nx, -m.nxy, m.nxy};
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        if (!ex[q]) continue;
        const double pj = p[i + off[q]];
        const double* Bq = Lc + (int64_t)(q * 9) * ns + s;
        t0 -= ilu_ld(Bq + 0 * ns) * pj;
        t1 -= ilu_ld(Bq + 3 * ns) * pj;
        t2 -= ilu_ld(Bq + 6 * ns) * pj;
    }
    stage_border(pc_map, pc_first, perf_well, B, pb, i, t0, t1, t2);
    const double* D = Dc + s;
    z[s] = D[0 * ns] * t0 + D[1 * ns] * t1 + D[2 * ns] * t2;
    z[lp + s] = D[3 * ns] * t0 + D[4 * ns] * t1 + D[5 * ns] * t2;
    z[2 * lp + s] = D[6 * ns] * t0 + D[7 * ns] * t1 + D[8 * ns] * t2;
}
__global__ __launch_bounds__(256) void k_stage_red(DevModel m, const double* __restrict__ Lc,
                                                   const double* __restrict__ Jdc, const double* __restrict__ Dc,
                                                   const double* __restrict__ v, const double* __restrict__ p,
                                                   const double* __restrict__ pb, const double* __restrict__ B,
                                                   const int32_t* __restrict__ pc_map,
                                                   const int32_t* __restrict__ pc_first,
                                                   const int32_t* __restrict__ perf_well, double* __restrict__ z) {
    k_stage_red_d(PF_BLK, m, Lc, Jdc, Dc, v, p, pb, B, pc_map, pc_first, perf_well, z);
}
struct F_k_stage_red {
    static constexpr int kLB = 256;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_stage_red_d(wg, a...);
    }
};

// Black slots: t_b from its blocks' P-columns and the border, then the
// forward black phase y_b = D~_b^{-1} (t_b - sum J_br y_r), z_b = y_b.
__device__ __forceinline__ void k_ilu_black_stage_d(const Blk& wg, DevModel m, const double* __restrict__ Lc,
                                                    const double* __restrict__ Jdc, const double* __restrict__ Dc,
                                                    const double* __restrict__ v, const double* __restrict__ p,
                                                    const double* __restrict__ pb, const double* __restrict__ B,
                                                    const int32_t* __restrict__ pc_map,
                                                    const int32_t* __restrict__ pc_first,
                                                    const int32_t* __restrict__ perf_well, double* __restrict__ z) {
    const int64_t v0 = xcd_block(wg) * blockDim.x + threadIdx.x;
    const int64_t ns = ilu_slots(m);
    if (v0 >= ns) return;
    const int64_t s = strip_slot(m, v0);
    const int64_t lp = 2 * ns, o = ns + s;     // this cell's entries
    int64_t ix, iy, iz;
    if (!ilu_slot_cell(m, 1, s, ix, iy, iz)) {
        z[o] = 0.0; z[lp + o] = 0.0; z[2 * lp + o] = 0.0;
        return;
    }
    const int64_t i = ix + m.nx * iy + m.nxy * iz;
    const double pi = p[i];
    const double* Jd = Jdc + 9 * ns + s;
    double t0 = v[o] - ilu_ld(Jd + 0 * ns) * pi;
    double t1 = v[lp + o] - ilu_ld(Jd + 3 * ns) * pi;
    double t2 = v[2 * lp + o] - ilu_ld(Jd + 6 * ns) * pi;
    const bool ex[6] = {ix > 0, ix + 1 < m.nx, iy > 0, iy + 1 < m.ny, iz > 0, iz + 1 < m.nz};
    const int64_t off[6] = {-1, 1, -(int64_t)m.nx, (int64_t)m.nx, -m.nxy, m.nxy};
    double s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        if (!ex[q]) continue;
        const double pj = p[i + off[q]];
        const int64_t r = cs_nbr(m, s, ix, q);          // red neighbour
        const double a = z[r], b = z[lp + r], c = z[2 * lp + r];
        const double* Bq = Lc + (int64_t)(54 + q * 9) * ns + s;
        const double e0 = ilu_ld(Bq + 0 * ns), e1 = ilu_ld(Bq + 1 * ns), e2 = ilu_ld(Bq + 2 * ns);
        const double e3 = ilu_ld(Bq + 3 * ns), e4 = ilu_ld(Bq + 4 * ns);   // entry (oil, C) is zero
        const double e6 = ilu_ld(Bq + 6 * ns), e7 = ilu_ld(Bq + 7 * ns), e8 = ilu_ld(Bq + 8 * ns);
        t0 -= e0 * pj;
        t1 -= e3 * pj;
        t2 -= e6 * pj;
        s0 += e0 * a + e1 * b + e2 * c;
        s1 += e3 * a + e4 * b;
        s2 += e6 * a + e7 * b + e8 * c;
    }
    stage_border(pc_map, pc_first, perf_well, B, pb, i, t0, t1, t2);
    t0 -= s0;
    t1 -= s1;
    t2 -= s2;
    const double* D = Dc + 9 * ns + s;
    z[o] = D[0 * ns] * t0 + D[1 * ns] * t1 + D[2 * ns] * t2;
    z[lp + o] = D[3 * ns] * t0 + D[4 * ns] * t1 + D[5 * ns] * t2;
    z[2 * lp + o] = D[6 * ns] * t0 + D[7 * ns] * t1 + D[8 * ns] * t2;
}
__global__ __launch_bounds__(256) void k_ilu_black_stage(DevModel m, const double* __restrict__ Lc,
                                                         const double* __restrict__ Jdc,
                                                         const double* __restrict__ Dc, const double* __restrict__ v,
                                                         const double* __restrict__ p, const double* __restrict__ pb,
                                                         const double* __restrict__ B,
                                                         const int32_t* __restrict__ pc_map,
                                                         const int32_t* __restrict__ pc_first,
                                                         const int32_t* __restrict__ perf_well,
                                                         double* __restrict__ z) {
    k_ilu_black_stage_d(PF_BLK, m, Lc, Jdc, Dc, v, p, pb, B, pc_map, pc_first, perf_well, z);
}
struct F_k_ilu_black_stage {
    static constexpr int kLB = 256;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_ilu_black_stage_d(wg, a...);
    }
};

// Flexible GMRES multiplies every preconditioned vector by J at once, so
// with red-black ILU(0) the last two steps of the preconditioner carry the
// product along.  Both kernels read only colour-split storage (Lc and Jdc
// hold J itself): the red rows of the product need no blocks of J at all
// (below), and the black rows read theirs once for the product.
//
// Red slots, after phase 1: z holds y_r on red and the smoother's z_b on
// black cells.  The backward phase z_r = y_r - D_r^{-1} sum J_rb z_b, then
// the pressure correction z_r += (p_r, 0, 0) (stored).  The red rows of the
// product need no arithmetic: red-black ILU(0) leaves the red diagonal
// blocks as they are (D_r = J_rr), so the factorisation M differs from J in
// black rows only, and with z = p + M^{-1} (v - J p) (the well entries of z
// being the pressure stage's pb) the red rows of J z are (J p)_r + (M z -
// M p)_r = v_r.  w_r = v_r is stored; the well border is then added to the
// black rows only.
__device__ __forceinline__ void k_ilu_red_spmv_d(const Blk& wg, DevModel m, const double* __restrict__ Lc,
                                                 const double* __restrict__ Dc, const double* __restrict__ v,
                                                 const double* __restrict__ p, double* __restrict__ z,
                                                 double* __restrict__ w) {
    const int64_t v0 = xcd_block(wg) * blockDim.x + threadIdx.x;
    const int64_t ns = ilu_slots(m);
    if (v0 >= ns) return;
    const int64_t s = strip_slot(m, v0);
    const int64_t lp = 2 * ns;
    int64_t ix, iy, iz;
    if (!ilu_slot_cell(m, 0, s, ix, iy, iz)) {
        w[s] = 0.0; w[lp + s] = 0.0; w[2 * lp + s] = 0.0;
        return;
    }
    const int64_t i = ix + m.nx * iy + m.nxy * iz;
    const bool ex[6] = {ix > 0, ix + 1 < m.nx, iy > 0, iy + 1 < m.ny, iz > 0, iz + 1 < m.nz};
    double s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        if (!ex[q]) continue;
        const int64_t r = ns + cs_nbr(m, s, ix, q);     // black neighbour
        const double a = z[r], b = z[lp + r], c = z[2 * lp + r];
        const double* B = Lc + (int64_t)(q * 9) * ns + s;
        const double e0 = ilu_ld(B + 0 * ns), e1 = ilu_ld(B + 1 * ns), e2 = ilu_ld(B + 2 * ns);
        const double e3 = ilu_ld(B + 3 * ns), e4 = ilu_ld(B + 4 * ns);   // entry (oil, C) is zero
        const double e6 = ilu_ld(B + 6 * ns), e7 = ilu_ld(B + 7 * ns), e8 = ilu_ld(B + 8 * ns);
        s0 += e0 * a + e1 * b + e2 * c;
        s1 += e3 * a + e4 * b;
        s2 += e6 * a + e7 * b + e8 * c;
    }
    const double t0 = -s0, t1 = -s1, t2 = -s2;
    const double* D = Dc + s;
    const double z0 = z[s] + (D[0 * ns] * t0 + D[1 * ns] * t1 + D[2 * ns] * t2) + p[i];
    const double z1 = z[lp + s] + (D[3 * ns] * t0 + D[4 * ns] * t1 + D[5 * ns] * t2);
    const double z2 = z[2 * lp + s] + (D[6 * ns] * t0 + D[7 * ns] * t1 + D[8 * ns] * t2);
    z[s] = z0;
    z[lp + s] = z1;
    z[2 * lp + s] = z2;
    w[s] = v[s];
    w[lp + s] = v[lp + s];
    w[2 * lp + s] = v[2 * lp + s];
}
__global__ __launch_bounds__(256) void k_ilu_red_spmv(DevModel m, const double* __restrict__ Lc,
                                                      const double* __restrict__ Dc, const double* __restrict__ v,
                                                      const double* __restrict__ p, double* __restrict__ z,
                                                      double* __restrict__ w) {
    k_ilu_red_spmv_d(PF_BLK, m, Lc, Dc, v, p, z, w);
}
struct F_k_ilu_red_spmv {
    static constexpr int kLB = 256;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_ilu_red_spmv_d(wg, a...);
    }
};

// Black slots, after k_ilu_red_spmv: the pressure correction z_b += (p_b,
// 0, 0) (stored) and w_b = J_bb z_b + sum J_br z_r over the final red
// values.  The nw threads past the black slots set the well entries z_w =
// pb (in PF order the smoother's well rows are zero).  The well border of
// w follows in k_spmv_border.
__device__ __forceinline__ void k_black_spmv_d(const Blk& wg, DevModel m, const double* __restrict__ Lc,
                                               const double* __restrict__ Jdc, const double* __restrict__ p,
                                               const double* __restrict__ pb, double* __restrict__ z,
                                               double* __restrict__ w) {
    const int64_t v0 = xcd_block(wg) * blockDim.x + threadIdx.x;
    const int64_t ns = ilu_slots(m);
    if (v0 >= ns) {
        if (v0 < ns + m.nw) z[3 * 2 * ns + (v0 - ns)] = pb[v0 - ns];
        return;
    }
    const int64_t s = strip_slot(m, v0);
    const int64_t lp = 2 * ns, o = ns + s;
    int64_t ix, iy, iz;
    if (!ilu_slot_cell(m, 1, s, ix, iy, iz)) {
        w[o] = 0.0; w[lp + o] = 0.0; w[2 * lp + o] = 0.0;
        return;
    }
    const int64_t i = ix + m.nx * iy + m.nxy * iz;
    const double z0 = z[o] + p[i], z1 = z[lp + o], z2 = z[2 * lp + o];
    z[o] = z0;
    const double* Jd = Jdc + 9 * ns + s;
    double y0 = ilu_ld(Jd + 0 * ns) * z0 + ilu_ld(Jd + 1 * ns) * z1 + ilu_ld(Jd + 2 * ns) * z2;
    double y1 = ilu_ld(Jd + 3 * ns) * z0 + ilu_ld(Jd + 4 * ns) * z1;   // entry (oil, C) is zero
    double y2 = ilu_ld(Jd + 6 * ns) * z0 + ilu_ld(Jd + 7 * ns) * z1 + ilu_ld(Jd + 8 * ns) * z2;
    const bool ex[6] = {ix > 0, ix + 1 < m.nx, iy > 0, iy + 1 < m.ny, iz > 0, iz + 1 < m.nz};
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        if (!ex[q]) continue;
        const int64_t r = cs_nbr(m, s, ix, q);          // red neighbour
        const double a = z[r], b = z[lp + r], c = z[2 * lp + r];
        const double* B = Lc + (int64_t)(54 + q * 9) * ns + s;
        y0 += ilu_ld(B + 0 * ns) * a + ilu_ld(B + 1 * ns) * b + ilu_ld(B + 2 * ns) * c;
        y1 += ilu_ld(B + 3 * ns) * a + ilu_ld(B + 4 * ns) * b;   // entry (oil, C) is zero
        y2 += ilu_ld(B + 6 * ns) * a + ilu_ld(B + 7 * ns) * b + ilu_ld(B + 8 * ns) * c;
    }
    w[o] = y0;
    w[lp + o] = y1;
    w[2 * lp + o] = y2;
}
__global__ __launch_bounds__(256) void k_black_spmv(DevModel m, const double* __restrict__ Lc,
                                                    const double* __restrict__ Jdc, const double* __restrict__ p,
                                                    const double* __restrict__ pb, double* __restrict__ z,
                                                    double* __restrict__ w) {
    k_black_spmv_d(PF_BLK, m, Lc, Jdc, p, pb, z, w);
}
struct F_k_black_spmv {
    static constexpr int kLB = 256;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_black_spmv_d(wg, a...);
    }
};


// FP32 block Jacobi: z = Dinv t (cells), t / D (wells)
__device__ __forceinline__ void k_bjac_apply_m_d(const Blk& wg, int64_t n, int nw, const float* __restrict__ Dinv,
                                                 const double* __restrict__ Dw, const float* __restrict__ t,
                                                 float* __restrict__ z) {
    const int64_t i = (int64_t)wg.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const float a = t[i], b = t[n + i], c = t[2 * n + i];
        z[i] = Dinv[0 * n + i] * a + Dinv[1 * n + i] * b + Dinv[2 * n + i] * c;
        z[n + i] = Dinv[3 * n + i] * a + Dinv[4 * n + i] * b + Dinv[5 * n + i] * c;
        z[2 * n + i] = Dinv[6 * n + i] * a + Dinv[7 * n + i] * b + Dinv[8 * n + i] * c;
    } else if (i < n + nw) {
        const int w = (int)(i - n);
        z[3 * n + w] = (float)((double)t[3 * n + w] / Dw[w]);
    }
}
__global__ void k_bjac_apply_m(int64_t n, int nw, const float* __restrict__ Dinv, const double* __restrict__ Dw,
                               const float* __restrict__ t, float* __restrict__ z) {
    k_bjac_apply_m_d(PF_BLK, n, nw, Dinv, Dw, t, z);
}
struct F_k_bjac_apply_m {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_bjac_apply_m_d(wg, a...);
    }
};


// Level arrays in the precision of the apply.
template <class T> struct Lv;
template <> struct Lv<double> {
    static const double* A(const MGLevel& L) { return L.A; }
    static const double* aux(const MGLevel& L) { return L.aux; }
    static double* x(const MGLevel& L) { return L.x; }
    static double* b(const MGLevel& L) { return L.b; }
    static const double* inv(const Sim& s) { return s.coarse_inv; }
    static double* pnat(const Sim& s) { return s.pnat; }
};
template <> struct Lv<float> {
    static const float* A(const MGLevel& L) { return L.A32; }
    static const float* aux(const MGLevel& L) { return L.aux32; }
    static float* x(const MGLevel& L) { return L.x32; }
    static float* b(const MGLevel& L) { return L.b32; }
    static const float* inv(const Sim& s) { return s.coarse_inv32; }
    static float* pnat(const Sim& s) { return s.pnat32; }
};

// Launch shape of a z-line half-sweep of level L.  Segment length: 4
// layers (8 above 256 layers, longer only where a column would need more
// than 64 segments: register kernel up to 8 layers, memory-staged beyond);
// on levels too small to fill the GPU with 8-layer segments (fewer than
// kZlineSmallThreads threads) 2 layers where that stays within the count, so
// that a latency-bound sweep is spread over more threads.  zline_len
// overrides; never more than 64 segments.  Block shape: 32 (else 16, else 8)
// columns per block where that still gives >= 128 blocks, so a wavefront
// reads runs of that many consecutive slots of each layer; otherwise the
// largest block of 256, 128 or 64 threads that gives >= 512 blocks.
struct ZlShape {
    int len, nseg, cpb;
    unsigned blocks, threads;
    int lmax;                        // register bound of the kernel (>= len)
};

ZlShape zline_shape(const Sim& s, const MGLevel& L) {
    const int64_t cols = (int64_t)((L.nx + 1) / 2) * L.ny;
    int len = L.nz <= 256 ? 4 : std::max(8, (L.nz + 63) / 64);
    if (s.opts.zline_len > 0) {
        len = s.opts.zline_len;
    } else if (cols * ((L.nz + 7) / 8) < kZlineSmallThreads && (L.nz + 1) / 2 <= 64 &&
               cols * ((L.nz + 1) / 2) <= kZlineSmallThreads) {
        len = 2;
    }
    int nseg = (L.nz + len - 1) / len;
    if (nseg > 64) nseg = 64;
    len = (L.nz + nseg - 1) / nseg;
    int cpb = 0;
    if (len <= 8)
        for (int cand : {32, 16, 8})
            if (cand * nseg <= 1024 && (cols + cand - 1) / cand >= 128) {
                cpb = cand;
                break;
            }
    if (cpb == 0) {
        int bs = 64;
        for (int cand : {256, 128}) {
            const int c = cand / nseg;
            if (c >= 1 && (cols + c - 1) / c >= 512) {
                bs = cand;
                break;
            }
        }
        cpb = std::max(1, bs / nseg);
    }
    int lmax = len <= 2 ? 2 : len <= 4 ? 4 : 8;
    unsigned threads = (unsigned)(cpb * nseg);
    if (s.fu && len <= 8) {
        // in a fusion group one block size for every level and member, so
        // that sweeps with the same segment bound share launches (the
        // columns a block holds do not change a column's arithmetic)
        cpb = std::max(1, 256 / nseg);
        threads = 256;
    }
    return ZlShape{len, nseg, cpb, (unsigned)((cols + cpb - 1) / cpb), threads, lmax};
}

// One z-line half-sweep of level L: segments in registers up to 8 layers,
// memory-staged beyond.
template <class T>
void zline_sweep(Sim& s, const MGLevel& L, int colour, int zero_init) {
    const Dims g = dims_of(L);
    const T* A = Lv<T>::A(L);
    const T* aux = Lv<T>::aux(L);
    T* x = Lv<T>::x(L);
    const T* b = Lv<T>::b(L);
    const ZlShape z = zline_shape(s, L);
    const int len = z.len, nseg = z.nseg, cpb = z.cpb;
    const dim3 blocks(z.blocks), threads(z.threads);
    if (len <= 8 && z.lmax == 2 && zero_init)
        launch<F_k_zline_seg<2, T, true>>(s, s.stream, (k_zline_seg<2, T, true>), blocks, threads, 0, g, A, aux, b, x,
                                          colour, len, nseg, cpb);
    else if (len <= 8 && z.lmax == 2)
        launch<F_k_zline_seg<2, T, false>>(s, s.stream, (k_zline_seg<2, T, false>), blocks, threads, 0, g, A, aux, b,
                                           x, colour, len, nseg, cpb);
    else if (len <= 8 && z.lmax == 4 && zero_init)
        launch<F_k_zline_seg<4, T, true>>(s, s.stream, (k_zline_seg<4, T, true>), blocks, threads, 0, g, A, aux, b, x,
                                          colour, len, nseg, cpb);
    else if (len <= 8 && z.lmax == 4)
        launch<F_k_zline_seg<4, T, false>>(s, s.stream, (k_zline_seg<4, T, false>), blocks, threads, 0, g, A, aux, b,
                                           x, colour, len, nseg, cpb);
    else if (len <= 8 && zero_init)
        launch<F_k_zline_seg<8, T, true>>(s, s.stream, (k_zline_seg<8, T, true>), blocks, threads, 0, g, A, aux, b, x,
                                          colour, len, nseg, cpb);
    else if (len <= 8)
        launch<F_k_zline_seg<8, T, false>>(s, s.stream, (k_zline_seg<8, T, false>), blocks, threads, 0, g, A, aux, b,
                                           x, colour, len, nseg, cpb);
    else
        launch<F_k_zline_seg_mem<T>>(s, s.stream, (k_zline_seg_mem<T>), blocks, threads, 0, g, A, aux, b, x, colour,
                                     zero_init, len, nseg, cpb);
    PF_LAUNCH_CHECK();
}

// sweeps full z-line sweeps (both colours) in one workgroup where every
// column of a colour fits it with the level's segment length; false
// (nothing launched) otherwise.  (Longer segments to make a larger level
// fit were slower than its two launches per sweep.)
template <class T>
bool zline_full_sweeps(Sim& s, const MGLevel& L, int zero_init, int sweeps) {
    const ZlShape z = zline_shape(s, L);
    const int64_t cols = (int64_t)((L.nx + 1) / 2) * L.ny;
    if (z.len > 8 || cols * z.nseg > 1024) return false;
    const Dims g = dims_of(L);
    const T* A = Lv<T>::A(L);
    const T* aux = Lv<T>::aux(L);
    T* x = Lv<T>::x(L);
    const T* b = Lv<T>::b(L);
    const int cpb = (int)cols;
    const dim3 threads(s.fu ? 1024u : (unsigned)(cpb * z.nseg));     // one shape in a fusion group
#define PF_ZF(LM)                                                                                          \
    if (zero_init)                                                                                         \
        launch<F_k_zline_full<LM, T, true>>(s, s.stream, (k_zline_full<LM, T, true>), dim3(1), threads, 0, g, A, \
                                            aux, b, x, z.len, z.nseg, cpb, sweeps);                        \
    else                                                                                                   \
        launch<F_k_zline_full<LM, T, false>>(s, s.stream, (k_zline_full<LM, T, false>), dim3(1), threads, 0, g,  \
                                             A, aux, b, x, z.len, z.nseg, cpb, sweeps);
    if (z.lmax == 2) { PF_ZF(2) }
    else if (z.lmax == 4) { PF_ZF(4) }
    else { PF_ZF(8) }
#undef PF_ZF
    PF_LAUNCH_CHECK();
    return true;
}

// b = Pi_r v on level 0 fused with the first V-cycle's first half-sweep;
// false (nothing launched) where level 0 is the coarsest or its segments
// take the memory-staged kernel.
template <class T>
bool restrict_p_zline(Sim& s, const double* v, int cs) {
    const MGLevel& L = s.mg[0];
    if (s.mg.size() < 2 || !L.split) return false;
    const ZlShape z = zline_shape(s, L);
    if (z.len > 8) return false;
    const Dims g = dims_of(L);
    const T *A = Lv<T>::A(L), *aux = Lv<T>::aux(L);
    T *b = Lv<T>::b(L), *x = Lv<T>::x(L);
    const dim3 blocks(z.blocks), threads(z.threads);
    if (z.lmax == 2)
        launch<F_k_restrict_p_zline<2, T>>(s, s.stream, (k_restrict_p_zline<2, T>), blocks, threads, 0, g, v, A, aux,
                                           b, x, z.len, z.nseg, z.cpb, cs);
    else if (z.lmax == 4)
        launch<F_k_restrict_p_zline<4, T>>(s, s.stream, (k_restrict_p_zline<4, T>), blocks, threads, 0, g, v, A, aux,
                                           b, x, z.len, z.nseg, z.cpb, cs);
    else
        launch<F_k_restrict_p_zline<8, T>>(s, s.stream, (k_restrict_p_zline<8, T>), blocks, threads, 0, g, v, A, aux,
                                           b, x, z.len, z.nseg, z.cpb, cs);
    PF_LAUNCH_CHECK();
    return true;
}

unsigned cast_grid(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > 8192) g = 8192;
    return (unsigned)(g > 0 ? g : 1);
}

void cast(Sim& s, int64_t n, const double* src, float* dst) {
    launch<F_k_cast_f32>(s, s.stream, k_cast_f32, dim3(cast_grid(n)), dim3(kBlock), 0, n, src, dst);
    PF_LAUNCH_CHECK();
}

}  // namespace

// ---------------------------------------------------------------------------
void cpr_choose_levels(Sim& s) {
    s.mg.clear();
    MGLevel L{};
    L.nx = s.m.nx; L.ny = s.m.ny; L.nz = s.m.nz;
    L.n = s.m.n;
    const int64_t cmax = std::max(8, s.opts.mg_coarse > 0 ? s.opts.mg_coarse : 96);
    for (;;) {
        if (L.n <= cmax) { L.cx = L.cy = L.cz = 1; L.split = 0; L.ns = L.n; s.mg.push_back(L); break; }
        const int64_t cols = (int64_t)L.nx * L.ny;
        int cx = L.nx > 1 ? 2 : 1, cy = L.ny > 1 ? 2 : 1;
        int cz = (cols >= kColsForXY || L.nz == 1) ? 1 : 2;
        if (cols < kColsForXY && cx == 1 && cy == 1) cz = 2;
        if (cx == 1 && cy == 1 && cz == 1) { L.cx = L.cy = L.cz = 1; L.split = 0; L.ns = L.n; s.mg.push_back(L); break; }
        L.cx = cx; L.cy = cy; L.cz = cz;
        L.split = 1;
        L.ns = lv_slots(dims_of(L));
        s.mg.push_back(L);
        MGLevel C{};
        C.nx = (L.nx + cx - 1) / cx;
        C.ny = (L.ny + cy - 1) / cy;
        C.nz = (L.nz + cz - 1) / cz;
        C.n = (int64_t)C.nx * C.ny * C.nz;
        L = C;
    }
}

// slots per colour of the colour-split ILU storage: ceil(nx/2) per x-line
static int64_t ilu_slot_count(const DevModel& m) { return (int64_t)((m.nx + 1) / 2) * m.ny * m.nz; }

void cpr_plan(Sim& s, Bump& b) {
    const int nl = (int)s.mg.size();
    const bool mixed = s.opts.precision == PF_PREC_MIXED;
    for (int l = 0; l < nl; ++l) {
        MGLevel& L = s.mg[l];
        L.A = b.take<double>(7 * L.ns);
        L.aux = b.take<double>(3 * L.ns);
        L.x = b.take<double>(L.ns);
        L.b = b.take<double>(L.ns);
        L.r = nullptr;
        if (mixed) {
            L.A32 = b.take<float>(7 * L.ns);
            L.aux32 = b.take<float>(3 * L.ns);
            L.x32 = b.take<float>(L.ns);
            L.b32 = b.take<float>(L.ns);
        }
    }
    s.pnat = b.take<double>(s.m.n);
    s.pnat32 = mixed ? b.take<float>(s.m.n) : nullptr;
    s.Ap = s.mg[0].A;
    const int64_t nc = s.mg.back().n;
    s.coarse_aug = b.take<double>((size_t)nc * 2 * nc);
    s.coarse_inv = b.take<double>((size_t)nc * nc);
    s.pb = b.take<double>(std::max(s.m.nw, 1));
    const bool ilu = s.opts.smoother == PF_SMOOTH_RBILU0;
    const int64_t ns = ilu_slot_count(s.m);
    // block Jacobi: 9 natural planes; ILU: 2 colours x 9 planes of ns slots (>= 9N)
    s.Dinv = b.take<double>(ilu ? 18 * ns : 9 * s.m.n);
    s.Lc = (ilu && !mixed) ? b.take<double>(108 * ns) : nullptr;
    s.Jdc = (ilu && !mixed) ? b.take<double>(18 * ns) : nullptr;
    if (mixed) {
        s.coarse_inv32 = b.take<float>((size_t)nc * nc);
        s.Jp32 = b.take<float>(21 * s.m.n);
        s.Joff16 = ilu ? b.take<uint16_t>(108 * ns) : nullptr;
        s.Dinv32 = b.take<float>(ilu ? 18 * ns : 9 * s.m.n);
        s.t32 = b.take<float>(s.nv);
    }
}

void cpr_setup(Sim& s) {
    const DevModel& m = s.m;
    if (s.coarse_pending) {
        // the previous inverse is done with the coarse matrix before it is rebuilt
        PF_HIP(hipStreamWaitEvent(s.stream, s.ev_join, 0));
        s.coarse_pending = false;
    }
    const int nl = (int)s.mg.size();
    const bool mixed = s.opts.precision == PF_PREC_MIXED;
    if (s.j_cs && !s.j_nat)
        launch<F_k_extract_ap_cs>(s, s.stream, k_extract_ap_cs, dim3(grid_for(m.n)), dim3(kBlock), 0,
                                  dims_of(s.mg[0]), s.Lc, s.Jdc, s.mg[0].A);
    else
        launch<F_k_extract_ap>(s, s.stream, k_extract_ap, dim3(grid_for(m.n)), dim3(kBlock), 0, dims_of(s.mg[0]),
                               s.J, s.mg[0].A);
    PF_LAUNCH_CHECK();
    for (int l = 0; l + 1 < nl; ++l) {
        const MGLevel& F = s.mg[l];
        const MGLevel& C = s.mg[l + 1];
        launch<F_k_galerkin>(s, s.stream, k_galerkin, dim3(grid_for(C.n)), dim3(kBlock), 0, dims_of(F), dims_of(C),
                             F.cx, F.cy, F.cz, F.A, C.A);
        PF_LAUNCH_CHECK();
    }
    const MGLevel& Cn = s.mg.back();
    launch<F_k_coarse_build>(s, s.stream, k_coarse_build, dim3(grid_for(Cn.n, 64)), dim3(64), 0, dims_of(Cn), Cn.A,
                             s.coarse_aug);
    PF_LAUNCH_CHECK();
    // the coarsest inverse (one workgroup, latency-bound) runs on the side
    // stream, from as soon as the coarsest operator exists, while the z-line
    // factorisations, the smoother set-up and the first V-cycle's way down
    // fill the GPU; joined before the first coarsest solve (vcycle).  A
    // simulator without a side stream runs it in order on its own stream.
    const bool side = s.aux && !s.fu;       // a fusion group has one stream
    hipStream_t cs = side ? s.aux : s.stream;
    if (side) {
        PF_HIP(hipEventRecord(s.ev_fork, s.stream));
        PF_HIP(hipStreamWaitEvent(s.aux, s.ev_fork, 0));
    }
    const size_t lds = (size_t)(2 * Cn.n * Cn.n + Cn.n) * sizeof(double);
    if (Cn.n <= kGJLds && lds <= (size_t)s.max_lds) {
        // 256 threads (>= 2n): a workgroup of 1024 waited for a compute unit with 16 free wave slots
        // while the ILU set-up filled the GPU (300^3: 5.7 ms against 146 us)
        launch<F_k_gauss_jordan_lds>(s, cs, k_gauss_jordan_lds, dim3(1), dim3(256), lds, (int)Cn.n, s.coarse_aug);
    } else {
        launch<F_k_gauss_jordan>(s, cs, k_gauss_jordan, dim3(1), dim3(1024), 0, (int)Cn.n, s.coarse_aug);
    }
    PF_LAUNCH_CHECK();
    launch<F_k_compact_inv>(s, cs, k_compact_inv, dim3(grid_for(Cn.n * Cn.n)), dim3(kBlock), 0, (int)Cn.n,
                            s.coarse_aug, s.coarse_inv, mixed ? s.coarse_inv32 : (float*)nullptr);
    PF_LAUNCH_CHECK();
    if (side) PF_HIP(hipEventRecord(s.ev_join, s.aux));
    for (int l = 0; l + 1 < nl; ++l) {
        const MGLevel& L = s.mg[l];
        launch<F_k_zline_setup>(s, s.stream, k_zline_setup, dim3(grid_for((int64_t)L.nx * L.ny)), dim3(kBlock), 0,
                                dims_of(L), L.A, L.aux);
        PF_LAUNCH_CHECK();
    }
    if (s.opts.smoother == PF_SMOOTH_RBILU0 && s.j_cs && !mixed) {
        // J is already in the colour-split storage: only the inverse diagonal blocks
        launch<F_k_ilu_diag>(s, s.stream, k_ilu_diag, dim3(grid_for(2 * ilu_slot_count(m))), dim3(kBlock), 0, m, s.Lc,
                             s.Jdc, s.Dinv);
        PF_LAUNCH_CHECK();
    } else if (s.opts.smoother == PF_SMOOTH_RBILU0) {
        ensure_j_natural(s);
        launch<F_k_ilu_setup>(s, s.stream, k_ilu_setup, dim3(grid_for(m.n)), dim3(kBlock), 0, m, s.J, s.Dinv, s.Lc,
                              s.Jdc, mixed ? s.Joff16 : (uint16_t*)nullptr);
        PF_LAUNCH_CHECK();
    } else {
        ensure_j_natural(s);
        launch_bjac_setup(s);
    }
    if (mixed) {
        ensure_j_natural(s);
        for (int l = 0; l < nl; ++l) {
            const MGLevel& L = s.mg[l];
            cast(s, 7 * L.ns, L.A, L.A32);
            cast(s, 3 * L.ns, L.aux, L.aux32);
        }
        launch<F_k_extract_lowp>(s, s.stream, k_extract_lowp, dim3(grid_for(m.n)), dim3(kBlock), 0, m.n, s.J, s.Jp32);
        PF_LAUNCH_CHECK();
        cast(s, s.opts.smoother == PF_SMOOTH_RBILU0 ? 18 * ilu_slot_count(m) : 9 * m.n, s.Dinv, s.Dinv32);
    }
    if (side) s.coarse_pending = true;
}

namespace {

template <class T>
void launch_prolong_chain(Sim& s, const Dims& g, const ProlongChain& pc, T* x, T* pout) {
    const dim3 grid(grid_for((int64_t)g.nx * g.ny * g.nz)), block(kBlock);
    switch (pc.nl) {
#define PF_CASE(K)                                                                                        \
    case K:                                                                                               \
        launch<F_k_prolong_chain<T, K>>(s, s.stream, (k_prolong_chain<T, K>), grid, block, 0, g, pc, x, pout); \
        break;
        PF_CASE(2) PF_CASE(3) PF_CASE(4) PF_CASE(5) PF_CASE(6) PF_CASE(7) PF_CASE(8) PF_CASE(9)
        PF_CASE(10) PF_CASE(11) PF_CASE(12) PF_CASE(13) PF_CASE(14) PF_CASE(15) PF_CASE(16)
#undef PF_CASE
        default: launch<F_k_prolong_chain<T, 0>>(s, s.stream, (k_prolong_chain<T, 0>), grid, block, 0, g, pc, x, pout);
    }
    PF_LAUNCH_CHECK();
}

// Pre-smoothing sweeps of a level: mg_pre, or mg_pre_small on the levels of
// at most max(mg_small_cells, n0 / 32) cells (n0: the finest level's cells)
// when n0 is at least ten times mg_small_cells.  A sweep on such a level
// costs little more than its launch or a small share of a fine-level sweep,
// and the better coarse correction saves FGMRES iterations whose cost grows
// with the finest level; on a small grid every launch counts and the extra
// sweeps do not pay.  (Measured: levels of up to 1/32 of n0 gain, those of
// 1/16 or more cost more iterations or sweep time than they save.)
int pre_sweeps(const Sim& s, const MGLevel& L) {
    const int64_t base = s.opts.mg_small_cells > 0 ? s.opts.mg_small_cells : kPreSmallCells;
    const int64_t n0 = s.mg[0].n;
    const int64_t small = std::max(base, n0 / kPreSmallFrac);
    const bool extra = L.n <= small && n0 >= 10 * base;
    const int p = extra ? (s.opts.mg_pre_small > 0 ? s.opts.mg_pre_small : kPreSmall) : s.opts.mg_pre;
    return std::max(1, p);
}

// One V-cycle from level l.  At level 0 of the last cycle, pout receives the
// level-0 correction in natural cell order.  first_done: the first colour-0
// half-sweep of level l (from x = 0) was done with the restriction onto it.
template <class T>
void vcycle(Sim& s, int l, int zero_init0 = 1, T* pout = nullptr, bool first_done = false) {
    const int nl = (int)s.mg.size();
    MGLevel& L = s.mg[l];
    const Dims g = dims_of(L);
    if (l == nl - 1) {
        if (s.coarse_pending) {
            PF_HIP(hipStreamWaitEvent(s.stream, s.ev_join, 0));     // the inverse from the side stream
            s.coarse_pending = false;
        }
        launch<F_k_coarse_apply<T>>(s, s.stream, k_coarse_apply<T>, dim3((unsigned)((L.n + 3) / 4)), dim3(256), 0,
                                    (int)L.n, Lv<T>::inv(s), Lv<T>::b(L), Lv<T>::x(L));
        PF_LAUNCH_CHECK();
    } else {
        const int pre = pre_sweeps(s, L), post = std::max(0, s.opts.mg_post);
        MGLevel& C = s.mg[l + 1];
        // a level that fits one workgroup takes all its pre-sweeps in one launch
        const bool whole = l > 0 && !first_done && zline_full_sweeps<T>(s, L, zero_init0, pre);
        for (int it = 0; it < (whole ? 0 : pre); ++it) {
            const int zi = (it == 0 && zero_init0) ? 1 : 0;
            if (!(it == 0 && first_done)) {
                ProfScope ps(s, l == 0 ? PF_K_ZLINE : 0);
                zline_sweep<T>(s, L, 0, zi);
            }
            zline_sweep<T>(s, L, 1, 0);
        }
        // pre-smoothing ended with a colour-1 half-sweep: those rows' residuals
        // are zero; after a single sweep from x = 0 the colour-0 rows' are
        // their lateral terms alone
        const bool lat = pre == 1 && zero_init0;
#define PF_RR(RB, LAT)                                                                                        \
    launch<F_k_resid_restrict<T, RB, LAT>>(s, s.stream, (k_resid_restrict<T, RB, LAT>), dim3(grid_for(C.n)), \
                                           dim3(kBlock), 0, g, dims_of(C), L.cx, L.cy, L.cz, Lv<T>::A(L),     \
                                           Lv<T>::x(L), Lv<T>::b(L), Lv<T>::b(C), 1)
        if (L.cx == 2 && L.cy == 2) {
            if (lat) PF_RR(true, true);
            else PF_RR(true, false);
        } else {
            if (lat) PF_RR(false, true);
            else PF_RR(false, false);
        }
#undef PF_RR
        PF_LAUNCH_CHECK();
        vcycle<T>(s, l + 1);
        if (post == 0 && nl <= kMaxChain) {
            // no post-smoothing: the whole upward pass is prolongation, done once from level 0
            if (l == 0) {
                ProlongChain pc{};
                pc.nl = nl;
                for (int q = 1; q < nl; ++q) {
                    const MGLevel& F = s.mg[q - 1];
                    pc.sx[q] = pc.sx[q - 1] + (F.cx == 2);
                    pc.sy[q] = pc.sy[q - 1] + (F.cy == 2);
                    pc.sz[q] = pc.sz[q - 1] + (F.cz == 2);
                    pc.d[q] = dims_of(s.mg[q]);
                    pc.x[q] = Lv<T>::x(s.mg[q]);
                }
                launch_prolong_chain<T>(s, g, pc, Lv<T>::x(L), pout);
                PF_LAUNCH_CHECK();
            }
            return;
        }
        launch<F_k_prolong_add<T>>(s, s.stream, k_prolong_add<T>, dim3(grid_for(L.n)), dim3(kBlock), 0, g, dims_of(C),
                                   L.cx, L.cy, L.cz, Lv<T>::x(C), Lv<T>::x(L));
        PF_LAUNCH_CHECK();
        for (int it = 0; it < post; ++it) {
            zline_sweep<T>(s, L, 1, 0);
            zline_sweep<T>(s, L, 0, 0);
        }
    }
    if (pout) {
        launch<F_k_gather_p<T>>(s, s.stream, k_gather_p<T>, dim3(grid_for(L.n)), dim3(kBlock), 0, g, Lv<T>::x(L),
                                pout);
        PF_LAUNCH_CHECK();
    }
}

}  // namespace

void mg_smooth_once(Sim& s, int level, int colour, int zero_init) {
    zline_sweep<double>(s, s.mg[level], colour, zero_init);
}

namespace {

// b = Pi_r v (water + oil rows of v, in the natural or, cs, the colour-split
// layout); p = V-cycle(s) from p = 0.  Returns p in natural cell order.
template <class T>
T* pressure_cycles(Sim& s, const double* v, int cs = 0) {
    const DevModel& m = s.m;
    T* p = Lv<T>::pnat(s);
    const bool fused = restrict_p_zline<T>(s, v, cs);
    if (!fused) {
        launch<F_k_restrict_p<T>>(s, s.stream, k_restrict_p<T>, dim3(grid_for(m.n)), dim3(kBlock), 0,
                                  dims_of(s.mg[0]), v, Lv<T>::b(s.mg[0]), cs);
        PF_LAUNCH_CHECK();
    }
    const int cycles = std::max(1, s.opts.mg_cycles);
    for (int c = 0; c < cycles; ++c)
        vcycle<T>(s, 0, c == 0 ? 1 : 0, c + 1 == cycles ? p : nullptr, fused && c == 0);
    return p;
}

// Pressure stage: the V-cycles, then well pressures from the well rows.
template <class T>
const T* pressure_stage(Sim& s, const double* v, int cs = 0) {
    const DevModel& m = s.m;
    const T* p = pressure_cycles<T>(s, v, cs);
    if (m.nw > 0) {
        // the well rows of v follow its three planes
        const double* vw = v + 3 * (cs ? 2 * cs_ns(m) : m.n);
        launch<F_k_well_pb<T>>(s, s.stream, k_well_pb<T>, dim3(m.nw), dim3(64), 0, m, s.wp_first, s.wp_idx,
                               s.perf_cell, s.Cw, s.Dw, vw, p, s.pb);
        PF_LAUNCH_CHECK();
    }
    return p;
}

// first_phase 1: the red phase 0 was done by k_stage_ilu0
void smoother_apply(Sim& s, const double* f, double* z, int first_phase = 0) {
    const DevModel& m = s.m;
    if (s.opts.smoother == PF_SMOOTH_RBILU0) {
        for (int ph = first_phase; ph < 3; ++ph) {
            ProfScope ps(s, ph == 1 ? PF_K_ILU : 0);
            launch<F_k_ilu_apply_t<double, double, double>>(s, s.stream, (k_ilu_apply_t<double, double, double>),
                                                            dim3(grid_for(ilu_slot_count(m))), dim3(kBlock), 0, m,
                                                            (const double*)s.Lc, (const double*)s.Dinv, f, z, ph);
            PF_LAUNCH_CHECK();
        }
        if (m.nw > 0) {
            launch<F_k_well_diag<double>>(s, s.stream, k_well_diag<double>, dim3(grid_for(m.nw, 64)), dim3(64), 0,
                                          m.n, m.nw, s.Dw, f, z);
            PF_LAUNCH_CHECK();
        }
    } else {
        launch<F_k_bjac_apply_add>(s, s.stream, k_bjac_apply_add, dim3(grid_for(m.n + m.nw)), dim3(kBlock), 0, m.n,
                                   m.nw, s.Dinv, s.Dw, f, (const double*)nullptr, (const double*)nullptr, z);
        PF_LAUNCH_CHECK();
    }
}

void smoother_apply_m(Sim& s, const float* f, float* z, int first_phase = 0) {
    const DevModel& m = s.m;
    if (s.opts.smoother == PF_SMOOTH_RBILU0) {
        for (int ph = first_phase; ph < 3; ++ph) {
            ProfScope ps(s, ph == 1 ? PF_K_ILU : 0);
            launch<F_k_ilu_apply_t<uint16_t, float, float>>(s, s.stream, (k_ilu_apply_t<uint16_t, float, float>),
                                                            dim3(grid_for(ilu_slot_count(m))), dim3(kBlock), 0, m,
                                                            (const uint16_t*)s.Joff16, (const float*)s.Dinv32, f, z,
                                                            ph);
            PF_LAUNCH_CHECK();
        }
        if (m.nw > 0) {
            launch<F_k_well_diag<float>>(s, s.stream, k_well_diag<float>, dim3(grid_for(m.nw, 64)), dim3(64), 0, m.n,
                                         m.nw, s.Dw, f, z);
            PF_LAUNCH_CHECK();
        }
    } else {
        launch<F_k_bjac_apply_m>(s, s.stream, k_bjac_apply_m, dim3(grid_for(m.n + m.nw)), dim3(kBlock), 0, m.n, m.nw,
                                 s.Dinv32, s.Dw, f, z);
        PF_LAUNCH_CHECK();
    }
}

}  // namespace

void smoother_once(Sim& s, const double* f) {
    if (s.opts.precision == PF_PREC_MIXED) {
        cast(s, s.nv, f, s.t32);
        smoother_apply_m(s, s.t32, s.Z32);
    } else {
        smoother_apply(s, f, s.t1);
    }
}

void mg_cycles_once(Sim& s, const double* v) {
    if (s.opts.precision == PF_PREC_MIXED) pressure_cycles<float>(s, v);
    else pressure_cycles<double>(s, v);
}

void cpr_apply(Sim& s, const double* v, double* z) {
    const DevModel& m = s.m;
    ensure_j_natural(s);
    if (s.opts.cpr_order == PF_CPR_PF) {
        const double* p = pressure_stage<double>(s, v);
        if (s.opts.smoother == PF_SMOOTH_RBILU0) {
            {
                ProfScope ps(s, PF_K_STAGE_RESID);
                launch<F_k_stage_ilu0<double, double, double>>(s, s.stream, (k_stage_ilu0<double, double, double>),
                                                               dim3(grid_for(m.n + m.nw)), dim3(kBlock), 0, m, s.J, v,
                                                               p, s.pb, s.B, s.pc_map, s.pc_first, s.perf_well,
                                                               (const double*)s.Dinv, s.t2, z);
                PF_LAUNCH_CHECK();
            }
            smoother_apply(s, s.t2, z, 1);
        } else {
            {
                ProfScope ps(s, PF_K_STAGE_RESID);
                launch<F_k_stage_resid<double, double>>(s, s.stream, (k_stage_resid<double, double>),
                                                        dim3(grid_for(m.n)), dim3(kBlock), 0, m, s.J, v, p, s.t2);
                PF_LAUNCH_CHECK();
            }
            if (m.nw > 0) {
                launch<F_k_stage_resid_border<double>>(s, s.stream, k_stage_resid_border<double>,
                                                       dim3(grid_for(m.npc + m.nw, 64)), dim3(64), 0, m, s.pc_cell,
                                                       s.pc_first, s.perf_well, s.B, s.pb, s.t2);
                PF_LAUNCH_CHECK();
            }
            smoother_apply(s, s.t2, z);
        }
        launch<F_k_add_pressure<double>>(s, s.stream, k_add_pressure<double>, dim3(grid_for(m.n + m.nw)),
                                         dim3(kBlock), 0, m.n, m.nw, p, s.pb, z);
        PF_LAUNCH_CHECK();
    } else {
        // Algorithm 2: y = S(v); r = v - J y; y += Pi_p M_g^{-1} Pi_r r
        smoother_apply(s, v, z);
        launch_spmv(s, z, s.t2);
        launch_axpby(s, s.nv, 1.0, v, -1.0, s.t2);
        const double* p = pressure_stage<double>(s, s.t2);
        launch<F_k_add_pressure<double>>(s, s.stream, k_add_pressure<double>, dim3(grid_for(m.n + m.nw)),
                                         dim3(kBlock), 0, m.n, m.nw, p, s.pb, z);
        PF_LAUNCH_CHECK();
    }
}

bool cpr_colour_split(const Sim& s) {
    return s.opts.cpr_order == PF_CPR_PF && s.opts.smoother == PF_SMOOTH_RBILU0 && s.Jdc;
}

bool j_colour_split_mode(const Sim& s) {
    return cpr_colour_split(s) && s.Lc && s.opts.precision == PF_PREC_FP64;
}

void ensure_j_natural(Sim& s) {
    if (s.j_nat) return;
    launch<F_k_j_natural>(s, s.stream, k_j_natural, dim3(grid_for(s.m.n)), dim3(kBlock), 0, s.m, s.Lc, s.Jdc, s.J);
    PF_LAUNCH_CHECK();
    s.j_nat = true;
}

// z = M^{-1} v and w = J~ z (FP64).  In PF order with the red-black ILU(0)
// smoother (cpr_colour_split) v, z and w are in the colour-split layout and
// the product rides on the last ILU phase (k_ilu_red_spmv, k_black_spmv);
// otherwise, in natural order, cpr_apply and the plain product.
void cpr_apply_spmv(Sim& s, const double* v, double* z, double* w) {
    const DevModel& m = s.m;
    if (!cpr_colour_split(s)) {
        cpr_apply(s, v, z);
        launch_spmv(s, z, w);
        return;
    }
    const double* p = pressure_stage<double>(s, v, 1);
    const int64_t ns = ilu_slot_count(m);
    {
        ProfScope ps(s, PF_K_STAGE_RESID);
        launch<F_k_stage_red>(s, s.stream, k_stage_red, dim3(grid_for(ns)), dim3(kBlock), 0, m, (const double*)s.Lc,
                              (const double*)s.Jdc, (const double*)s.Dinv, v, p, s.pb, s.B, s.pc_map, s.pc_first,
                              s.perf_well, z);
        PF_LAUNCH_CHECK();
    }
    {
        ProfScope ps(s, PF_K_ILU);
        launch<F_k_ilu_black_stage>(s, s.stream, k_ilu_black_stage, dim3(grid_for(ns)), dim3(kBlock), 0, m,
                                    (const double*)s.Lc, (const double*)s.Jdc, (const double*)s.Dinv, v, p, s.pb, s.B,
                                    s.pc_map, s.pc_first, s.perf_well, z);
        PF_LAUNCH_CHECK();
    }
    {
        ProfScope ps(s, PF_K_RED_SPMV);
        launch<F_k_ilu_red_spmv>(s, s.stream, k_ilu_red_spmv, dim3(grid_for(ns)), dim3(kBlock), 0, m,
                                 (const double*)s.Lc, (const double*)s.Dinv, v, p, z, w);
        PF_LAUNCH_CHECK();
    }
    {
        ProfScope ps(s, PF_K_BLACK_SPMV);
        launch<F_k_black_spmv>(s, s.stream, k_black_spmv, dim3(grid_for(ns + m.nw)), dim3(kBlock), 0, m,
                               (const double*)s.Lc, (const double*)s.Jdc, p, s.pb, z, w);
        PF_LAUNCH_CHECK();
    }
    launch_spmv_border(s, z, w, 2);     // black rows and wells: the red rows are complete
}

// Mixed precision: FP32 multigrid and stage residual, BF16/FP32 smoother,
// FP32 output; the caller's Krylov vector v stays FP64.
void cpr_apply(Sim& s, const double* v, float* z) {
    const DevModel& m = s.m;
    if (s.opts.cpr_order == PF_CPR_PF) {
        const float* p = pressure_stage<float>(s, v);
        if (s.opts.smoother == PF_SMOOTH_RBILU0) {
            {
                ProfScope ps(s, PF_K_STAGE_RESID);
                launch<F_k_stage_ilu0<float, float, float>>(s, s.stream, (k_stage_ilu0<float, float, float>),
                                                            dim3(grid_for(m.n + m.nw)), dim3(kBlock), 0, m,
                                                            (const float*)s.Jp32, v, p, s.pb, s.B, s.pc_map,
                                                            s.pc_first, s.perf_well, (const float*)s.Dinv32, s.t32, z);
                PF_LAUNCH_CHECK();
            }
            smoother_apply_m(s, s.t32, z, 1);
        } else {
            {
                ProfScope ps(s, PF_K_STAGE_RESID);
                launch<F_k_stage_resid<float, float>>(s, s.stream, (k_stage_resid<float, float>), dim3(grid_for(m.n)),
                                                      dim3(kBlock), 0, m, (const float*)s.Jp32, v, p, s.t32);
                PF_LAUNCH_CHECK();
            }
            if (m.nw > 0) {
                launch<F_k_stage_resid_border<float>>(s, s.stream, k_stage_resid_border<float>,
                                                      dim3(grid_for(m.npc + m.nw, 64)), dim3(64), 0, m, s.pc_cell,
                                                      s.pc_first, s.perf_well, s.B, s.pb, s.t32);
                PF_LAUNCH_CHECK();
            }
            smoother_apply_m(s, s.t32, z);
        }
        launch<F_k_add_pressure<float>>(s, s.stream, k_add_pressure<float>, dim3(grid_for(m.n + m.nw)), dim3(kBlock),
                                        0, m.n, m.nw, p, s.pb, z);
        PF_LAUNCH_CHECK();
    } else {
        cast(s, s.nv, v, s.t32);
        smoother_apply_m(s, s.t32, z);
        launch_spmv(s, z, s.t2);
        launch_axpby(s, s.nv, 1.0, v, -1.0, s.t2);
        const float* p = pressure_stage<float>(s, s.t2);
        launch<F_k_add_pressure<float>>(s, s.stream, k_add_pressure<float>, dim3(grid_for(m.n + m.nw)), dim3(kBlock),
                                        0, m.n, m.nw, p, s.pb, z);
        PF_LAUNCH_CHECK();
    }
}

}  // namespace pf
