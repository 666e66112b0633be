// Two-stage CPR preconditioner (Sec. 3.4, Algorithm 2).
//
// Stage "P": the pressure block.  Its operator A_p is the P-column of the sum
// of the (row-scaled) water and oil equations - a total-volume combination
// of the two phase equations, which stays non-singular where the water
// relative permeability vanishes - and the restriction sums the water and
// oil residuals of a cell.  A_p is solved approximately by one multigrid
// V-cycle on the structured grid:
//   * smoother: z-line Gauss-Seidel, columns coloured as a checkerboard in
//     (x, y); each column's tridiagonal system is solved exactly with
//     factors precomputed at set-up (the vertical couplings of thin layers
//     are the strongest, so they are relaxed implicitly);
//   * coarsening: unsmoothed box aggregation with a Galerkin coarse operator,
//     which stays a 7-point stencil; only x and y are aggregated while a
//     level keeps >= 4096 columns, then 2x2x2;
//   * coarsest level (<= mg_coarse cells): dense inverse by Gauss-Jordan.
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

__global__ void k_extract_ap(int64_t n, const double* __restrict__ J, double* __restrict__ A) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int d = 0; d < 7; ++d) {
        const double* Jd = J + (int64_t)d * 9 * n;
        A[(int64_t)d * n + i] = Jd[0 * n + i] + Jd[3 * n + i];   // (water + oil) rows, P column
    }
}

struct Dims { int nx, ny, nz; };

// Galerkin coarse operator of box aggregation (piecewise-constant
// prolongation): couplings inside an aggregate fold into the coarse
// diagonal; couplings across its face in direction d become coarse
// coefficient d.
__global__ void k_galerkin(Dims f, Dims c, int cx, int cy, int cz, const double* __restrict__ Af,
                           double* __restrict__ Ac) {
    const int64_t nc = (int64_t)c.nx * c.ny * c.nz;
    const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nc) return;
    const int64_t nf = (int64_t)f.nx * f.ny * f.nz;
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
                const int64_t i = ix + (int64_t)f.nx * (iy + (int64_t)f.ny * iz);
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
    for (int d = 0; d < 7; ++d) Ac[(int64_t)d * nc + I] = acc[d];
}

// Thomas factors of every z-column: aux[0..n) = c'_k, aux[n..2n) = 1/den_k,
// aux[2n..3n) = -a_k/den_k (the forward recurrence d'_k = alpha_k d'_{k-1} +
// r_k/den_k).
__global__ void k_zline_setup(Dims g, const double* __restrict__ A, double* __restrict__ aux) {
    const int64_t nxy = (int64_t)g.nx * g.ny;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nxy) return;
    const int64_t n = nxy * g.nz;
    double cprev = 0.0;
    int64_t i = t;
    for (int k = 0; k < g.nz; ++k, i += nxy) {
        const double den = A[i] - A[5 * n + i] * cprev;
        const double id = 1.0 / den;
        const double cp = A[6 * n + i] * id;
        aux[i] = cp;
        aux[n + i] = id;
        aux[2 * n + i] = -A[5 * n + i] * id;
        cprev = cp;
    }
}

// One half-sweep of z-line Gauss-Seidel over the columns of one colour
// ((ix + iy) % 2 == colour).  With zero_init the neighbours are taken as 0
// (first half-sweep from a zero initial guess).
template <class T>
__global__ __launch_bounds__(256) void k_zline(Dims g, const T* __restrict__ A, const T* __restrict__ aux,
                                               const T* __restrict__ b, T* __restrict__ x, int colour,
                                               int zero_init) {
    const int hx = (g.nx + 1) >> 1;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)hx * g.ny) return;
    const int iy = (int)(t / hx);
    const int ix = 2 * (int)(t - (int64_t)iy * hx) + ((iy + colour) & 1);
    if (ix >= g.nx) return;
    const int64_t nxy = (int64_t)g.nx * g.ny;
    const int64_t n = nxy * g.nz;
    const bool xm = ix > 0, xp = ix + 1 < g.nx, ym = iy > 0, yp = iy + 1 < g.ny;
    int64_t i = ix + (int64_t)g.nx * iy;
    T dprev = 0;
    for (int k = 0; k < g.nz; ++k, i += nxy) {
        T r = b[i];
        if (!zero_init) {
            if (xm) r -= A[n + i] * x[i - 1];
            if (xp) r -= A[2 * n + i] * x[i + 1];
            if (ym) r -= A[3 * n + i] * x[i - g.nx];
            if (yp) r -= A[4 * n + i] * x[i + g.nx];
        }
        const T d = aux[2 * n + i] * dprev + r * aux[n + i];
        x[i] = d;
        dprev = d;
    }
    i -= nxy;
    T xn = x[i];
    for (int k = g.nz - 2; k >= 0; --k) {
        i -= nxy;
        const T v = x[i] - aux[i] * xn;
        x[i] = v;
        xn = v;
    }
}


// Segmented half-sweep of z-line Gauss-Seidel.  A block holds 64 consecutive
// columns of the active colour (one per lane) and nseg wavefronts; wavefront
// s owns layers [s*L, (s+1)*L) of those columns.  Both Thomas recurrences
// are affine in the carried value, so each segment first folds its cells
// into one affine map; the maps of the segments above (forward) or below
// (backward) are composed through LDS; then every segment finishes its own
// cells.  Loads are coalesced along x and the column work is spread over
// nseg times more wavefronts than a thread-per-column sweep.
template <int LMAX, class T>
__global__ __launch_bounds__(LMAX <= 8 ? 1024 : 512) void k_zline_seg(Dims g, const T* __restrict__ A,
                                                    const T* __restrict__ aux, const T* __restrict__ b,
                                                    T* __restrict__ x, int colour, int zero_init, int L) {
    __shared__ T sA[16][64];
    __shared__ T sB[16][64];
    const int lane = threadIdx.x & 63, seg = threadIdx.x >> 6;
    const int nseg = blockDim.x >> 6;
    const int hx = (g.nx + 1) >> 1;
    const int64_t tcol = xcd_block() * 64 + lane;
    bool active = tcol < (int64_t)hx * g.ny;
    int iy = 0, ix = 0;
    if (active) {
        iy = (int)(tcol / hx);
        ix = 2 * (int)(tcol - (int64_t)iy * hx) + ((iy + colour) & 1);
        active = ix < g.nx;
    }
    const int64_t nxy = (int64_t)g.nx * g.ny;
    const int64_t n = nxy * g.nz;
    const int k0 = seg * L;
    const int64_t i0 = ix + (int64_t)g.nx * iy + (int64_t)k0 * nxy;
    const bool xm = ix > 0, xp = ix + 1 < g.nx, ym = iy > 0, yp = iy + 1 < g.ny;
    T al[LMAX], be[LMAX], cp[LMAX];
    T Fa = 1, Fb = 0;
#pragma unroll
    for (int j = 0; j < LMAX; ++j) {
        al[j] = 1;
        be[j] = 0;
        cp[j] = 0;
        if (active && j < L && k0 + j < g.nz) {
            const int64_t i = i0 + (int64_t)j * nxy;
            cp[j] = aux[i];
            T r = b[i];
            if (!zero_init) {
                if (xm) r -= A[n + i] * x[i - 1];
                if (xp) r -= A[2 * n + i] * x[i + 1];
                if (ym) r -= A[3 * n + i] * x[i - g.nx];
                if (yp) r -= A[4 * n + i] * x[i + g.nx];
            }
            al[j] = aux[2 * n + i];
            be[j] = r * aux[n + i];
            Fb = al[j] * Fb + be[j];
            Fa = al[j] * Fa;
        }
    }
    sA[seg][lane] = Fa;
    sB[seg][lane] = Fb;
    __syncthreads();
    T y = 0;
    for (int q = 0; q < seg; ++q) y = sA[q][lane] * y + sB[q][lane];
    // forward values d'_k (kept in be); then this segment's backward map
#pragma unroll
    for (int j = 0; j < LMAX; ++j) {
        if (active && j < L && k0 + j < g.nz) {
            y = al[j] * y + be[j];
            be[j] = y;
        }
    }
    T Ga = 1, Gb = 0;
#pragma unroll
    for (int j = LMAX - 1; j >= 0; --j) {
        if (active && j < L && k0 + j < g.nz) {
            const T gm = -cp[j];
            al[j] = gm;
            Gb = gm * Gb + be[j];
            Ga = gm * Ga;
        }
    }
    __syncthreads();
    sA[seg][lane] = Ga;
    sB[seg][lane] = Gb;
    __syncthreads();
    T xin = 0;
    for (int q = nseg - 1; q > seg; --q) xin = sA[q][lane] * xin + sB[q][lane];
#pragma unroll
    for (int j = LMAX - 1; j >= 0; --j) {
        if (active && j < L && k0 + j < g.nz) {
            xin = al[j] * xin + be[j];
            x[i0 + (int64_t)j * nxy] = xin;
        }
    }
}

// Fine residual b - A x summed over each aggregate (restriction = P^T).
template <class T>
__global__ void k_resid_restrict(Dims f, Dims c, int cx, int cy, int cz, const T* __restrict__ A,
                                 const T* __restrict__ x, const T* __restrict__ b,
                                 T* __restrict__ bc) {
    const int64_t nc = (int64_t)c.nx * c.ny * c.nz;
    const int64_t I = xcd_block() * blockDim.x + threadIdx.x;
    if (I >= nc) return;
    const int64_t nf = (int64_t)f.nx * f.ny * f.nz;
    const int64_t fxy = (int64_t)f.nx * f.ny;
    const int64_t cxy = (int64_t)c.nx * c.ny;
    const int IZ = (int)(I / cxy);
    const int64_t rem = I - IZ * cxy;
    const int IY = (int)(rem / c.nx);
    const int IX = (int)(rem - (int64_t)IY * c.nx);
    T s = 0;
    // the aggregate has at most 2x2x2 cells; unrolled so all loads issue together
#pragma unroll
    for (int dz = 0; dz < 2; ++dz) {
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                const int iz = IZ * cz + dz, iy = IY * cy + dy, ix = IX * cx + dx;
                if (dz < cz && dy < cy && dx < cx && iz < f.nz && iy < f.ny && ix < f.nx) {
                    const int64_t i = ix + (int64_t)f.nx * (iy + (int64_t)f.ny * iz);
                    T r = b[i] - A[i] * x[i];
                    if (ix > 0) r -= A[nf + i] * x[i - 1];
                    if (ix + 1 < f.nx) r -= A[2 * nf + i] * x[i + 1];
                    if (iy > 0) r -= A[3 * nf + i] * x[i - f.nx];
                    if (iy + 1 < f.ny) r -= A[4 * nf + i] * x[i + f.nx];
                    if (iz > 0) r -= A[5 * nf + i] * x[i - fxy];
                    if (iz + 1 < f.nz) r -= A[6 * nf + i] * x[i + fxy];
                    s += r;
                }
            }
        }
    }
    bc[I] = s;
}

template <class T>
__global__ void k_prolong_add(Dims f, Dims c, int cx, int cy, int cz, const T* __restrict__ xc,
                              T* __restrict__ x) {
    const int64_t nf = (int64_t)f.nx * f.ny * f.nz;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nf) return;
    const int64_t fxy = (int64_t)f.nx * f.ny;
    const int iz = (int)(i / fxy);
    const int64_t rem = i - iz * fxy;
    const int iy = (int)(rem / f.nx);
    const int ix = (int)(rem - (int64_t)iy * f.nx);
    const int64_t I = (ix / cx) + (int64_t)c.nx * ((iy / cy) + (int64_t)c.ny * (iz / cz));
    x[i] += xc[I];
}

// Dense coarsest matrix (row-major, augmented with the identity: n x 2n).
__global__ void k_coarse_build(Dims g, const double* __restrict__ A, double* __restrict__ M) {
    const int64_t n = (int64_t)g.nx * g.ny * g.nz;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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

// Gauss-Jordan with partial pivoting on the augmented matrix, one block.
__global__ __launch_bounds__(1024) void k_gauss_jordan(int n, double* __restrict__ M) {
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


// Gauss-Jordan with partial pivoting in LDS for n <= kGJLds (augmented n x 2n
// matrix held in shared memory), result written back to M.
constexpr int kGJLds = 96;
__global__ __launch_bounds__(1024) void k_gauss_jordan_lds(int n, double* __restrict__ M) {
    extern __shared__ double sm[];
    double* S = sm;                       // n x 2n
    double* fcol = sm + 2 * n * n;        // n
    __shared__ int piv;
    const int W = 2 * n;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int idx = tid; idx < n * W; idx += nt) S[idx] = M[idx];
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        if (tid == 0) {
            double best = -1.0;
            int p = k;
            for (int r = k; r < n; ++r) {
                const double v = fabs(S[r * W + k]);
                if (v > best) { best = v; p = r; }
            }
            piv = p;
        }
        __syncthreads();
        const int p = piv;
        if (p != k)
            for (int c = tid; c < W; c += nt) {
                const double a = S[k * W + c];
                S[k * W + c] = S[p * W + c];
                S[p * W + c] = a;
            }
        __syncthreads();
        const double inv = 1.0 / S[k * W + k];
        __syncthreads();
        for (int c = tid; c < W; c += nt) S[k * W + c] *= inv;
        for (int r = tid; r < n; r += nt) fcol[r] = (r == k) ? 0.0 : S[r * W + k];
        __syncthreads();
        for (int idx = tid; idx < n * W; idx += nt) {
            const int r = idx / W;
            const double f = fcol[r];
            if (f != 0.0) S[idx] -= f * S[k * W + (idx - r * W)];
        }
        __syncthreads();
    }
    for (int idx = tid; idx < n * W; idx += nt) M[idx] = S[idx];
}

// The inverse (right half of the reduced augmented matrix) in compact n x n
// form, in FP64 and FP32.
__global__ void k_compact_inv(int n, const double* __restrict__ M, double* __restrict__ inv, float* __restrict__ inv32) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * n) return;
    const int64_t r = idx / n, c = idx - r * n;
    const double v = M[r * 2 * n + n + c];
    inv[idx] = v;
    if (inv32) inv32[idx] = (float)v;
}

// x = Minv b with the compact (n x n) coarsest inverse: one wavefront per
// row, lanes over the columns, fixed-order shuffle reduction.
template <class T>
__global__ __launch_bounds__(256) void k_coarse_apply(int n, const T* __restrict__ Minv, const T* __restrict__ b,
                                                      T* __restrict__ x) {
    const int r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= n) return;
    const T* row = Minv + (int64_t)r * n;
    T s = 0;
    for (int c = lane; c < n; c += 64) s += row[c] * b[c];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if (lane == 0) x[r] = s;
}

// Pressure restriction: water + oil residual of each cell.
template <class T>
__global__ void k_restrict_p(int64_t n, const double* __restrict__ v, T* __restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (T)(v[i] + v[n + i]);
}

// Well bottom-hole pressures of the pressure stage from the well rows:
// pb_w = (v_w - sum_perf dW/dP * p_cell) / D_w.  One 64-lane block per well.
template <class T>
__global__ __launch_bounds__(64) void k_well_pb(DevModel m, const int32_t* __restrict__ wp_first,
                                                const int32_t* __restrict__ wp_idx,
                                                const int32_t* __restrict__ perf_cell, const double* __restrict__ Cw,
                                                const double* __restrict__ Dw, const double* __restrict__ v,
                                                const T* __restrict__ p, double* __restrict__ pb) {
    const int w = blockIdx.x;
    double s = 0.0;
    for (int k = wp_first[w] + (int)threadIdx.x; k < wp_first[w + 1]; k += 64) {
        const int q = wp_idx[k];
        s += Cw[3 * q] * (double)p[perf_cell[q]];
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if (threadIdx.x == 0) pb[w] = (v[3 * m.n + w] - s) / Dw[w];
}

// t = v - J * Pi_p(p, pb) on the cells: only the P-columns of the blocks.
__global__ __launch_bounds__(256) void k_stage_resid(DevModel m, const double* __restrict__ J,
                                                     const double* __restrict__ v, const double* __restrict__ p,
                                                     double* __restrict__ t) {
    const int64_t i = xcd_block() * blockDim.x + threadIdx.x;
    if (i >= m.n) return;
    const int64_t n = m.n;
    const int64_t iz = i / m.nxy;
    const int64_t rem = i - iz * m.nxy;
    const int64_t iy = rem / m.nx;
    const int64_t ix = rem - iy * m.nx;
    const double pi = p[i];
    double t0 = v[i] - J[0 * n + i] * pi;
    double t1 = v[n + i] - J[3 * n + i] * pi;
    double t2 = v[2 * n + i] - J[6 * n + i] * pi;
    const bool ex[6] = {ix > 0, ix + 1 < m.nx, iy > 0, iy + 1 < m.ny, iz > 0, iz + 1 < m.nz};
    const int64_t off[6] = {-1, 1, -(int64_t)m.nx, (int64_t)m.nx, -m.nxy, m.nxy};
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        if (!ex[f]) continue;
        const double pj = p[i + off[f]];
        const double* B = J + (int64_t)(f + 1) * 9 * n + i;
        t0 -= B[0 * n] * pj;
        t1 -= B[3 * n] * pj;
        t2 -= B[6 * n] * pj;
    }
    t[i] = t0;
    t[n + i] = t1;
    t[2 * n + i] = t2;
}

// Border part of the stage residual: perforated cells subtract B * pb; the
// well rows are exactly satisfied by pb (their residual is 0).
template <class T>
__global__ void k_stage_resid_border(DevModel m, const int32_t* __restrict__ pc_cell,
                                     const int32_t* __restrict__ pc_first, const int32_t* __restrict__ perf_well,
                                     const double* __restrict__ B, const double* __restrict__ pb,
                                     T* __restrict__ t) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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

// z = Dinv t (block Jacobi on cells, 1/D on wells) + Pi_p(p, pb)
__global__ void k_bjac_apply_add(int64_t n, int nw, const double* __restrict__ Dinv, const double* __restrict__ Dw,
                                 const double* __restrict__ t, const double* __restrict__ p,
                                 const double* __restrict__ pb, double* __restrict__ z) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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

// z += Pi_p(p, pb)
template <class T>
__global__ void k_add_pressure(int64_t n, int nw, const T* __restrict__ p, const double* __restrict__ pb,
                               T* __restrict__ z) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) z[i] += p[i];
    else if (i < n + nw) z[3 * n + (i - n)] = (T)(z[3 * n + (i - n)] + pb[i - n]);
}

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

// colour 0 (red): Dinv = D^{-1}; colour 1 (black): Dinv = D~^{-1} (needs red done)
__global__ void k_ilu_setup(DevModel m, const double* __restrict__ J, double* __restrict__ Dinv, int colour) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m.n) return;
    int64_t ix, iy, iz;
    decode(m, i, ix, iy, iz);
    if (((ix + iy + iz) & 1) != colour) return;
    const int64_t n = m.n;
    double a[9];
    for (int e = 0; e < 9; ++e) a[e] = J[e * n + i];
    if (colour == 1) {
        const bool ex[6] = {ix > 0, ix + 1 < m.nx, iy > 0, iy + 1 < m.ny, iz > 0, iz + 1 < m.nz};
        const int64_t off[6] = {-1, 1, -(int64_t)m.nx, (int64_t)m.nx, -m.nxy, m.nxy};
        for (int f = 0; f < 6; ++f) {
            if (!ex[f]) continue;
            const int64_t r = i + off[f];
            const int fr = f ^ 1;       // direction from r back to i
            double Jbr[9], Jrb[9], Dr[9], T[9];
            for (int e = 0; e < 9; ++e) {
                Jbr[e] = J[((int64_t)(f + 1) * 9 + e) * n + i];
                Jrb[e] = J[((int64_t)(fr + 1) * 9 + e) * n + r];
                Dr[e] = Dinv[e * n + r];
            }
            // T = Dr * Jrb
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
    for (int e = 0; e < 9; ++e) Dinv[e * n + i] = r[e];
}

// Forward red: y_r = Dinv_r f_r.  Forward black: y_b = Dinv_b (f_b - sum J_br y_r).
// Backward red: z_r = y_r - Dinv_r sum J_rb z_b.  phase 0, 1, 2 respectively.
// The result is written to z (y and z share storage); p/pb are added in the
// last phase when given (stage-1 prolongation).
__global__ __launch_bounds__(256) void k_ilu_apply(DevModel m, const double* __restrict__ J,
                                                   const double* __restrict__ Dinv, const double* __restrict__ f,
                                                   double* __restrict__ z, int phase) {
    const int64_t i = xcd_block() * blockDim.x + threadIdx.x;
    if (i >= m.n) return;
    int64_t ix, iy, iz;
    decode(m, i, ix, iy, iz);
    const int col = (int)((ix + iy + iz) & 1);
    const int64_t n = m.n;
    if (phase == 0 && col != 0) return;
    if (phase == 1 && col != 1) return;
    if (phase == 2 && col != 0) return;
    double t0, t1, t2;
    if (phase == 2) { t0 = 0.0; t1 = 0.0; t2 = 0.0; }
    else { t0 = f[i]; t1 = f[n + i]; t2 = f[2 * n + i]; }
    if (phase >= 1) {
        const bool ex[6] = {ix > 0, ix + 1 < m.nx, iy > 0, iy + 1 < m.ny, iz > 0, iz + 1 < m.nz};
        const int64_t off[6] = {-1, 1, -(int64_t)m.nx, (int64_t)m.nx, -m.nxy, m.nxy};
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            if (!ex[q]) continue;
            const int64_t j = i + off[q];
            const double a = z[j], b = z[n + j], c = z[2 * n + j];
            const double* B = J + (int64_t)(q + 1) * 9 * n + i;
            s0 += B[0 * n] * a + B[1 * n] * b + B[2 * n] * c;
            s1 += B[3 * n] * a + B[4 * n] * b + B[5 * n] * c;
            s2 += B[6 * n] * a + B[7 * n] * b + B[8 * n] * c;
        }
        t0 -= s0; t1 -= s1; t2 -= s2;
    }
    const double u0 = Dinv[0 * n + i] * t0 + Dinv[1 * n + i] * t1 + Dinv[2 * n + i] * t2;
    const double u1 = Dinv[3 * n + i] * t0 + Dinv[4 * n + i] * t1 + Dinv[5 * n + i] * t2;
    const double u2 = Dinv[6 * n + i] * t0 + Dinv[7 * n + i] * t1 + Dinv[8 * n + i] * t2;
    if (phase == 2) {
        z[i] += u0; z[n + i] += u1; z[2 * n + i] += u2;
    } else {
        z[i] = u0; z[n + i] = u1; z[2 * n + i] = u2;
    }
}

template <class T>
__global__ void k_well_diag(int64_t n, int nw, const double* __restrict__ Dw, const T* __restrict__ f,
                            T* __restrict__ z) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w < nw) z[3 * n + w] = (T)(f[3 * n + w] / Dw[w]);
}


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

__global__ void k_cast_f32(int64_t n, const double* __restrict__ src, float* __restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (float)src[i];
}

// Jp32[(d*3 + row)*n + i]: FP32 P-columns of the 7 blocks (stage residual);
// Joff16[(q*9 + e)*n + i]: BF16 off-diagonal blocks q = 0..5 (-x..+z) (ILU).
__global__ void k_extract_lowp(int64_t n, const double* __restrict__ J, float* __restrict__ Jp32,
                               uint16_t* __restrict__ Joff16) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int d = 0; d < 7; ++d)
        for (int r = 0; r < 3; ++r) Jp32[(int64_t)(d * 3 + r) * n + i] = (float)J[(int64_t)(d * 9 + 3 * r) * n + i];
    if (Joff16)
        for (int q = 0; q < 6; ++q)
            for (int e = 0; e < 9; ++e)
                Joff16[(int64_t)(q * 9 + e) * n + i] = f32_to_bf16((float)J[(int64_t)((q + 1) * 9 + e) * n + i]);
}

// FP32 stage residual t = v - J Pi_p p (cells), FP32 accumulation.
__global__ __launch_bounds__(256) void k_stage_resid_m(DevModel m, const float* __restrict__ Jp,
                                                       const double* __restrict__ v, const float* __restrict__ p,
                                                       float* __restrict__ t) {
    const int64_t i = xcd_block() * blockDim.x + threadIdx.x;
    if (i >= m.n) return;
    const int64_t n = m.n;
    const int64_t iz = i / m.nxy;
    const int64_t rem = i - iz * m.nxy;
    const int64_t iy = rem / m.nx;
    const int64_t ix = rem - iy * m.nx;
    const float pi = p[i];
    float t0 = (float)v[i] - Jp[0 * n + i] * pi;
    float t1 = (float)v[n + i] - Jp[1 * n + i] * pi;
    float t2 = (float)v[2 * n + i] - Jp[2 * n + i] * pi;
    const bool ex[6] = {ix > 0, ix + 1 < m.nx, iy > 0, iy + 1 < m.ny, iz > 0, iz + 1 < m.nz};
    const int64_t off[6] = {-1, 1, -(int64_t)m.nx, (int64_t)m.nx, -m.nxy, m.nxy};
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        if (!ex[f]) continue;
        const float pj = p[i + off[f]];
        const float* B = Jp + (int64_t)(f + 1) * 3 * n + i;
        t0 -= B[0 * n] * pj;
        t1 -= B[1 * n] * pj;
        t2 -= B[2 * n] * pj;
    }
    t[i] = t0;
    t[n + i] = t1;
    t[2 * n + i] = t2;
}

// Red-black block ILU(0) apply with BF16 off-diagonal blocks, FP32 inverse
// diagonals and FP32 vectors (phases as in k_ilu_apply).
__global__ __launch_bounds__(256) void k_ilu_apply_m(DevModel m, const uint16_t* __restrict__ Joff,
                                                     const float* __restrict__ Dinv, const float* __restrict__ f,
                                                     float* __restrict__ z, int phase) {
    const int64_t i = xcd_block() * blockDim.x + threadIdx.x;
    if (i >= m.n) return;
    const int64_t n = m.n;
    const int64_t iz = i / m.nxy;
    const int64_t rem = i - iz * m.nxy;
    const int64_t iy = rem / m.nx;
    const int64_t ix = rem - iy * m.nx;
    const int col = (int)((ix + iy + iz) & 1);
    if ((phase == 1) != (col == 1)) return;
    float t0, t1, t2;
    if (phase == 2) { t0 = 0.f; t1 = 0.f; t2 = 0.f; }
    else { t0 = f[i]; t1 = f[n + i]; t2 = f[2 * n + i]; }
    if (phase >= 1) {
        const bool ex[6] = {ix > 0, ix + 1 < m.nx, iy > 0, iy + 1 < m.ny, iz > 0, iz + 1 < m.nz};
        const int64_t off[6] = {-1, 1, -(int64_t)m.nx, (int64_t)m.nx, -m.nxy, m.nxy};
        float s0 = 0.f, s1 = 0.f, s2 = 0.f;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            if (!ex[q]) continue;
            const int64_t j = i + off[q];
            const float a = z[j], b = z[n + j], c = z[2 * n + j];
            const uint16_t* B = Joff + (int64_t)q * 9 * n + i;
            s0 += bf16_to_f32(B[0 * n]) * a + bf16_to_f32(B[1 * n]) * b + bf16_to_f32(B[2 * n]) * c;
            s1 += bf16_to_f32(B[3 * n]) * a + bf16_to_f32(B[4 * n]) * b + bf16_to_f32(B[5 * n]) * c;
            s2 += bf16_to_f32(B[6 * n]) * a + bf16_to_f32(B[7 * n]) * b + bf16_to_f32(B[8 * n]) * c;
        }
        t0 -= s0; t1 -= s1; t2 -= s2;
    }
    const float u0 = Dinv[0 * n + i] * t0 + Dinv[1 * n + i] * t1 + Dinv[2 * n + i] * t2;
    const float u1 = Dinv[3 * n + i] * t0 + Dinv[4 * n + i] * t1 + Dinv[5 * n + i] * t2;
    const float u2 = Dinv[6 * n + i] * t0 + Dinv[7 * n + i] * t1 + Dinv[8 * n + i] * t2;
    if (phase == 2) {
        z[i] += u0; z[n + i] += u1; z[2 * n + i] += u2;
    } else {
        z[i] = u0; z[n + i] = u1; z[2 * n + i] = u2;
    }
}

// FP32 block Jacobi: z = Dinv t (cells), t / D (wells)
__global__ void k_bjac_apply_m(int64_t n, int nw, const float* __restrict__ Dinv, const double* __restrict__ Dw,
                               const float* __restrict__ t, float* __restrict__ z) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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

Dims dims_of(const MGLevel& L) { return Dims{L.nx, L.ny, L.nz}; }

// Level arrays in the precision of the apply.
template <class T> struct Lv;
template <> struct Lv<double> {
    static const double* A(const MGLevel& L) { return L.A; }
    static const double* aux(const MGLevel& L) { return L.aux; }
    static double* x(const MGLevel& L) { return L.x; }
    static double* b(const MGLevel& L) { return L.b; }
    static const double* inv(const Sim& s) { return s.coarse_inv; }
};
template <> struct Lv<float> {
    static const float* A(const MGLevel& L) { return L.A32; }
    static const float* aux(const MGLevel& L) { return L.aux32; }
    static float* x(const MGLevel& L) { return L.x32; }
    static float* b(const MGLevel& L) { return L.b32; }
    static const float* inv(const Sim& s) { return s.coarse_inv32; }
};

// One z-line half-sweep of level L: the segmented kernel when the column
// height allows (<= 384 layers), else thread-per-column.
template <class T>
void zline_sweep(Sim& s, const MGLevel& L, int colour, int zero_init) {
    const Dims g = dims_of(L);
    const int64_t cols = (int64_t)((L.nx + 1) / 2) * L.ny;
    const T* A = Lv<T>::A(L);
    const T* aux = Lv<T>::aux(L);
    T* x = Lv<T>::x(L);
    const T* b = Lv<T>::b(L);
    // up to 16 segments of <= 8 layers, or 8 segments of <= 24 / <= 48 layers
    const int lmax = L.nz <= 128 ? 8 : L.nz <= 192 ? 24 : L.nz <= 384 ? 48 : 0;
    if (lmax > 0) {
        const int nseg = (L.nz + lmax - 1) / lmax;
        const int len = (L.nz + nseg - 1) / nseg;
        const unsigned blocks = (unsigned)((cols + 63) / 64);
        if (lmax == 8)
            hipLaunchKernelGGL((k_zline_seg<8, T>), dim3(blocks), dim3(64 * nseg), 0, s.stream, g, A, aux, b, x,
                               colour, zero_init, len);
        else if (lmax == 24)
            hipLaunchKernelGGL((k_zline_seg<24, T>), dim3(blocks), dim3(64 * nseg), 0, s.stream, g, A, aux, b, x,
                               colour, zero_init, len);
        else
            hipLaunchKernelGGL((k_zline_seg<48, T>), dim3(blocks), dim3(64 * nseg), 0, s.stream, g, A, aux, b, x,
                               colour, zero_init, len);
    } else {
        hipLaunchKernelGGL(k_zline<T>, dim3(grid_for(cols)), dim3(kBlock), 0, s.stream, g, A, aux, b, x, colour,
                           zero_init);
    }
    PF_LAUNCH_CHECK();
}

unsigned cast_grid(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > 8192) g = 8192;
    return (unsigned)(g > 0 ? g : 1);
}

void cast(Sim& s, int64_t n, const double* src, float* dst) {
    hipLaunchKernelGGL(k_cast_f32, dim3(cast_grid(n)), dim3(kBlock), 0, s.stream, n, src, dst);
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
        if (L.n <= cmax) { L.cx = L.cy = L.cz = 1; s.mg.push_back(L); break; }
        const int64_t cols = (int64_t)L.nx * L.ny;
        int cx = L.nx > 1 ? 2 : 1, cy = L.ny > 1 ? 2 : 1;
        int cz = (cols >= kColsForXY || L.nz == 1) ? 1 : 2;
        if (cols < kColsForXY && cx == 1 && cy == 1) cz = 2;
        if (cx == 1 && cy == 1 && cz == 1) { L.cx = L.cy = L.cz = 1; s.mg.push_back(L); break; }
        L.cx = cx; L.cy = cy; L.cz = cz;
        s.mg.push_back(L);
        MGLevel C{};
        C.nx = (L.nx + cx - 1) / cx;
        C.ny = (L.ny + cy - 1) / cy;
        C.nz = (L.nz + cz - 1) / cz;
        C.n = (int64_t)C.nx * C.ny * C.nz;
        L = C;
    }
}

void cpr_plan(Sim& s, Bump& b) {
    const int nl = (int)s.mg.size();
    const bool mixed = s.opts.precision == PF_PREC_MIXED;
    for (int l = 0; l < nl; ++l) {
        MGLevel& L = s.mg[l];
        L.A = b.take<double>(7 * L.n);
        L.aux = b.take<double>(3 * L.n);
        L.x = b.take<double>(L.n);
        L.b = b.take<double>(L.n);
        L.r = nullptr;
        if (mixed) {
            L.A32 = b.take<float>(7 * L.n);
            L.aux32 = b.take<float>(3 * L.n);
            L.x32 = b.take<float>(L.n);
            L.b32 = b.take<float>(L.n);
        }
    }
    s.Ap = s.mg[0].A;
    const int64_t nc = s.mg.back().n;
    s.coarse_aug = b.take<double>((size_t)nc * 2 * nc);
    s.coarse_inv = b.take<double>((size_t)nc * nc);
    s.pb = b.take<double>(std::max(s.m.nw, 1));
    s.Dinv = b.take<double>(9 * s.m.n);
    if (mixed) {
        s.coarse_inv32 = b.take<float>((size_t)nc * nc);
        s.Jp32 = b.take<float>(21 * s.m.n);
        s.Joff16 = b.take<uint16_t>(54 * s.m.n);
        s.Dinv32 = b.take<float>(9 * s.m.n);
        s.t32 = b.take<float>(s.nv);
    }
}

void cpr_setup(Sim& s) {
    const DevModel& m = s.m;
    const int nl = (int)s.mg.size();
    const bool mixed = s.opts.precision == PF_PREC_MIXED;
    hipLaunchKernelGGL(k_extract_ap, dim3(grid_for(m.n)), dim3(kBlock), 0, s.stream, m.n, s.J, s.mg[0].A);
    PF_LAUNCH_CHECK();
    for (int l = 0; l + 1 < nl; ++l) {
        const MGLevel& F = s.mg[l];
        const MGLevel& C = s.mg[l + 1];
        hipLaunchKernelGGL(k_galerkin, dim3(grid_for(C.n)), dim3(kBlock), 0, s.stream, dims_of(F), dims_of(C), F.cx,
                           F.cy, F.cz, F.A, C.A);
        PF_LAUNCH_CHECK();
    }
    for (int l = 0; l + 1 < nl; ++l) {
        const MGLevel& L = s.mg[l];
        hipLaunchKernelGGL(k_zline_setup, dim3(grid_for((int64_t)L.nx * L.ny)), dim3(kBlock), 0, s.stream,
                           dims_of(L), L.A, L.aux);
        PF_LAUNCH_CHECK();
    }
    const MGLevel& Cn = s.mg.back();
    hipLaunchKernelGGL(k_coarse_build, dim3(grid_for(Cn.n, 64)), dim3(64), 0, s.stream, dims_of(Cn), Cn.A,
                       s.coarse_aug);
    PF_LAUNCH_CHECK();
    const size_t lds = (size_t)(2 * Cn.n * Cn.n + Cn.n) * sizeof(double);
    if (Cn.n <= kGJLds && lds <= (size_t)s.max_lds) {
        hipLaunchKernelGGL(k_gauss_jordan_lds, dim3(1), dim3(1024), lds, s.stream, (int)Cn.n, s.coarse_aug);
    } else {
        hipLaunchKernelGGL(k_gauss_jordan, dim3(1), dim3(1024), 0, s.stream, (int)Cn.n, s.coarse_aug);
    }
    PF_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_compact_inv, dim3(grid_for(Cn.n * Cn.n)), dim3(kBlock), 0, s.stream, (int)Cn.n,
                       s.coarse_aug, s.coarse_inv, mixed ? s.coarse_inv32 : (float*)nullptr);
    PF_LAUNCH_CHECK();
    if (s.opts.smoother == PF_SMOOTH_RBILU0) {
        hipLaunchKernelGGL(k_ilu_setup, dim3(grid_for(m.n)), dim3(kBlock), 0, s.stream, m, s.J, s.Dinv, 0);
        PF_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_ilu_setup, dim3(grid_for(m.n)), dim3(kBlock), 0, s.stream, m, s.J, s.Dinv, 1);
        PF_LAUNCH_CHECK();
    } else {
        launch_bjac_setup(s);
    }
    if (mixed) {
        for (int l = 0; l < nl; ++l) {
            const MGLevel& L = s.mg[l];
            cast(s, 7 * L.n, L.A, L.A32);
            cast(s, 3 * L.n, L.aux, L.aux32);
        }
        hipLaunchKernelGGL(k_extract_lowp, dim3(grid_for(m.n)), dim3(kBlock), 0, s.stream, m.n, s.J, s.Jp32,
                           s.opts.smoother == PF_SMOOTH_RBILU0 ? s.Joff16 : (uint16_t*)nullptr);
        PF_LAUNCH_CHECK();
        cast(s, 9 * m.n, s.Dinv, s.Dinv32);
    }
}

namespace {

template <class T>
void vcycle(Sim& s, int l, int zero_init0 = 1) {
    const int nl = (int)s.mg.size();
    MGLevel& L = s.mg[l];
    if (l == nl - 1) {
        hipLaunchKernelGGL(k_coarse_apply<T>, dim3((unsigned)((L.n + 3) / 4)), dim3(256), 0, s.stream, (int)L.n,
                           Lv<T>::inv(s), Lv<T>::b(L), Lv<T>::x(L));
        PF_LAUNCH_CHECK();
        return;
    }
    const Dims g = dims_of(L);
    const int pre = std::max(1, s.opts.mg_pre), post = std::max(0, s.opts.mg_post);
    for (int it = 0; it < pre; ++it) {
        {
            ProfScope ps(s, l == 0 ? PF_K_ZLINE : 0);
            zline_sweep<T>(s, L, 0, (it == 0 && zero_init0) ? 1 : 0);
        }
        zline_sweep<T>(s, L, 1, 0);
    }
    MGLevel& C = s.mg[l + 1];
    hipLaunchKernelGGL(k_resid_restrict<T>, dim3(grid_for(C.n)), dim3(kBlock), 0, s.stream, g, dims_of(C), L.cx,
                       L.cy, L.cz, Lv<T>::A(L), Lv<T>::x(L), Lv<T>::b(L), Lv<T>::b(C));
    PF_LAUNCH_CHECK();
    vcycle<T>(s, l + 1);
    hipLaunchKernelGGL(k_prolong_add<T>, dim3(grid_for(L.n)), dim3(kBlock), 0, s.stream, g, dims_of(C), L.cx, L.cy,
                       L.cz, Lv<T>::x(C), Lv<T>::x(L));
    PF_LAUNCH_CHECK();
    for (int it = 0; it < post; ++it) {
        zline_sweep<T>(s, L, 1, 0);
        zline_sweep<T>(s, L, 0, 0);
    }
}

}  // namespace

void mg_smooth_once(Sim& s, int level, int colour, int zero_init) {
    zline_sweep<double>(s, s.mg[level], colour, zero_init);
}

namespace {

// Pressure stage: b = Pi_r v; p = V-cycle(s); well pressures from the well rows.
template <class T>
void pressure_stage(Sim& s, const double* v) {
    const DevModel& m = s.m;
    hipLaunchKernelGGL(k_restrict_p<T>, dim3(grid_for(m.n)), dim3(kBlock), 0, s.stream, m.n, v, Lv<T>::b(s.mg[0]));
    PF_LAUNCH_CHECK();
    const int cycles = std::max(1, s.opts.mg_cycles);
    for (int c = 0; c < cycles; ++c) vcycle<T>(s, 0, c == 0 ? 1 : 0);
    if (m.nw > 0) {
        hipLaunchKernelGGL(k_well_pb<T>, dim3(m.nw), dim3(64), 0, s.stream, m, s.wp_first, s.wp_idx, s.perf_cell,
                           s.Cw, s.Dw, v, (const T*)Lv<T>::x(s.mg[0]), s.pb);
        PF_LAUNCH_CHECK();
    }
}

void smoother_apply(Sim& s, const double* f, double* z) {
    const DevModel& m = s.m;
    if (s.opts.smoother == PF_SMOOTH_RBILU0) {
        for (int ph = 0; ph < 3; ++ph) {
            ProfScope ps(s, ph == 1 ? PF_K_ILU : 0);
            hipLaunchKernelGGL(k_ilu_apply, dim3(grid_for(m.n)), dim3(kBlock), 0, s.stream, m, s.J, s.Dinv, f, z, ph);
            PF_LAUNCH_CHECK();
        }
        if (m.nw > 0) {
            hipLaunchKernelGGL(k_well_diag<double>, dim3(grid_for(m.nw, 64)), dim3(64), 0, s.stream, m.n, m.nw, s.Dw,
                               f, z);
            PF_LAUNCH_CHECK();
        }
    } else {
        hipLaunchKernelGGL(k_bjac_apply_add, dim3(grid_for(m.n + m.nw)), dim3(kBlock), 0, s.stream, m.n, m.nw,
                           s.Dinv, s.Dw, f, (const double*)nullptr, (const double*)nullptr, z);
        PF_LAUNCH_CHECK();
    }
}

void smoother_apply_m(Sim& s, const float* f, float* z) {
    const DevModel& m = s.m;
    if (s.opts.smoother == PF_SMOOTH_RBILU0) {
        for (int ph = 0; ph < 3; ++ph) {
            ProfScope ps(s, ph == 1 ? PF_K_ILU : 0);
            hipLaunchKernelGGL(k_ilu_apply_m, dim3(grid_for(m.n)), dim3(kBlock), 0, s.stream, m, s.Joff16, s.Dinv32, f,
                               z, ph);
            PF_LAUNCH_CHECK();
        }
        if (m.nw > 0) {
            hipLaunchKernelGGL(k_well_diag<float>, dim3(grid_for(m.nw, 64)), dim3(64), 0, s.stream, m.n, m.nw, s.Dw,
                               f, z);
            PF_LAUNCH_CHECK();
        }
    } else {
        hipLaunchKernelGGL(k_bjac_apply_m, dim3(grid_for(m.n + m.nw)), dim3(kBlock), 0, s.stream, m.n, m.nw, s.Dinv32,
                           s.Dw, f, z);
        PF_LAUNCH_CHECK();
    }
}

}  // namespace

void cpr_apply(Sim& s, const double* v, double* z) {
    const DevModel& m = s.m;
    if (s.opts.cpr_order == PF_CPR_PF) {
        pressure_stage<double>(s, v);
        {
            ProfScope ps(s, PF_K_STAGE_RESID);
            hipLaunchKernelGGL(k_stage_resid, dim3(grid_for(m.n)), dim3(kBlock), 0, s.stream, m, s.J, v, s.mg[0].x,
                               s.t2);
            PF_LAUNCH_CHECK();
        }
        if (m.nw > 0) {
            hipLaunchKernelGGL(k_stage_resid_border<double>, dim3(grid_for(m.npc + m.nw, 64)), dim3(64), 0, s.stream, m,
                               s.pc_cell, s.pc_first, s.perf_well, s.B, s.pb, s.t2);
            PF_LAUNCH_CHECK();
        }
        smoother_apply(s, s.t2, z);
        hipLaunchKernelGGL(k_add_pressure<double>, dim3(grid_for(m.n + m.nw)), dim3(kBlock), 0, s.stream, m.n, m.nw,
                           s.mg[0].x, s.pb, z);
        PF_LAUNCH_CHECK();
    } else {
        // Algorithm 2: y = S(v); r = v - J y; y += Pi_p M_g^{-1} Pi_r r
        smoother_apply(s, v, z);
        launch_spmv(s, z, s.t2);
        launch_axpby(s, s.nv, 1.0, v, -1.0, s.t2);
        pressure_stage<double>(s, s.t2);
        hipLaunchKernelGGL(k_add_pressure<double>, dim3(grid_for(m.n + m.nw)), dim3(kBlock), 0, s.stream, m.n, m.nw,
                           s.mg[0].x, s.pb, z);
        PF_LAUNCH_CHECK();
    }
}

// Mixed precision: FP32 multigrid and stage residual, BF16/FP32 smoother,
// FP32 output; the caller's Krylov vector v stays FP64.
void cpr_apply(Sim& s, const double* v, float* z) {
    const DevModel& m = s.m;
    if (s.opts.cpr_order == PF_CPR_PF) {
        pressure_stage<float>(s, v);
        {
            ProfScope ps(s, PF_K_STAGE_RESID);
            hipLaunchKernelGGL(k_stage_resid_m, dim3(grid_for(m.n)), dim3(kBlock), 0, s.stream, m, s.Jp32, v,
                               s.mg[0].x32, s.t32);
            PF_LAUNCH_CHECK();
        }
        if (m.nw > 0) {
            hipLaunchKernelGGL(k_stage_resid_border<float>, dim3(grid_for(m.npc + m.nw, 64)), dim3(64), 0, s.stream, m,
                               s.pc_cell, s.pc_first, s.perf_well, s.B, s.pb, s.t32);
            PF_LAUNCH_CHECK();
        }
        smoother_apply_m(s, s.t32, z);
        hipLaunchKernelGGL(k_add_pressure<float>, dim3(grid_for(m.n + m.nw)), dim3(kBlock), 0, s.stream, m.n, m.nw,
                           s.mg[0].x32, s.pb, z);
        PF_LAUNCH_CHECK();
    } else {
        cast(s, s.nv, v, s.t32);
        smoother_apply_m(s, s.t32, z);
        launch_spmv(s, z, s.t2);
        launch_axpby(s, s.nv, 1.0, v, -1.0, s.t2);
        pressure_stage<float>(s, s.t2);
        hipLaunchKernelGGL(k_add_pressure<float>, dim3(grid_for(m.n + m.nw)), dim3(kBlock), 0, s.stream, m.n, m.nw,
                           s.mg[0].x32, s.pb, z);
        PF_LAUNCH_CHECK();
    }
}

}  // namespace pf
