// Linear algebra kernels of the flexible GMRES solve: stencil block SpMV
// with the well border, vector updates, block-Jacobi, and the Arnoldi
// process (classical Gram-Schmidt with re-orthogonalisation, Hessenberg and
// Givens rotations kept on the device).
#include "pf_internal.h"

#include <algorithm>
#include <cfloat>

namespace pf {
namespace {

// J is streamed once per product (it does not fit the caches): non-temporal
// loads keep the caches for x.
__device__ __forceinline__ double jld(const double* p) { return __builtin_nontemporal_load(p); }

// y = J x over the cells: 7 neighbour blocks, each 3x3, stored as 63 planes.
// Entry (oil row, C column) of every block is zero (the oil equation does
// not involve the polymer concentration; the assembly writes 0 there), so
// those 7 planes are not read.  x may be FP32 (the preconditioned vectors of the mixed-precision mode);
// the product is FP64.
template <class TX>
__device__ __forceinline__ void k_spmv_d(const Blk& wg, DevModel m, const double* __restrict__ J,
                                         const TX* __restrict__ x, double* __restrict__ y) {
    const int64_t i = xcd_block(wg) * blockDim.x + threadIdx.x;
    if (i >= m.n) return;
    const int64_t n = m.n;
    const int64_t iz = i / m.nxy;
    const int64_t rem = i - iz * m.nxy;
    const int64_t iy = rem / m.nx;
    const int64_t ix = rem - iy * m.nx;
    double y0, y1, y2;
    {
        const double a = (double)x[i], b = (double)x[n + i], c = (double)x[2 * n + i];
        y0 = jld(J + 0 * n + i) * a + jld(J + 1 * n + i) * b + jld(J + 2 * n + i) * c;
        y1 = jld(J + 3 * n + i) * a + jld(J + 4 * n + i) * b;
        y2 = jld(J + 6 * n + i) * a + jld(J + 7 * n + i) * b + jld(J + 8 * n + i) * c;
    }
    const bool ex[6] = {ix > 0, ix + 1 < m.nx, iy > 0, iy + 1 < m.ny, iz > 0, iz + 1 < m.nz};
    const int64_t off[6] = {-1, 1, -(int64_t)m.nx, (int64_t)m.nx, -m.nxy, m.nxy};
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        if (!ex[f]) continue;
        const int64_t j = i + off[f];
        const double* B = J + (int64_t)(f + 1) * 9 * n + i;
        const double a = (double)x[j], b = (double)x[n + j], c = (double)x[2 * n + j];
        y0 += jld(B + 0 * n) * a + jld(B + 1 * n) * b + jld(B + 2 * n) * c;
        y1 += jld(B + 3 * n) * a + jld(B + 4 * n) * b;
        y2 += jld(B + 6 * n) * a + jld(B + 7 * n) * b + jld(B + 8 * n) * c;
    }
    y[i] = y0;
    y[n + i] = y1;
    y[2 * n + i] = y2;
}
template <class TX>
__global__ __launch_bounds__(256) void k_spmv(DevModel m, const double* __restrict__ J, const TX* __restrict__ x,
                                              double* __restrict__ y) {
    k_spmv_d<TX>(PF_BLK, m, J, x, y);
}
template <class TX>
struct F_k_spmv {
    static constexpr int kLB = 256;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_spmv_d<TX>(wg, a...);
    }
};

// Well border of y = J x: perforated cells add B * Pb (one thread per
// perforated cell, blocks [0, ncb)); well rows are sum C * x_cell + D * Pb
// (one 64-lane block per well after those, lanes over the perforations,
// fixed-order shuffle reduction).
template <class TX>
__device__ __forceinline__ void k_spmv_border_d(const Blk& wg, DevModel m, int ncb,
                                                const int32_t* __restrict__ pc_cell,
                                                const int32_t* __restrict__ pc_first,
                                                const int32_t* __restrict__ perf_well,
                                                const int32_t* __restrict__ perf_cell,
                                                const int32_t* __restrict__ wp_first,
                                                const int32_t* __restrict__ wp_idx, const double* __restrict__ B,
                                                const double* __restrict__ Cw, const double* __restrict__ Dw,
                                                const TX* __restrict__ x, double* __restrict__ y, int cs) {
    // plane length and a cell's offset in the natural (cs 0) or the colour-split
    // layout (cs 1; cs 2: the cell rows of black cells only, the wells' rows all)
    const int64_t n = cs ? 2 * cs_ns(m) : m.n;
    if ((int)wg.x < ncb) {
        const int64_t t = (int64_t)wg.x * blockDim.x + threadIdx.x;
        if (t >= m.npc) return;
        const int64_t i = cs ? cs_index(m, pc_cell[t]) : pc_cell[t];
        if (cs == 2 && i < cs_ns(m)) return;             // red rows left as they are
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        for (int64_t k = pc_first[t]; k < pc_first[t + 1]; ++k) {
            const double pb = (double)x[3 * n + perf_well[k]];
            a0 += B[3 * k] * pb;
            a1 += B[3 * k + 1] * pb;
            a2 += B[3 * k + 2] * pb;
        }
        y[i] += a0;
        y[n + i] += a1;
        y[2 * n + i] += a2;
        return;
    }
    const int w = (int)wg.x - ncb;
    double s = 0.0;
    for (int k = wp_first[w] + (int)threadIdx.x; k < wp_first[w + 1]; k += 64) {
        const int p = wp_idx[k];
        const int64_t c = cs ? cs_index(m, perf_cell[p]) : perf_cell[p];
        s += Cw[3 * p] * (double)x[c] + Cw[3 * p + 1] * (double)x[n + c] + Cw[3 * p + 2] * (double)x[2 * n + c];
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if (threadIdx.x == 0) y[3 * n + w] = s + Dw[w] * (double)x[3 * n + w];
}
template <class TX>
__global__ __launch_bounds__(64) void k_spmv_border(DevModel m, int ncb, const int32_t* __restrict__ pc_cell,
                                                    const int32_t* __restrict__ pc_first,
                                                    const int32_t* __restrict__ perf_well,
                                                    const int32_t* __restrict__ perf_cell,
                                                    const int32_t* __restrict__ wp_first,
                                                    const int32_t* __restrict__ wp_idx, const double* __restrict__ B,
                                                    const double* __restrict__ Cw, const double* __restrict__ Dw,
                                                    const TX* __restrict__ x, double* __restrict__ y, int cs) {
    k_spmv_border_d<TX>(PF_BLK, m, ncb, pc_cell, pc_first, perf_well, perf_cell, wp_first, wp_idx, B, Cw, Dw, x, y,
                        cs);
}
template <class TX>
struct F_k_spmv_border {
    static constexpr int kLB = 64;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_spmv_border_d<TX>(wg, a...);
    }
};

// Natural -> colour-split layout, times scale (pad slots get zero), and
// back; wells copied.
__device__ __forceinline__ void k_to_cs_d(const Blk& wg, DevModel m, const double* __restrict__ x,
                                          double* __restrict__ y, double scale) {
    const int64_t ns = cs_ns(m), lp = 2 * ns;
    const int64_t q = (int64_t)wg.x * blockDim.x + threadIdx.x;
    if (q >= 3 * lp + m.nw) return;
    if (q >= 3 * lp) { y[q] = scale * x[3 * m.n + (q - 3 * lp)]; return; }
    const int64_t e = q / lp, r = q - e * lp;
    const int c = r >= ns ? 1 : 0;
    const int64_t sl = r - c * ns;
    const int64_t hx = (m.nx + 1) >> 1;
    const int64_t line = sl / hx, t = sl - line * hx;
    const int64_t iz = line / m.ny, iy = line - iz * m.ny;
    const int64_t ix = 2 * t + ((c + iy + iz) & 1);
    y[q] = ix < m.nx ? scale * x[e * m.n + ix + m.nx * iy + m.nxy * iz] : 0.0;
}
__global__ void k_to_cs(DevModel m, const double* __restrict__ x, double* __restrict__ y, double scale) {
    k_to_cs_d(PF_BLK, m, x, y, scale);
}
struct F_k_to_cs {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_to_cs_d(wg, a...);
    }
};

__device__ __forceinline__ void k_from_cs_d(const Blk& wg, DevModel m, const double* __restrict__ x,
                                            double* __restrict__ y) {
    const int64_t lp = 2 * cs_ns(m);
    const int64_t q = (int64_t)wg.x * blockDim.x + threadIdx.x;
    if (q >= 3 * m.n + m.nw) return;
    if (q >= 3 * m.n) { y[q] = x[3 * lp + (q - 3 * m.n)]; return; }
    const int64_t e = q / m.n, i = q - e * m.n;
    y[q] = x[e * lp + cs_index(m, i)];
}
__global__ void k_from_cs(DevModel m, const double* __restrict__ x, double* __restrict__ y) {
    k_from_cs_d(PF_BLK, m, x, y);
}
struct F_k_from_cs {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_from_cs_d(wg, a...);
    }
};

// Small device-to-host read-backs of a fusion group: a kernel writes the
// member's pinned host buffer.
__device__ __forceinline__ void k_copy_words_d(const Blk& wg, const uint32_t* __restrict__ src,
                                               uint32_t* __restrict__ dst, int n) {
    for (int i = (int)threadIdx.x; i < n; i += (int)blockDim.x) dst[i] = src[i];
}
__global__ __launch_bounds__(64) void k_copy_words(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst,
                                                   int n) {
    k_copy_words_d(PF_BLK, src, dst, n);
}
struct F_k_copy_words {
    static constexpr int kLB = 64;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_copy_words_d(wg, a...);
    }
};

__device__ __forceinline__ void k_axpby_d(const Blk& wg, int64_t n, double a, const double* __restrict__ x, double b,
                                          double* __restrict__ y) {
    for (int64_t i = (int64_t)wg.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)wg.n * blockDim.x)
        y[i] = (b == 0.0) ? a * x[i] : a * x[i] + b * y[i];
}
__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
    k_axpby_d(PF_BLK, n, a, x, b, y);
}
struct F_k_axpby {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_axpby_d(wg, a...);
    }
};

__device__ __forceinline__ void k_copy_d(const Blk& wg, int64_t n, const double* __restrict__ x,
                                         double* __restrict__ y) {
    for (int64_t i = (int64_t)wg.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)wg.n * blockDim.x)
        y[i] = x[i];
}
__global__ void k_copy(int64_t n, const double* __restrict__ x, double* __restrict__ y) {
    k_copy_d(PF_BLK, n, x, y);
}
struct F_k_copy {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_copy_d(wg, a...);
    }
};

__device__ __forceinline__ void k_fill_d(const Blk& wg, int64_t n, double v, double* __restrict__ y) {
    for (int64_t i = (int64_t)wg.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)wg.n * blockDim.x)
        y[i] = v;
}
__global__ void k_fill(int64_t n, double v, double* __restrict__ y) {
    k_fill_d(PF_BLK, n, v, y);
}
struct F_k_fill {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_fill_d(wg, a...);
    }
};

// 3x3 inverse by the adjugate (scale-safe: every term of the determinant
// carries one entry of each column).
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

__device__ __forceinline__ void k_bjac_setup_d(const Blk& wg, int64_t n, const double* __restrict__ J,
                                               double* __restrict__ Dinv) {
    const int64_t i = (int64_t)wg.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double a[9], r[9];
    for (int e = 0; e < 9; ++e) a[e] = J[e * n + i];
    inv3(a, r);
    for (int e = 0; e < 9; ++e) Dinv[e * n + i] = r[e];
}
__global__ void k_bjac_setup(int64_t n, const double* __restrict__ J, double* __restrict__ Dinv) {
    k_bjac_setup_d(PF_BLK, n, J, Dinv);
}
struct F_k_bjac_setup {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_bjac_setup_d(wg, a...);
    }
};

// z = D^{-1} r per cell block; wells z = r / Dw
__device__ __forceinline__ void k_bjac_apply_d(const Blk& wg, int64_t n, int nw, const double* __restrict__ Dinv,
                                               const double* __restrict__ Dw, const double* __restrict__ r,
                                               double* __restrict__ z) {
    const int64_t i = (int64_t)wg.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const double a = r[i], b = r[n + i], c = r[2 * n + i];
        z[i] = Dinv[0 * n + i] * a + Dinv[1 * n + i] * b + Dinv[2 * n + i] * c;
        z[n + i] = Dinv[3 * n + i] * a + Dinv[4 * n + i] * b + Dinv[5 * n + i] * c;
        z[2 * n + i] = Dinv[6 * n + i] * a + Dinv[7 * n + i] * b + Dinv[8 * n + i] * c;
    } else if (i < n + nw) {
        const int w = (int)(i - n);
        z[3 * n + w] = r[3 * n + w] / Dw[w];
    }
}
__global__ void k_bjac_apply(int64_t n, int nw, const double* __restrict__ Dinv, const double* __restrict__ Dw,
                             const double* __restrict__ r, double* __restrict__ z) {
    k_bjac_apply_d(PF_BLK, n, nw, Dinv, Dw, r, z);
}
struct F_k_bjac_apply {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_bjac_apply_d(wg, a...);
    }
};

// ---------------------------------------------------------------------------
// Arnoldi.  Vectors V[k] (k = 0..j) are rows of V with leading dimension ld.
// k_mdot: partial sums of <V[k], w> for k in the block's chunk of 16 and
// (in the last slot, index nk) <w, w>.  part[k*G + block].

// Slots [k0, k0 + KN) of the dot products: slot k < nk is <V[k], w>, slot
// nk is <w, w>.  KN is a compile-time count so all loads of an element are
// issued together.  RT: only the first kn of the KN slots (a count that
// varies between the members of one merged launch; each slot's sum is
// formed as with KN = kn).
template <int KN, bool RT>
__device__ __forceinline__ void k_mdot_d(const Blk& wg, int64_t nv, int nk, int k0, const double* __restrict__ V,
                                         int64_t ld, const double* __restrict__ w, double* __restrict__ part,
                                         const KrylovCtl* __restrict__ kc, int gated, int kn) {
    if (gated && kc->reorth == 0) return;
    __shared__ double lds[KN * 4];
    const double* src[KN];
#pragma unroll
    for (int q = 0; q < KN; ++q) src[q] = (k0 + q < nk) ? V + (int64_t)(k0 + q) * ld : w;
    double acc[KN];
#pragma unroll
    for (int q = 0; q < KN; ++q) acc[q] = 0.0;
    for (int64_t i = (int64_t)wg.x * blockDim.x + threadIdx.x; i < nv; i += (int64_t)wg.n * blockDim.x) {
        const double wi = w[i];
#pragma unroll
        for (int q = 0; q < KN; ++q)
            if (!RT || q < kn) acc[q] += src[q][i] * wi;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < KN; ++q) {
        if (RT && q >= kn) break;
        double a = acc[q];
        for (int o = 32; o > 0; o >>= 1) a += __shfl_down(a, o, 64);
        if (lane == 0) lds[q * 4 + wid] = a;
    }
    __syncthreads();
    if (threadIdx.x < (RT ? kn : KN)) {
        const int q = threadIdx.x;
        const double a = ((lds[q * 4] + lds[q * 4 + 1]) + lds[q * 4 + 2]) + lds[q * 4 + 3];
        part[(int64_t)(k0 + q) * wg.n + wg.x] = a;
    }
}
template <int KN, bool RT>
__global__ __launch_bounds__(256) void k_mdot(int64_t nv, int nk, int k0, const double* __restrict__ V, int64_t ld,
                                              const double* __restrict__ w, double* __restrict__ part,
                                              const KrylovCtl* __restrict__ kc, int gated, int kn) {
    k_mdot_d<KN, RT>(PF_BLK, nv, nk, k0, V, ld, w, part, kc, gated, kn);
}
template <int KN, bool RT>
struct F_k_mdot {
    static constexpr int kLB = 256;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_mdot_d<KN, RT>(wg, a...);
    }
};

__device__ __forceinline__ double block_sum_fixed(double v, double* lds) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        r = lds[0];
        for (int q = 1; q < (int)(blockDim.x >> 6); ++q) r += lds[q];
    }
    return r;
}

// One block per dot product: folds the partials.  mode 0: first CGS pass
// (H(:,j) = h, slot nk holds |w|^2 -> wnorm0); mode 1: second pass (gated;
// H(:,j) += h); mode 2: initial norm of a cycle (slot 0 only -> beta).
__device__ __forceinline__ void k_dot_finish_d(const Blk& wg, int nk, int G, const double* __restrict__ part,
                                               KrylovCtl* __restrict__ kc, int j, int mode, int first) {
    if (mode == 1 && kc->reorth == 0) return;
    __shared__ double lds[16];
    const int k = wg.x;
    double a = 0.0;
    for (int b = threadIdx.x; b < G; b += blockDim.x) a += part[(int64_t)k * G + b];
    const double v = block_sum_fixed(a, lds);
    if (threadIdx.x != 0) return;
    constexpr int ld = kMaxRestart + 1;
    if (mode == 2) {
        const double beta = sqrt(v);
        kc->beta = beta;
        if (first) kc->beta0 = beta;
        for (int q = 0; q <= kMaxRestart; ++q) kc->g[q] = 0.0;
        kc->g[0] = beta;
        kc->inv_h = (beta > 0.0 && beta <= DBL_MAX) ? 1.0 / beta : 0.0;
        kc->rel = (kc->beta0 > 0.0) ? beta / kc->beta0 : 0.0;
        kc->breakdown = !(beta > 0.0 && beta <= DBL_MAX);
        return;
    }
    if (k < nk) {
        kc->h[k] = v;
        if (mode == 0) kc->H[j * ld + k] = v;
        else kc->H[j * ld + k] += v;
    } else if (mode == 0) {
        kc->wnorm0 = sqrt(v);
    }
}
__global__ __launch_bounds__(256) void k_dot_finish(int nk, int G, const double* __restrict__ part,
                                                    KrylovCtl* __restrict__ kc, int j, int mode, int first) {
    k_dot_finish_d(PF_BLK, nk, G, part, kc, j, mode, first);
}
struct F_k_dot_finish {
    static constexpr int kLB = 256;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_dot_finish_d(wg, a...);
    }
};

// A CGS pass leaves w with components along the basis of about eps times
// |w| before the pass, i.e. eps / ratio relative to |w| after it.  The
// second pass is taken when the pass removed more than 90 % of the norm
// (ratio < kReorthEta), so every basis vector is orthogonal to the others
// to within about 10 eps.  (Kahan's bound of 1/sqrt(2) would keep one eps,
// but with a CPR-preconditioned operator the projection removes most of w
// on nearly every iteration, and the second pass then doubled the
// orthogonalisation for no change in the iteration counts.)
constexpr double kReorthEta = 0.1;

// The first pass's update can normalise w at once: with an orthonormal basis
// |w - V h|^2 = |w|^2 - |h|^2, which is accurate to a few eps relative to
// the new norm as long as the pass keeps more than kReorthEta of |w| (the
// case that needs no second pass).  fused_scale returns 1 / that norm, or 0
// where the prediction is not trusted (severe cancellation, or the test
// would call for the second pass); the update and the close compute it from
// the same values in the same order, so they agree.
__device__ __forceinline__ double fused_scale(const KrylovCtl* kc, int nk) {
    double hs = 0.0;
    for (int k = 0; k < nk; ++k) hs += kc->h[k] * kc->h[k];
    const double w0 = kc->wnorm0;
    const double p2 = w0 * w0 - hs;
    const bool ok = p2 > 0.0 && p2 <= DBL_MAX && p2 >= kReorthEta * kReorthEta * (w0 * w0);
    return ok ? 1.0 / sqrt(p2) : 0.0;
}

// w -= sum_k h[k] V[k]; partial sums of the new |w|^2.  KN > 0: exactly KN
// vectors, fully unrolled; KN == 0: runtime count nk.  fuse (first pass):
// the result is also scaled by fused_scale when that is non-zero.
template <int KN>
__device__ __forceinline__ void k_mupdate_d(const Blk& wg, int64_t nv, int nk, const double* __restrict__ V,
                                            int64_t ld, double* __restrict__ w, double* __restrict__ part,
                                            const KrylovCtl* __restrict__ kc, int gated, int fuse) {
    if (gated && kc->reorth == 0) return;
    __shared__ double lds[16];
    double sc = fuse ? fused_scale(kc, nk) : 0.0;
    if (sc == 0.0) sc = 1.0;
    double ss = 0.0;
    if (KN > 0) {
        double h[KN > 0 ? KN : 1];
#pragma unroll
        for (int k = 0; k < KN; ++k) h[k] = kc->h[k];
        for (int64_t i = (int64_t)wg.x * blockDim.x + threadIdx.x; i < nv;
             i += (int64_t)wg.n * blockDim.x) {
            double a = w[i];
#pragma unroll
            for (int k = 0; k < KN; ++k) a -= h[k] * V[(int64_t)k * ld + i];
            a *= sc;
            w[i] = a;
            ss += a * a;
        }
    } else {
        for (int64_t i = (int64_t)wg.x * blockDim.x + threadIdx.x; i < nv;
             i += (int64_t)wg.n * blockDim.x) {
            double a = w[i];
#pragma unroll 8
            for (int k = 0; k < nk; ++k) a -= kc->h[k] * V[(int64_t)k * ld + i];
            a *= sc;
            w[i] = a;
            ss += a * a;
        }
    }
    const double v = block_sum_fixed(ss, lds);
    if (threadIdx.x == 0) part[wg.x] = v;
}
template <int KN>
__global__ __launch_bounds__(256) void k_mupdate(int64_t nv, int nk, const double* __restrict__ V, int64_t ld,
                                                 double* __restrict__ w, double* __restrict__ part,
                                                 const KrylovCtl* __restrict__ kc, int gated, int fuse) {
    k_mupdate_d<KN>(PF_BLK, nv, nk, V, ld, w, part, kc, gated, fuse);
}
template <int KN>
struct F_k_mupdate {
    static constexpr int kLB = 256;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_mupdate_d<KN>(wg, a...);
    }
};

// Norm of w after a CGS pass; then either request re-orthogonalisation
// (stage 0) or finish column j: Givens rotations and residual estimate.
// fuse: the first pass's update may have normalised w (fused_scale); then
// h(j+1, j) is the predicted norm and w needs no further scaling unless its
// measured norm strays from 1.
__device__ __forceinline__ void k_arnoldi_close_d(const Blk& wg, int G, const double* __restrict__ part,
                                                  KrylovCtl* __restrict__ kc, int j, int stage, int always_reorth,
                                                  int fuse) {
    if (stage == 1 && kc->reorth == 0) return;
    __shared__ double lds[16];
    double a = 0.0;
    for (int b = threadIdx.x; b < G; b += blockDim.x) a += part[b];
    const double ss = block_sum_fixed(a, lds);
    if (threadIdx.x != 0) return;
    const double wm = sqrt(ss);          // norm of w as stored
    double wn = wm;                      // h(j+1, j)
    kc->normalised = 0;
    if (stage == 0) {
        const double sc = fuse ? fused_scale(kc, j + 1) : 0.0;
        if (sc > 0.0) {
            // w holds (w - V h) * sc: no second pass by construction
            kc->reorth = 0;
            if (fabs(wm - 1.0) <= 1e-10) {
                wn = 1.0 / sc;
                kc->normalised = 1;
            } else {
                wn = wm / sc;
            }
        } else {
            // a large cancellation calls for a second pass
            const int again = always_reorth || !(wm > kReorthEta * kc->wnorm0);
            kc->reorth = again;
            if (again) {
                kc->wnorm = wm;
                return;
            }
        }
    }
    kc->wnorm = wn;
    constexpr int ld = kMaxRestart + 1;
    double* col = kc->H + j * ld;
    col[j + 1] = wn;
    for (int i = 0; i < j; ++i) {
        const double t0 = kc->cs[i] * col[i] + kc->sn[i] * col[i + 1];
        const double t1 = -kc->sn[i] * col[i] + kc->cs[i] * col[i + 1];
        col[i] = t0;
        col[i + 1] = t1;
    }
    const double hj = col[j], hj1 = col[j + 1];
    const double r = hypot(hj, hj1);
    const double c = (r > 0.0) ? hj / r : 1.0;
    const double s = (r > 0.0) ? hj1 / r : 0.0;
    kc->cs[j] = c;
    kc->sn[j] = s;
    col[j] = r;
    col[j + 1] = 0.0;
    const double gj = kc->g[j];
    kc->g[j] = c * gj;
    kc->g[j + 1] = -s * gj;
    kc->rel = (kc->beta0 > 0.0) ? fabs(kc->g[j + 1]) / kc->beta0 : 0.0;
    const bool ok = wn > 1e-300 && wn <= DBL_MAX && r > 0.0 && r <= DBL_MAX && wm > 0.0 && wm <= DBL_MAX;
    // scale that turns the stored w into V[j+1] (1 when already normalised)
    kc->inv_h = ok ? (kc->normalised ? 1.0 : 1.0 / wm) : 0.0;
    kc->breakdown = !ok;
}
__global__ __launch_bounds__(256) void k_arnoldi_close(int G, const double* __restrict__ part,
                                                       KrylovCtl* __restrict__ kc, int j, int stage,
                                                       int always_reorth, int fuse) {
    k_arnoldi_close_d(PF_BLK, G, part, kc, j, stage, always_reorth, fuse);
}
struct F_k_arnoldi_close {
    static constexpr int kLB = 256;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_arnoldi_close_d(wg, a...);
    }
};

// out = v * kc->inv_h  (in place allowed)
__device__ __forceinline__ void k_scale_ctl_d(const Blk& wg, int64_t n, const double* __restrict__ v,
                                              double* __restrict__ out, const KrylovCtl* __restrict__ kc) {
    const double s = kc->inv_h;
    for (int64_t i = (int64_t)wg.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)wg.n * blockDim.x)
        out[i] = v[i] * s;
}
__global__ void k_scale_ctl(int64_t n, const double* __restrict__ v, double* __restrict__ out,
                            const KrylovCtl* __restrict__ kc) {
    k_scale_ctl_d(PF_BLK, n, v, out, kc);
}
struct F_k_scale_ctl {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_scale_ctl_d(wg, a...);
    }
};

// y = R^{-1} g for the k x k upper triangle left by the rotations.
__device__ __forceinline__ void k_solve_small_d(const Blk& wg, KrylovCtl* kc, int k) {
    if (threadIdx.x != 0 || wg.x != 0) return;
    constexpr int ld = kMaxRestart + 1;
    for (int i = k - 1; i >= 0; --i) {
        double s = kc->g[i];
        for (int q = i + 1; q < k; ++q) s -= kc->H[q * ld + i] * kc->y[q];
        const double d = kc->H[i * ld + i];
        kc->y[i] = (d != 0.0) ? s / d : 0.0;
    }
}
__global__ void k_solve_small(KrylovCtl* kc, int k) {
    k_solve_small_d(PF_BLK, kc, k);
}
struct F_k_solve_small {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_solve_small_d(wg, a...);
    }
};

// dx += sum_i y[i] Z[i]
template <class TZ>
// dx += Z y; first: dx = Z y, the sum starting from 0 as from a zeroed dx
__device__ __forceinline__ void k_zcomb_d(const Blk& wg, int64_t nv, int k, const TZ* __restrict__ Z, int64_t ld,
                                          const KrylovCtl* __restrict__ kc, double* __restrict__ dx, int first) {
    for (int64_t i = (int64_t)wg.x * blockDim.x + threadIdx.x; i < nv; i += (int64_t)wg.n * blockDim.x) {
        double a = first ? 0.0 : dx[i];
        for (int q = 0; q < k; ++q) a += kc->y[q] * (double)Z[(int64_t)q * ld + i];
        dx[i] = a;
    }
}
template <class TZ>
__global__ void k_zcomb(int64_t nv, int k, const TZ* __restrict__ Z, int64_t ld, const KrylovCtl* __restrict__ kc,
                        double* __restrict__ dx, int first) {
    k_zcomb_d<TZ>(PF_BLK, nv, k, Z, ld, kc, dx, first);
}
template <class TZ>
struct F_k_zcomb {
    static constexpr int kLB = 1024;
    template <class... A>
    __device__ __forceinline__ void operator()(const Blk& wg, const A&... a) const {
        k_zcomb_d<TZ>(wg, a...);
    }
};

unsigned stream_grid(int64_t n) {
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > 8192) g = 8192;
    return (unsigned)(g > 0 ? g : 1);
}

}  // namespace

namespace {
template <class TX>
void spmv_border_t(Sim& s, const TX* x, double* y, int cs = 0) {
    const DevModel& m = s.m;
    const int ncb = (int)((m.npc + 63) / 64);
    if (ncb + m.nw > 0) {
        launch<F_k_spmv_border<TX>>(s, s.stream, k_spmv_border<TX>, dim3(ncb + m.nw), dim3(64), 0, m, ncb, s.pc_cell,
                                    s.pc_first, s.perf_well, s.perf_cell, s.wp_first, s.wp_idx, s.B, s.Cw, s.Dw, x, y,
                                    cs);
        PF_LAUNCH_CHECK();
    }
}
template <class TX>
void spmv_t(Sim& s, const TX* x, double* y) {
    const DevModel& m = s.m;
    ensure_j_natural(s);
    {
        ProfScope ps(s, PF_K_SPMV);
        launch<F_k_spmv<TX>>(s, s.stream, k_spmv<TX>, dim3(grid_for(m.n)), dim3(kBlock), 0, m, s.J, x, y);
        PF_LAUNCH_CHECK();
    }
    spmv_border_t<TX>(s, x, y);
}
}  // namespace

void launch_spmv_border(Sim& s, const double* x, double* y, int cs) { spmv_border_t<double>(s, x, y, cs); }

void launch_to_cs(Sim& s, const double* x, double* y, double scale) {
    launch<F_k_to_cs>(s, s.stream, k_to_cs, dim3(grid_for(s.nvc)), dim3(kBlock), 0, s.m, x, y, scale);
    PF_LAUNCH_CHECK();
}

void launch_from_cs(Sim& s, const double* x, double* y) {
    launch<F_k_from_cs>(s, s.stream, k_from_cs, dim3(grid_for(s.nv)), dim3(kBlock), 0, s.m, x, y);
    PF_LAUNCH_CHECK();
}
void launch_spmv(Sim& s, const double* x, double* y) { spmv_t<double>(s, x, y); }
void launch_spmv(Sim& s, const float* x, double* y) { spmv_t<float>(s, x, y); }

void launch_axpby(Sim& s, int64_t n, double a, const double* x, double b, double* y) {
    launch<F_k_axpby>(s, s.stream, k_axpby, dim3(stream_grid(n)), dim3(kBlock), 0, n, a, x, b, y);
    PF_LAUNCH_CHECK();
}

void launch_copy(Sim& s, int64_t n, const double* x, double* y) {
    launch<F_k_copy>(s, s.stream, k_copy, dim3(stream_grid(n)), dim3(kBlock), 0, n, x, y);
    PF_LAUNCH_CHECK();
}

void launch_copy_words(Sim& s, const void* src, void* dst, size_t bytes) {
    launch<F_k_copy_words>(s, s.stream, k_copy_words, dim3(1), dim3(64), 0, (const uint32_t*)src, (uint32_t*)dst,
                           (int)(bytes / 4));
}

void launch_fill(Sim& s, int64_t n, double v, double* y) {
    launch<F_k_fill>(s, s.stream, k_fill, dim3(stream_grid(n)), dim3(kBlock), 0, n, v, y);
    PF_LAUNCH_CHECK();
}

void launch_bjac_setup(Sim& s) {
    launch<F_k_bjac_setup>(s, s.stream, k_bjac_setup, dim3(grid_for(s.m.n)), dim3(kBlock), 0, s.m.n, s.J, s.Dinv);
    PF_LAUNCH_CHECK();
}

void launch_bjac_apply(Sim& s, const double* r, double* z) {
    launch<F_k_bjac_apply>(s, s.stream, k_bjac_apply, dim3(grid_for(s.m.n + s.m.nw)), dim3(kBlock), 0, s.m.n, s.m.nw,
                           s.Dinv, s.Dw, r, z);
    PF_LAUNCH_CHECK();
}

void launch_norm_to_ctl(Sim& s, const double* v, int first) {
    const int G = kRedBlocks;
    launch<F_k_mdot<1, false>>(s, s.stream, k_mdot<1, false>, dim3(G), dim3(kBlock), 0, s.nk, 0, 0,
                               (const double*)nullptr, (int64_t)0, v, s.part, s.kc, 0, 1);
    PF_LAUNCH_CHECK();
    launch<F_k_dot_finish>(s, s.stream, k_dot_finish, dim3(1), dim3(kBlock), 0, 0, G, s.part, s.kc, 0, 2, first);
    PF_LAUNCH_CHECK();
}

void launch_scale_by_ctl(Sim& s, const double* v, double* out, int /*which*/) {
    launch<F_k_scale_ctl>(s, s.stream, k_scale_ctl, dim3(stream_grid(s.nk)), dim3(kBlock), 0, s.nk, v, out, s.kc);
    PF_LAUNCH_CHECK();
}

namespace {

template <int KN>
void mdot_launch(Sim& s, int nk, int k0, const double* w, int gated) {
    launch<F_k_mdot<KN, false>>(s, s.stream, k_mdot<KN, false>, dim3(kRedBlocks), dim3(kBlock), 0, s.nk, nk, k0,
                                s.V, s.kst, w, s.part, s.kc, gated, KN);
    PF_LAUNCH_CHECK();
}

// dot products of slots [0, nslots): slot k < nk is <V[k], w>, slot nk is <w, w>
void mdot_all(Sim& s, int nk, int nslots, const double* w, int gated) {
    for (int k0 = 0; k0 < nslots; k0 += kDotChunk) {
        const int kn = std::min(kDotChunk, nslots - k0);
        if (s.fu) {
            // in a fusion group one kernel for every chunk size, so that
            // members at different iterations share launches
            launch<F_k_mdot<kDotChunk, true>>(s, s.stream, k_mdot<kDotChunk, true>, dim3(kRedBlocks), dim3(kBlock),
                                              0, s.nk, nk, k0, s.V, s.kst, w, s.part, s.kc, gated, kn);
            continue;
        }
        switch (kn) {
#define PF_CASE(K) case K: mdot_launch<K>(s, nk, k0, w, gated); break;
            PF_CASE(1) PF_CASE(2) PF_CASE(3) PF_CASE(4) PF_CASE(5) PF_CASE(6) PF_CASE(7) PF_CASE(8)
            PF_CASE(9) PF_CASE(10) PF_CASE(11) PF_CASE(12) PF_CASE(13) PF_CASE(14) PF_CASE(15) PF_CASE(16)
#undef PF_CASE
        }
    }
}

template <int KN>
void mupdate_launch(Sim& s, int nk, double* w, int gated, int fuse) {
    launch<F_k_mupdate<KN>>(s, s.stream, k_mupdate<KN>, dim3(kRedBlocks), dim3(kBlock), 0, s.nk, nk, s.V, s.kst, w,
                            s.part, s.kc, gated, fuse);
    PF_LAUNCH_CHECK();
}

void mupdate_any(Sim& s, int nk, double* w, int gated, int fuse) {
    // in a fusion group the kernel with a run-time vector count (the same
    // sums in the same order), shared by members at different iterations
    switch (s.fu ? 0 : nk) {
#define PF_CASE(K) case K: mupdate_launch<K>(s, nk, w, gated, fuse); return;
        PF_CASE(1) PF_CASE(2) PF_CASE(3) PF_CASE(4) PF_CASE(5) PF_CASE(6) PF_CASE(7) PF_CASE(8)
        PF_CASE(9) PF_CASE(10) PF_CASE(11) PF_CASE(12) PF_CASE(13) PF_CASE(14) PF_CASE(15) PF_CASE(16)
        PF_CASE(17) PF_CASE(18) PF_CASE(19) PF_CASE(20) PF_CASE(21) PF_CASE(22) PF_CASE(23) PF_CASE(24)
        PF_CASE(25) PF_CASE(26) PF_CASE(27) PF_CASE(28) PF_CASE(29) PF_CASE(30) PF_CASE(31) PF_CASE(32)
#undef PF_CASE
        default: mupdate_launch<0>(s, nk, w, gated, fuse);
    }
}

}  // namespace

// Column j of the Arnoldi process in CGS passes.  launch_arnoldi: the first
// pass (dot products, update, norm and the second-pass test; with reorth = 1
// the second pass follows at once).  The host reads the test with the
// residual estimate and calls launch_arnoldi_second only when the device
// asked for it, so the usual iteration launches no second-pass kernels;
// where the first pass's update did not already normalise w (kc->normalised),
// launch_normalise then scales w into V[j+1].
void launch_arnoldi(Sim& s, int j, double* w) {
    const int G = kRedBlocks;
    const int nk = j + 1;
    const int always = s.opts.reorth ? 1 : 0;
    // pass 1: <V[k], w> for k <= j and <w, w>
    {
        ProfScope ps(s, PF_K_MDOT);
        mdot_all(s, nk, nk + 1, w, 0);
    }
    launch<F_k_dot_finish>(s, s.stream, k_dot_finish, dim3(nk + 1), dim3(kBlock), 0, nk, G, s.part, s.kc, j, 0, 0);
    PF_LAUNCH_CHECK();
    {
        ProfScope ps(s, PF_K_MUPDATE);
        mupdate_any(s, nk, w, 0, !always);
    }
    launch<F_k_arnoldi_close>(s, s.stream, k_arnoldi_close, dim3(1), dim3(kBlock), 0, G, s.part, s.kc, j, 0, always,
                              !always);
    PF_LAUNCH_CHECK();
    if (always) launch_arnoldi_second(s, j, w);
}

// The second CGS pass (its kernels return at once unless the first pass's
// test asked for it).
void launch_arnoldi_second(Sim& s, int j, double* w) {
    const int G = kRedBlocks;
    const int nk = j + 1;
    const int always = s.opts.reorth ? 1 : 0;
    mdot_all(s, nk, nk, w, 1);
    launch<F_k_dot_finish>(s, s.stream, k_dot_finish, dim3(nk), dim3(kBlock), 0, nk, G, s.part, s.kc, j, 1, 0);
    PF_LAUNCH_CHECK();
    mupdate_any(s, nk, w, 1, 0);
    launch<F_k_arnoldi_close>(s, s.stream, k_arnoldi_close, dim3(1), dim3(kBlock), 0, G, s.part, s.kc, j, 1, always,
                              0);
    PF_LAUNCH_CHECK();
}

void launch_normalise(Sim& s, double* w) {
    launch<F_k_scale_ctl>(s, s.stream, k_scale_ctl, dim3(stream_grid(s.nk)), dim3(kBlock), 0, s.nk, w, w, s.kc);
    PF_LAUNCH_CHECK();
}

void launch_solve_small(Sim& s, int k) {
    launch<F_k_solve_small>(s, s.stream, k_solve_small, dim3(1), dim3(64), 0, s.kc, k);
    PF_LAUNCH_CHECK();
}

void launch_zcomb(Sim& s, int k, double* dx, bool first) {
    if (s.opts.precision == PF_PREC_MIXED)
        launch<F_k_zcomb<float>>(s, s.stream, k_zcomb<float>, dim3(stream_grid(s.nk)), dim3(kBlock), 0, s.nk, k,
                                 s.Z32, s.kst, s.kc, dx, (int)first);
    else
        launch<F_k_zcomb<double>>(s, s.stream, k_zcomb<double>, dim3(stream_grid(s.nk)), dim3(kBlock), 0, s.nk, k,
                                  s.Z, s.kst, s.kc, dx, (int)first);
    PF_LAUNCH_CHECK();
}

}  // namespace pf
