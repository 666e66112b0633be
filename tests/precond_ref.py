"""Plain numpy definitions of the CPR second-stage smoothers (Sec. 3.4), the
reference for the library's smoother kernels: block Jacobi, and red-black
block ILU(0) on the 7-point block stencil.

In red-black order (colour (ix + iy + iz) mod 2, red = 0) the red-red and
black-black parts of the 7-point operator are block diagonal, so ILU(0)
keeps the red diagonal blocks D_r and modifies the black ones,
    D~_b = D_b - sum_{r neighbour of b} J_br D_r^{-1} J_rb,
dropping the fill between distinct black cells.  Its application is
    y_r = D_r^{-1} f_r,  y_b = D~_b^{-1} (f_b - sum J_br y_r),
    z_b = y_b,           z_r = y_r - D_r^{-1} sum J_rb z_b.
Well rows are divided by their diagonal."""
import numpy as np

# plane d of the Jacobian couples a cell to its neighbour in direction d
OPP = {1: 2, 2: 1, 3: 4, 4: 3, 5: 6, 6: 5}


def grid_index(dims):
    nx, ny, nz = dims
    i = np.arange(nx * ny * nz)
    iz, rem = np.divmod(i, nx * ny)
    iy, ix = np.divmod(rem, nx)
    return ix, iy, iz


def neighbours(dims):
    """nb[d] (d = 1..6: -x, +x, -y, +y, -z, +z): neighbour index or -1."""
    nx, ny, nz = dims
    ix, iy, iz = grid_index(dims)
    i = np.arange(nx * ny * nz)
    nb = {1: np.where(ix > 0, i - 1, -1), 2: np.where(ix + 1 < nx, i + 1, -1),
          3: np.where(iy > 0, i - nx, -1), 4: np.where(iy + 1 < ny, i + nx, -1),
          5: np.where(iz > 0, i - nx * ny, -1), 6: np.where(iz + 1 < nz, i + nx * ny, -1)}
    return nb


def blocks(J, n):
    """(7, n, 3, 3) blocks from the 63 planes J[(d*9 + e)*n + i], e = 3 row + col."""
    return np.asarray(J, dtype=np.float64).reshape(7, 3, 3, n).transpose(0, 3, 1, 2).copy()


def ilu_factor(B, dims):
    """(Dinv, Dt_inv): inverse red diagonal blocks (black entries unused) and
    inverse modified black diagonal blocks (red entries unused)."""
    n = B.shape[1]
    ix, iy, iz = grid_index(dims)
    red = (ix + iy + iz) % 2 == 0
    nb = neighbours(dims)
    Dinv = np.linalg.inv(B[0])
    Dt = B[0].copy()
    for d in range(1, 7):
        j = nb[d]
        m = (~red) & (j >= 0)
        b, r = np.nonzero(m)[0], j[m]
        # J_br D_r^{-1} J_rb, with J_rb the block of r towards b
        Dt[b] -= B[d][b] @ Dinv[r] @ B[OPP[d]][r]
    return Dinv, np.linalg.inv(Dt), red, nb


def ilu_apply(B, dims, f, Dw=None):
    """z = M^{-1} f for the red-black block ILU(0); f = (3n [+ wells]) planes."""
    n = B.shape[1]
    Dinv, Dtinv, red, nb = ilu_factor(B, dims)
    fc = np.asarray(f[:3 * n], dtype=np.float64).reshape(3, n).T      # (n, 3)
    y = np.zeros((n, 3))
    y[red] = np.einsum("nij,nj->ni", Dinv[red], fc[red])
    g = fc.copy()
    for d in range(1, 7):
        j = nb[d]
        m = (~red) & (j >= 0)
        g[m] -= np.einsum("nij,nj->ni", B[d][m], y[j[m]])
    blk = ~red
    y[blk] = np.einsum("nij,nj->ni", Dtinv[blk], g[blk])
    h = np.zeros((n, 3))
    for d in range(1, 7):
        j = nb[d]
        m = red & (j >= 0)
        h[m] += np.einsum("nij,nj->ni", B[d][m], y[j[m]])
    z = y.copy()
    z[red] = y[red] - np.einsum("nij,nj->ni", Dinv[red], h[red])
    out = z.T.reshape(-1)
    if Dw is not None and len(f) > 3 * n:
        out = np.concatenate([out, np.asarray(f[3 * n:]) / Dw])
    return out


def bjac_apply(B, f, Dw=None):
    n = B.shape[1]
    fc = np.asarray(f[:3 * n], dtype=np.float64).reshape(3, n).T
    out = np.einsum("nij,nj->ni", np.linalg.inv(B[0]), fc).T.reshape(-1)
    if Dw is not None and len(f) > 3 * n:
        out = np.concatenate([out, np.asarray(f[3 * n:]) / Dw])
    return out


def bf16_round(x):
    """FP64 -> FP32 -> BF16 (round to nearest even) -> FP32, as stored by the
    mixed-precision smoother."""
    f = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (f >> 16) & 1
    r = ((f + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def ilu_apply_mixed(B, dims, f, Dw=None):
    """The mixed-precision form: BF16 off-diagonal blocks, FP32 inverse
    diagonal blocks (factored in FP64), FP32 vectors and arithmetic."""
    n = B.shape[1]
    Dinv, Dtinv, red, nb = ilu_factor(B, dims)
    Dinv32 = np.where(red[:, None, None], Dinv, Dtinv).astype(np.float32)
    L = {d: bf16_round(B[d]).reshape(B[d].shape) for d in range(1, 7)}
    fc = np.asarray(f[:3 * n], dtype=np.float64).astype(np.float32).reshape(3, n).T
    y = np.zeros((n, 3), np.float32)
    y[red] = np.einsum("nij,nj->ni", Dinv32[red], fc[red])
    g = fc.copy()
    for d in range(1, 7):
        j = nb[d]
        m = (~red) & (j >= 0)
        g[m] -= np.einsum("nij,nj->ni", L[d][m], y[j[m]])
    blk = ~red
    y[blk] = np.einsum("nij,nj->ni", Dinv32[blk], g[blk])
    h = np.zeros((n, 3), np.float32)
    for d in range(1, 7):
        j = nb[d]
        m = red & (j >= 0)
        h[m] += np.einsum("nij,nj->ni", L[d][m], y[j[m]])
    z = y.copy()
    z[red] = y[red] - np.einsum("nij,nj->ni", Dinv32[red], h[red])
    out = z.T.reshape(-1).astype(np.float64)
    if Dw is not None and len(f) > 3 * n:
        out = np.concatenate([out, np.asarray(f[3 * n:]) / Dw])
    return out
