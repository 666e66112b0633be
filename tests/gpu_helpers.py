"""Helpers shared by the GPU parity tests: layout conversion between the
library's plane layout / stencil Jacobian and the oracle's block-wise CSR.
Test code only; neither the oracle nor the library imports it."""
import numpy as np
import scipy.sparse as sp


def planes_to_block(v, n, nw):
    out = np.empty(3 * n + nw)
    out[0:3 * n:3] = v[0:n]
    out[1:3 * n:3] = v[n:2 * n]
    out[2:3 * n:3] = v[2 * n:3 * n]
    out[3 * n:] = v[3 * n:]
    return out


def block_to_planes(v, n, nw):
    out = np.empty(3 * n + nw)
    out[0:n] = v[0:3 * n:3]
    out[n:2 * n] = v[1:3 * n:3]
    out[2 * n:3 * n] = v[2:3 * n:3]
    out[3 * n:] = v[3 * n:]
    return out


def stencil_to_csr(case, J, border, perf_well, perf_cell):
    """Library Jacobian (63 planes + per-perforation border) -> CSR in the
    oracle's block-wise ordering."""
    nx, ny, nz = case.nx, case.ny, case.nz
    n = nx * ny * nz
    nw = len(case.wells)
    Jp = J.reshape(7, 9, n)
    i = np.arange(n)
    iz, rem = np.divmod(i, nx * ny)
    iy, ix = np.divmod(rem, nx)
    nb = [i, i - 1, i + 1, i - nx, i + nx, i - nx * ny, i + nx * ny]
    ok = [np.ones(n, bool), ix > 0, ix + 1 < nx, iy > 0, iy + 1 < ny, iz > 0, iz + 1 < nz]
    rows, cols, vals = [], [], []
    for d in range(7):
        for e in range(9):
            r, c = divmod(e, 3)
            m = ok[d]
            rows.append(3 * i[m] + r)
            cols.append(3 * nb[d][m] + c)
            vals.append(Jp[d, e][m])
    if border is not None and len(perf_well):
        for k, (w, cell) in enumerate(zip(perf_well, perf_cell)):
            for e in range(3):
                rows.append(np.array([3 * cell + e])); cols.append(np.array([3 * n + w]))
                vals.append(np.array([border[k, e]]))
                rows.append(np.array([3 * n + w])); cols.append(np.array([3 * cell + e]))
                vals.append(np.array([border[k, 3 + e]]))
        for w in range(nw):
            k = int(np.where(perf_well == w)[0][0])
            rows.append(np.array([3 * n + w])); cols.append(np.array([3 * n + w]))
            vals.append(np.array([border[k, 6]]))
    rows = np.concatenate(rows); cols = np.concatenate(cols); vals = np.concatenate(vals)
    return sp.coo_matrix((vals, (rows, cols)), shape=(3 * n + nw, 3 * n + nw)).tocsr()


def field_rel_err(a, b, floor):
    """max |a - b| / max(||b||_inf, floor)"""
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))) if b.size else 0.0, floor))
