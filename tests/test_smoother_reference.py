"""The numpy red-black block ILU(0) of tests/precond_ref.py checked on the
CPU against what ILU(0) must satisfy: the preconditioner M it applies
equals the operator A on every red row and column block and on the black
diagonal blocks, and differs from A only by the dropped fill between
distinct black cells (the off-diagonal part of A_br D_r^{-1} A_rb)."""
import numpy as np
import pytest

from precond_ref import bjac_apply, blocks, grid_index, ilu_apply, neighbours


def _random_planes(dims, seed):
    nx, ny, nz = dims
    n = nx * ny * nz
    rng = np.random.default_rng(seed)
    nb = neighbours(dims)
    J = np.zeros((7, 3, 3, n))
    for d in range(1, 7):
        J[d] = rng.uniform(-1.0, 0.2, (3, 3, n)) * (nb[d] >= 0)
    J[0] = rng.uniform(-0.5, 0.5, (3, 3, n))
    for e in range(3):
        J[0, e, e] = 8.0 + rng.uniform(0, 1, n)
    return J.reshape(-1)


def _dense(B, dims):
    n = B.shape[1]
    nb = neighbours(dims)
    A = np.zeros((3 * n, 3 * n))
    rows = np.arange(n)
    for r in range(3):
        for c in range(3):
            A[r * n + rows, c * n + rows] = B[0][:, r, c]
            for d in range(1, 7):
                m = nb[d] >= 0
                A[r * n + rows[m], c * n + nb[d][m]] = B[d][m, r, c]
    return A


@pytest.mark.parametrize("dims", [(4, 3, 2), (3, 3, 3), (5, 1, 1)])
def test_ilu_reference_reproduces_the_operator_off_the_dropped_fill(dims):
    n = int(np.prod(dims))
    B = blocks(_random_planes(dims, 7), n)
    A = _dense(B, dims)
    Minv = np.column_stack([ilu_apply(B, dims, e) for e in np.eye(3 * n)])
    M = np.linalg.inv(Minv)
    ix, iy, iz = grid_index(dims)
    red = np.tile((ix + iy + iz) % 2 == 0, 3)
    blk = ~red
    assert np.allclose(M[np.ix_(red, red)], A[np.ix_(red, red)], atol=1e-10)
    assert np.allclose(M[np.ix_(red, blk)], A[np.ix_(red, blk)], atol=1e-10)
    assert np.allclose(M[np.ix_(blk, red)], A[np.ix_(blk, red)], atol=1e-10)
    # black-black: A_bb (block diagonal) + off-diagonal part of A_br A_rr^{-1} A_rb
    S = A[np.ix_(blk, red)] @ np.linalg.solve(A[np.ix_(red, red)], A[np.ix_(red, blk)])
    cell = np.tile(np.arange(n), 3)[blk]
    same = cell[:, None] == cell[None, :]
    expect = A[np.ix_(blk, blk)] + np.where(same, 0.0, S)
    assert np.allclose(M[np.ix_(blk, blk)], expect, atol=1e-10)


def test_ilu_reference_is_exact_without_fill():
    # two cells: the red cell has one black neighbour, nothing is dropped
    dims = (2, 1, 1)
    B = blocks(_random_planes(dims, 3), 2)
    A = _dense(B, dims)
    f = np.random.default_rng(1).standard_normal(6)
    assert np.allclose(ilu_apply(B, dims, f), np.linalg.solve(A, f), rtol=1e-12, atol=1e-14)


def test_block_jacobi_reference():
    dims = (3, 2, 2)
    n = 12
    B = blocks(_random_planes(dims, 5), n)
    A = _dense(B, dims)
    f = np.random.default_rng(2).standard_normal(3 * n)
    D = np.zeros_like(A)
    for k in range(n):
        idx = [k, n + k, 2 * n + k]
        D[np.ix_(idx, idx)] = A[np.ix_(idx, idx)]
    assert np.allclose(bjac_apply(B, f), np.linalg.solve(D, f), rtol=1e-12)


@pytest.mark.parametrize("dims", [(4, 3, 2), (5, 4, 3), (7, 1, 2)])
def test_red_rows_of_the_two_stage_product_are_the_right_hand_side(dims):
    """z = x_p + M^{-1} (v - A x_p), with x_p a pressure-only correction as the
    CPR first stage gives it: M and A share their red rows, so (A z)_r =
    (A x_p)_r + (v - A x_p)_r = v_r, up to rounding.  The FP64 product kernel
    stores v_r as the red rows of w = A z on this identity.  The black rows
    differ from v by the dropped fill, so the check is not vacuous."""
    n = int(np.prod(dims))
    B = blocks(_random_planes(dims, 11), n)
    A = _dense(B, dims)
    rng = np.random.default_rng(3)
    v = rng.standard_normal(3 * n)
    xp = np.zeros(3 * n)
    xp[:n] = rng.standard_normal(n)
    z = xp + ilu_apply(B, dims, v - A @ xp)
    w = A @ z
    ix, iy, iz = grid_index(dims)
    red = np.tile((ix + iy + iz) % 2 == 0, 3)
    scale = np.abs(A) @ np.abs(z) + np.abs(v)
    assert np.all(np.abs(w[red] - v[red]) <= 1e-13 * scale[red])
    assert np.max(np.abs(w[~red] - v[~red])) > 1e-6 * np.max(np.abs(v))
