"""The numpy multigrid used as the reference of the GPU pressure multigrid
(tests/test_gpu_mg.py) checked on the CPU against what it must satisfy:
a z-line half-sweep solves the rows of its colour exactly, and repeated
V-cycles on an M-matrix converge to the direct solution."""
import numpy as np
import pytest

from test_gpu_mg import _agg, _op, _vcycles_ref, _zline_ref


def _mmatrix(dims, seed):
    """7-point M-matrix planes (diag, -x, +x, -y, +y, -z, +z) with random
    symmetric couplings and a small diagonal excess."""
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    tx = rng.uniform(0.1, 2.0, (nz, ny, nx + 1))
    ty = rng.uniform(0.1, 2.0, (nz, ny + 1, nx))
    tz = rng.uniform(0.1, 20.0, (nz + 1, ny, nx))
    tx[:, :, 0] = tx[:, :, -1] = 0
    ty[:, 0, :] = ty[:, -1, :] = 0
    tz[0] = tz[-1] = 0
    A = np.zeros((7, nz, ny, nx))
    A[1], A[2] = -tx[:, :, :-1], -tx[:, :, 1:]
    A[3], A[4] = -ty[:, :-1, :], -ty[:, 1:, :]
    A[5], A[6] = -tz[:-1], -tz[1:]
    A[0] = -A[1:].sum(axis=0) + rng.uniform(1e-3, 1e-2, (nz, ny, nx))
    return A.reshape(7, -1)


def _hierarchy(dims, seed):
    levels = [(dims, _mmatrix(dims, seed))]
    while np.prod(levels[-1][0]) > 40:
        fd, Af = levels[-1]
        cd = tuple((d + 1) // 2 if d > 1 else 1 for d in fd)
        P = _agg(fd, cd)
        G = (P.T @ _op(fd, Af) @ P).tocoo()
        nxc, nyc, nzc = cd
        Ac = np.zeros((7, int(np.prod(cd))))
        offs = {0: 0, -1: 1, 1: 2, -nxc: 3, nxc: 4, -nxc * nyc: 5, nxc * nyc: 6}
        for r, c, v in zip(G.row, G.col, G.data):
            Ac[offs[c - r], r] += v
        levels.append((cd, Ac))
    return levels


@pytest.mark.parametrize("dims", [(6, 5, 4), (7, 3, 9)])
def test_zline_reference_solves_its_rows(dims):
    _, Ap = _hierarchy(dims, 1)[0]
    A = _op(dims, Ap)
    nx, ny, nz = dims
    rng = np.random.default_rng(2)
    b, x0 = rng.standard_normal((2, nx * ny * nz))
    i = np.arange(nx * ny * nz)
    colour_of = (i % nx + (i // nx) % ny) % 2
    for colour in (0, 1):
        x1 = _zline_ref(Ap, dims, x0, b, colour)
        act = colour_of == colour
        assert np.array_equal(x1[~act], x0[~act])
        assert np.max(np.abs((b - A @ x1)[act])) <= 1e-12 * np.max(np.abs(b))


@pytest.mark.parametrize("post", [0, 1])
def test_vcycle_reference_converges_to_the_direct_solution(post):
    dims = (12, 10, 6)
    levels = _hierarchy(dims, 4)
    assert len(levels) >= 3
    A = _op(dims, levels[0][1])
    rng = np.random.default_rng(5)
    b = rng.standard_normal(int(np.prod(dims)))
    exact = np.linalg.solve(A.toarray(), b)
    # one application of 60 cycles is the 60th iterate of the stationary method
    x = _vcycles_ref(levels, b, 60, 2, post)
    assert np.max(np.abs(x - exact)) <= 1e-11 * np.max(np.abs(exact))
    # and a single cycle already reduces the error
    x1 = _vcycles_ref(levels, b, 1, 2, post)
    assert np.max(np.abs(x1 - exact)) < 0.5 * np.max(np.abs(exact))


@pytest.mark.parametrize("dims", [(6, 5, 4), (7, 3, 9), (1, 4, 6)])
def test_one_sweep_from_zero_leaves_the_lateral_residual(dims):
    """One z-line sweep from x = 0 (colour 0, then colour 1): the colour-1
    rows' residual is zero, and the colour-0 rows' is minus their lateral
    couplings times the new colour-1 values (their own columns were solved
    with zero lateral neighbours), the form the restriction after such a
    sweep uses."""
    _, Ap = _hierarchy(dims, 3)[0]
    A = _op(dims, Ap)
    nx, ny, nz = dims
    n = nx * ny * nz
    b = np.random.default_rng(4).standard_normal(n)
    x = _zline_ref(Ap, dims, np.zeros(n), b, 0)
    x = _zline_ref(Ap, dims, x, b, 1)
    r = b - A @ x
    i = np.arange(n)
    ix, iy = i % nx, (i // nx) % ny
    c0 = (ix + iy) % 2 == 0
    lat = np.zeros(n)
    for d, off, ok in ((1, -1, ix > 0), (2, 1, ix + 1 < nx), (3, -nx, iy > 0), (4, nx, iy + 1 < ny)):
        lat[ok] -= Ap[d][ok] * x[i[ok] + off]
    tol = 1e-12 * np.max(np.abs(b))
    assert np.max(np.abs(r[~c0]), initial=0.0) <= tol
    assert np.max(np.abs(r[c0] - lat[c0])) <= tol
    if nx * ny > 1:
        assert np.max(np.abs(lat[c0])) > 1e-3 * np.max(np.abs(b))
