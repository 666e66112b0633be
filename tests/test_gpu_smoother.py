"""The CPR second-stage smoother (Sec. 3.4: block Jacobi, or red-black
block ILU(0) on colour-split storage) through the C ABI hook
pf_smoother_apply, against the plain numpy definitions of
tests/precond_ref.py built from the Jacobian that pf_assemble returns:
FP64 to 1e-12 relative, the mixed-precision form (BF16 off-diagonal
blocks, FP32 inverse diagonals and arithmetic) against the same rounding
in numpy to 1e-4."""
import numpy as np
import pytest

from paper_1807_05298_amd import inputs as I
from precond_ref import bjac_apply, blocks, ilu_apply, ilu_apply_mixed

pytestmark = pytest.mark.gpu


def _pf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_05298_amd import polyflood
    return polyflood


def _setup(shape, seed, **opts):
    pf = _pf()
    nx, ny, nz = shape
    wells = [I.Well(0, 0, 0, nz - 1, True, I.CTRL_WRATE, 30.0 / I.DAY, c_inj=1.0),
             I.Well(nx - 1, ny - 1, 0, nz - 1, False, I.CTRL_BHP, 200e5)]
    case = I.box_case(nx, ny, nz, seed=seed, wells=wells, dz=1.0, sigma=1.5, corr=(2.0, 2.0, 2.0))
    sim = pf.Simulator(case, pf.default_opts(max_lin_it=5, **opts))
    sim.begin_step()
    sim.assemble(case.dts[0], with_jacobian=False, with_border=False)
    rng = np.random.default_rng(seed)
    sim.linear_solve(rng.standard_normal(sim.nv), 1e-3)
    _, J, border = sim.assemble(case.dts[0])
    st = sim.static()
    Dw = np.zeros(sim.nw)
    Dw[st["perf_well"]] = border[:, 6]
    return sim, J, Dw


SHAPES = [(10, 8, 3), (13, 9, 4), (7, 5, 11), (32, 20, 6)]
# layers of at least 65,536 cells: the ILU set-up takes the cells in y-strips
LARGE = [(330, 200, 2)]


@pytest.mark.parametrize("shape", SHAPES + LARGE)
def test_rb_ilu0_matches_numpy(shape):
    sim, J, Dw = _setup(shape, 3)
    n = int(np.prod(shape))
    f = np.random.default_rng(4).standard_normal(sim.nv)
    z = sim.smoother_apply(f)
    ref = ilu_apply(blocks(J, n), shape, f, Dw)
    assert np.max(np.abs(z - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("shape", SHAPES + LARGE)
def test_rb_ilu0_mixed_matches_numpy(shape):
    pf = _pf()
    sim, J, Dw = _setup(shape, 5, precision=pf.PREC_MIXED)
    n = int(np.prod(shape))
    f = np.random.default_rng(6).standard_normal(sim.nv)
    z = sim.smoother_apply(f)
    ref = ilu_apply_mixed(blocks(J, n), shape, f, Dw)
    assert np.max(np.abs(z - ref)) <= 1e-4 * np.max(np.abs(ref))
    # and within BF16 rounding of the FP64 smoother
    ref64 = ilu_apply(blocks(J, n), shape, f, Dw)
    assert np.max(np.abs(z - ref64)) <= 5e-2 * np.max(np.abs(ref64))


@pytest.mark.parametrize("shape", SHAPES[:2])
def test_block_jacobi_matches_numpy(shape):
    pf = _pf()
    sim, J, Dw = _setup(shape, 7, smoother=pf.SMOOTH_BJAC)
    n = int(np.prod(shape))
    f = np.random.default_rng(8).standard_normal(sim.nv)
    z = sim.smoother_apply(f)
    ref = bjac_apply(blocks(J, n), f, Dw)
    assert np.max(np.abs(z - ref)) <= 1e-12 * np.max(np.abs(ref))
