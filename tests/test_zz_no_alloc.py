"""pf_create_static - the simulator on the library's fixed per-GPU
workspace, for callers that cannot allocate device memory - against
pf_create on the same models: two calls in a row, the second with a smaller
model, each giving the states of pf_create bit for bit; the size limit and
the one-holder rule fail cleanly."""
import numpy as np
import pytest

from paper_1807_05298_amd import inputs as I

pytestmark = pytest.mark.gpu


def _pf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_05298_amd import polyflood
    return polyflood


def _run(pf, case, opts, n_steps, static):
    sim = pf.Simulator(case, opts, static_workspace=static)
    out = []
    for k in range(n_steps):
        st = sim.step(float(case.dts[k]))
        assert st["converged"]
        out.append(sim.get_state())
    sim.close()
    return out


def _cases():
    big = I.box_case(21, 17, 6, seed=8, sigma=1.2, corr=(1.0, 2.0, 2.0), dts=[I.DAY] * 3,
                     wells=[I.Well(0, 0, 0, 5, True, I.CTRL_WRATE, 60.0 / I.DAY, c_inj=1.0),
                            I.Well(20, 16, 0, 5, False, I.CTRL_BHP, 200e5),
                            I.Well(20, 0, 1, 5, False, I.CTRL_LRATE, -20.0 / I.DAY)])
    small = I.box_case(9, 7, 3, seed=9, dts=[I.DAY] * 3)
    return big, small


def test_static_workspace_matches_pf_create_twice_in_a_row():
    pf = _pf()
    big, small = _cases()
    opts = pf.default_opts(tol_res=1e-10, tol_upd=1e-9, max_newton=20)
    assert pf.workspace_size(big, opts) > pf.workspace_size(small, opts)
    assert pf.workspace_size(big, opts) <= pf.STATIC_WORKSPACE_BYTES
    for case in (big, small):               # the second call reuses the array with a smaller model
        ref = _run(pf, case, opts, 3, static=False)
        got = _run(pf, case, opts, 3, static=True)
        for a, b in zip(ref, got):
            for fa, fb in zip(a, b):
                assert np.array_equal(fa, fb)


def test_static_workspace_mixed_precision_matches():
    pf = _pf()
    _, small = _cases()
    opts = pf.default_opts(precision=pf.PREC_MIXED, tol_res=1e-10, tol_upd=1e-9, max_newton=20)
    ref = _run(pf, small, opts, 2, static=False)
    got = _run(pf, small, opts, 2, static=True)
    for a, b in zip(ref, got):
        for fa, fb in zip(a, b):
            assert np.array_equal(fa, fb)


def test_static_workspace_limits():
    pf = _pf()
    _, small = _cases()
    opts = pf.default_opts()
    held = pf.Simulator(small, opts, static_workspace=True)
    with pytest.raises(pf.PFError) as e:
        pf.Simulator(small, opts, static_workspace=True)
    assert e.value.status == pf.PF_EBUSY
    held.close()
    again = pf.Simulator(small, opts, static_workspace=True)     # released by pf_destroy
    again.close()
    too_big = I.box_case(60, 60, 20, seed=1)
    assert pf.workspace_size(too_big, opts) > pf.STATIC_WORKSPACE_BYTES
    with pytest.raises(pf.PFError) as e:
        pf.Simulator(too_big, opts, static_workspace=True)
    assert e.value.status == pf.PF_ENOMEM
    ok = pf.Simulator(small, opts, static_workspace=True)       # a failed creation holds nothing
    ok.close()
