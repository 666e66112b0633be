"""Parity at full size, in the launch configuration bench.py times:

* 60x220x85 (1.12M cells): residual and Jacobian rows of a sample of cells
  (random, boundary and perforated) against the oracle's rows; after the
  bench's warm-up steps, one 5-day step whose state is a root of the
  oracle's own backward-Euler residual to the bench's tolerance (a property
  that holds at any size);
* 300^3 (27M cells), mixed precision: the first scheduled step, then a
  1-day step whose state is an oracle root on every perforated cell and a
  random sample of the others;
* 200x200x50 (2M cells): FP64 and mixed precision reach the same root (per
  field within 1e-6), and the mixed state is an oracle root on a sample;
* the paper's high-resolution model (27.4M blocks): the first sub-step is an
  oracle root on every perforated cell and a random sample.
"""
import numpy as np
import pytest

import oracle
from paper_1807_05298_amd import inputs as I
from tests.gpu_helpers import field_rel_err, planes_to_block

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::scipy.sparse.SparseEfficiencyWarning")]


def _pf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_05298_amd import polyflood
    return polyflood


def _sample_cells(case, rng, k=1500):
    n = case.n
    nx, ny, nz = case.nx, case.ny, case.nz
    cells = set(rng.choice(n, k, replace=False).tolist())
    for iz in (0, nz - 1):
        for iy in (0, ny - 1):
            for ix in (0, nx - 1, nx // 2):
                cells.add(ix + nx * (iy + ny * iz))
    for w in case.wells:
        for kz in (w.k_top, (w.k_top + w.k_bot) // 2, w.k_bot):
            cells.add(w.ix + nx * (w.iy + ny * kz))
    return np.array(sorted(cells), dtype=np.int64)


def test_c2_assembly_sampled_rows():
    pf = _pf()
    case = I.case_c2()
    rng = np.random.default_rng(21)
    n = case.n
    sim = pf.Simulator(case, pf.default_opts())
    xn = (case.P0, case.S0, case.C0, case.Pb0)
    x = (case.P0 + rng.uniform(-5e5, 5e5, n), rng.uniform(0.2, 0.8, n), rng.uniform(0.0, 1.2, n),
         case.Pb0 + rng.uniform(-1e5, 1e5, case.n_wells))
    dt = 5 * I.DAY
    sim.set_state(*xn)
    sim.begin_step()
    sim.set_state(*x)
    R, J, _ = sim.assemble(dt, with_border=False)
    o = oracle.Oracle(case)
    xb = o.pack(*x)
    Mn = o.accum(o.pack(*xn))
    cells = _sample_cells(case, rng)
    Ro = o.residual_cells(xb, Mn, dt, cells) / o.res_scale[:3 * n].reshape(-1, 3)[cells]
    Rg = np.stack([R[cells], R[n + cells], R[2 * n + cells]], axis=1)
    assert np.max(np.abs(Rg - Ro)) <= 1e-11 + 1e-10 * np.max(np.abs(Ro))
    Jo = o.jacobian(xb, Mn, dt, cells=cells, with_wells=False)
    Jo = Jo.multiply(1.0 / o.res_scale[:, None]).tocsr()      # the library's row scaling
    Jp = J.reshape(7, 9, n)
    nx, ny = case.nx, case.ny
    offs = [0, -1, 1, -nx, nx, -nx * ny, nx * ny]
    worst = 0.0
    where = None
    for i in cells:
        for e in range(3):
            row = Jo.getrow(3 * i + e)
            ref = dict(zip(row.indices.tolist(), row.data.tolist()))
            scale = max(abs(v) for v in ref.values())
            for d in range(7):
                j = i + offs[d]
                for c in range(3):
                    g = Jp[d, 3 * e + c, i]
                    r = ref.pop(3 * j + c, 0.0) if 0 <= j < n else 0.0
                    if abs(g - r) / scale > worst:
                        worst = abs(g - r) / scale
                        where = dict(cell=int(i), xyz=(int(i % nx), int(i // nx % ny), int(i // (nx * ny))),
                                     row=e, block=d, col=c, gpu=float(g), oracle=float(r), scale=float(scale))
            # what is left in the oracle's row are well columns (not in the cell blocks)
            assert all(k >= 3 * n for k in ref), ref
    assert worst <= 1e-11, (worst, where)


def test_c2_bench_step_is_an_oracle_root():
    """After the bench's warm-up, one backward-Euler step of 5 days driven
    through pf_begin_step / pf_newton_iteration with the bench's options:
    the state returned is a root of the oracle's residual to the bench's
    tolerance."""
    pf = _pf()
    case = I.case_c2()
    opts = pf.default_opts(tol_res=1e-6, tol_upd=1e-3, dt_init=0.25 * I.DAY)
    sim = pf.Simulator(case, opts)
    for k in range(2):
        sim.step(float(case.dts[k]))
    xs = sim.get_state()
    dt = float(case.dts[2])
    sim.begin_step()
    converged = False
    for _ in range(opts.max_newton + 1):
        st = sim.newton_iteration(dt)
        if st["converged"]:
            converged = True
            break
    assert converged
    x1 = sim.get_state()
    o = oracle.Oracle(case)
    R = o.residual(o.pack(*x1), o.accum(o.pack(*xs)), dt)
    r = np.abs(R / o.res_scale)
    assert np.max(r) <= 1.01 * opts.tol_res, np.max(r)
    # something happened: water and polymer moved away from the injector
    assert np.max(x1[1]) > 0.3 and np.max(x1[2]) > 0.1


def _perforated_cells(case):
    out = []
    for w in case.wells:
        if w.direction == I.WELL_X:
            out += [i + case.nx * (w.iy + case.ny * w.k_top) for i in range(w.ix, w.ix_last + 1)]
        else:
            out += [w.ix + case.nx * (w.iy + case.ny * k) for k in range(w.k_top, w.k_bot + 1)]
    return np.unique(np.array(out, dtype=np.int64))


def _sampled_root_residual(o, case, xs, x1, dt, rng, k_random):
    """max |R~| of the oracle's residual over every perforated cell and a
    random sample of the others, at the GPU's end-of-step state."""
    n = case.n
    cells = np.unique(np.concatenate([_perforated_cells(case), rng.choice(n, k_random, replace=False)]))
    Mn = o.accum(o.pack(*xs))
    Ro = o.residual_cells(o.pack(*x1), Mn, dt, cells)
    return np.max(np.abs(Ro / o.res_scale[:3 * n].reshape(-1, 3)[cells])), len(cells)


def test_c5_mixed_first_step_is_an_oracle_root():
    """The 300^3 case (27M cells, 100 wells) in mixed precision: the first
    scheduled 10-day step from the initial state (sub-steps from 0.25 d), as
    the bench runs it.  The state returned is a root of the oracle's residual
    to the Newton tolerance on every perforated cell and 20,000 others."""
    pf = _pf()
    case = I.case_c5()
    opts = pf.default_opts(precision=pf.PREC_MIXED, dt_init=0.25 * I.DAY)
    sim = pf.Simulator(case, opts)
    dt = float(case.dts[0])
    st = sim.step(dt)
    assert st["converged"] and abs(st["dt_taken"] - dt) < 1e-6 * dt
    # the last sub-step's start state is not exposed by pf_step: take one more
    # backward-Euler step of 1 day through the Newton-iteration entry point
    xs = sim.get_state()
    sim.begin_step()
    dt1 = 1.0 * I.DAY
    for _ in range(opts.max_newton + 1):
        if sim.newton_iteration(dt1)["converged"]:
            break
    else:
        raise AssertionError("no convergence")
    x1 = sim.get_state()
    o = oracle.Oracle(case)
    r, ncells = _sampled_root_residual(o, case, xs, x1, dt1, np.random.default_rng(5), 20000)
    assert r <= 1.01 * opts.tol_res, (r, ncells)
    assert np.min(x1[2]) >= 0.0 and np.max(x1[1]) > 0.25


def test_c3_mixed_and_fp64_reach_the_same_root():
    """The 200x200x50 case (2M cells): one 5-day step (sub-steps from
    0.25 d) in FP64 and in mixed precision (FP32/BF16 CPR inside FP64
    FGMRES), both to tol_res 1e-9 / tol_upd 1e-8.  Per field, max |mixed -
    fp64| / max(|fp64|_inf, floor) stays within 1e-6 for P and S (and C, Pb),
    and the mixed state is a root of the oracle's residual."""
    pf = _pf()
    case = I.case_c3()
    res = {}
    for name, prec in (("fp64", pf.PREC_FP64), ("mixed", pf.PREC_MIXED)):
        opts = pf.default_opts(precision=prec, tol_res=1e-9, tol_upd=1e-8, dt_init=0.25 * I.DAY, max_newton=16)
        sim = pf.Simulator(case, opts)
        st = sim.step(float(case.dts[0]))
        assert st["converged"]
        res[name] = sim.get_state()
        if name == "mixed":
            # a further 1-day backward-Euler step whose start state is known
            sim.begin_step()
            dt1 = 1.0 * I.DAY
            for _ in range(opts.max_newton + 1):
                if sim.newton_iteration(dt1)["converged"]:
                    break
            else:
                raise AssertionError("no convergence")
            x1 = sim.get_state()
            o = oracle.Oracle(case)
            r, ncells = _sampled_root_residual(o, case, res["mixed"], x1, dt1, np.random.default_rng(3), 50000)
            assert r <= 1.01 * opts.tol_res, (r, ncells)
        sim.close()
    floor_c = max(w.c_inj for w in case.wells if w.injector)
    errs = dict(P=field_rel_err(res["mixed"][0], res["fp64"][0], 1.0),
                S=field_rel_err(res["mixed"][1], res["fp64"][1], 1.0),
                C=field_rel_err(res["mixed"][2], res["fp64"][2], floor_c),
                Pb=field_rel_err(res["mixed"][3], res["fp64"][3], 1.0))
    print("c3 mixed vs fp64 per-field relative error:", errs)
    assert all(v <= 1e-6 for v in errs.values()), errs


def test_paper_high_resolution_first_substep_is_an_oracle_root():
    """The paper's high-resolution performance model (951x1920x15, 27.4M
    blocks, Table 3 layers, four corner injectors, horizontal producer):
    the first 0.005-day sub-step from the initial state, as the bench starts
    it, converges to a root of the oracle's residual on every perforated
    cell and 20,000 others."""
    pf = _pf()
    case = I.case_paper_high()
    opts = pf.default_opts(precision=pf.PREC_MIXED)
    sim = pf.Simulator(case, opts)
    xs = (case.P0, case.S0, case.C0, case.Pb0)
    dt = 0.005 * I.DAY
    sim.begin_step()
    for _ in range(opts.max_newton + 1):
        if sim.newton_iteration(dt)["converged"]:
            break
    else:
        raise AssertionError("no convergence")
    x1 = sim.get_state()
    o = oracle.Oracle(case)
    r, ncells = _sampled_root_residual(o, case, xs, x1, dt, np.random.default_rng(9), 20000)
    assert r <= 1.01 * opts.tol_res, (r, ncells)


# ---------------------------------------------------------------------------
# Tight FP64 steps checked against the oracle's residual on every cell, and
# whole runs compared with stored oracle roots
# ---------------------------------------------------------------------------
TIGHT = dict(inexact=0, lin_tol=1e-9, tol_res=1e-10, tol_upd=1e-8, max_newton=20)


def _tight_step_root_check(pf, case, sim, dt, label):
    """One backward-Euler step of length dt from the simulator's current
    state at the tight tolerances, through pf_begin_step /
    pf_newton_iteration; returns max |R~| of the oracle's residual over every
    cell and well at the GPU's end state (the start state is the GPU's)."""
    sim.set_opts(pf.default_opts(**TIGHT))
    xs = sim.get_state()
    sim.begin_step()
    for _ in range(TIGHT["max_newton"] + 1):
        if sim.newton_iteration(dt)["converged"]:
            break
    else:
        raise AssertionError(f"{label}: no convergence at tol_res 1e-10")
    x1 = sim.get_state()
    o = oracle.Oracle(case)
    Mn = o.accum_threaded(o.pack(*xs))
    xb = o.pack(*x1)
    n = case.n
    Rc = o.cell_residuals(xb, Mn, dt)
    rc = np.abs(Rc / o.res_scale[:3 * n].reshape(-1, 3))
    rw = np.abs(o.well_residuals(xb) / o.res_scale[3 * n:]) if case.n_wells else np.zeros(1)
    worst = int(np.argmax(rc.max(axis=1)))
    print(f"{label}: oracle max|R~| cells {rc.max():.3e} (cell {worst}), wells {rw.max():.3e}")
    return max(float(rc.max()), float(rw.max())), x1


def test_c2_fp64_tight_step_is_an_oracle_root_on_every_cell():
    """60x220x85 (1.12M cells), FP64: after the bench's two warm-up steps,
    a 5-day step to tol_res 1e-10 is a root of the oracle's residual on every
    one of the 3,366,005 rows to that tolerance."""
    pf = _pf()
    case = I.case_c2()
    sim = pf.Simulator(case, pf.default_opts(tol_res=1e-6, tol_upd=1e-3, dt_init=0.25 * I.DAY))
    for k in range(2):
        sim.step(float(case.dts[k]))
    r, x1 = _tight_step_root_check(pf, case, sim, float(case.dts[2]), "c2 fp64")
    assert r <= 1.01e-10, r
    assert np.max(x1[1]) > 0.3 and np.max(x1[2]) > 0.1


def test_c5_fp64_tight_step_is_an_oracle_root_on_every_cell():
    """300^3 (27M cells, 100 wells), FP64 as the bench runs it: the first
    10-day step from the initial state (sub-steps from 0.25 d), then a 1-day
    step to tol_res 1e-10 that is a root of the oracle's residual on every one
    of the 81,000,100 rows to that tolerance."""
    pf = _pf()
    case = I.case_c5()
    sim = pf.Simulator(case, pf.default_opts(dt_init=0.25 * I.DAY))
    st = sim.step(float(case.dts[0]))
    assert st["converged"] and abs(st["dt_taken"] - float(case.dts[0])) < 1e-6 * float(case.dts[0])
    r, x1 = _tight_step_root_check(pf, case, sim, 1.0 * I.DAY, "c5 fp64")
    assert r <= 1.01e-10, r
    assert np.min(x1[2]) >= 0.0 and np.max(x1[1]) > 0.25


def _golden_root(name, case):
    """The oracle's states written by tests/golden/make_oracle_roots.py for
    this case; the inputs must be the ones the file was made from."""
    from tests.golden import make_oracle_roots as G
    g = np.load(G.path(name))
    assert str(g["digest"]) == G.input_digest(case), \
        f"inputs of {name} changed since its oracle roots were written: rerun make_oracle_roots.py {name}"
    return g, G


def _gpu_schedule(pf, case, n_steps, opts):
    sim = pf.Simulator(case, opts)
    out = []
    for k in range(n_steps):
        sim.apply_events(case, k)
        st = sim.step(float(case.dts[k]))
        assert st["converged"], (k, st)
        out.append(sim.get_state())
    sim.close()
    return out


def _compare_golden(case, g, states, tol, label):
    floor_c = max([w.c_inj for w in case.wells if w.injector] + [1.0])
    worst = {}
    for k, x in enumerate(states):
        ref = (g["P"][k], g["S"][k], g["C"][k], g["Pb"][k])
        for name, a, b, floor in zip(("P", "S", "C", "Pb"), x, ref, (1.0, 1.0, floor_c, 1.0)):
            worst[name] = max(worst.get(name, 0.0), field_rel_err(a, b, floor) if b.size else 0.0)
    print(f"{label}: per-field error against the oracle {worst}")
    assert all(v <= tol for v in worst.values()), (label, worst)
    return worst


def test_serving_realisation_matches_the_oracle():
    """The smallest realisation of the serving generator (33x26x47, 40,326
    cells), its first two 5-day steps from sub-steps of 0.25 d, FP64 at
    tol_res 1e-10: every state agrees with the oracle's to 1e-8 per field,
    through a simulator and through the serving loop, with one stream per
    slot and with fused launches beside another realisation."""
    pf = _pf()
    case = I.serving_realisation(17)
    g, G = _golden_root("c4_r17", case)
    opts = pf.default_opts(tol_res=G.TOL_RES, tol_upd=G.TOL_UPD, dt_init=G.DT_INIT, max_newton=20)
    states = _gpu_schedule(pf, case, 2, opts)
    _compare_golden(case, g, states, 1e-8, "c4 realisation 17")
    first = (g["P"][0], g["S"][0], g["C"][0], g["Pb"][0])
    # through the serving loop, one stream per slot and fused (with a second realisation in the mix);
    # the server returns the end state of the schedule: compare it with the oracle's second step
    other = I.serving_realisation(30)
    for fused in (0, 1):
        sv = pf.Server(2 * pf.workspace_size(case, opts) + 2 * pf.workspace_size(other, opts), max_slots=2,
                       fused=fused)
        t = sv.submit(case, opts, n_steps=2)
        sv.submit(other, opts, n_steps=2)
        sv.wait()
        state, res = sv.poll(t)
        sv.close()
        assert state == 2
        _compare_golden(case, g, [first, (res["P"], res["S"], res["C"], res["Pb"])], 1e-8,
                        f"c4 realisation 17 (server, fused={fused})")


def test_paper_low_resolution_matches_the_oracle():
    """The paper's 95x192x5 performance-test reservoir (91,200 blocks, Table 3
    layers, four BHP-limited corner injectors and the horizontal producer) at
    its own size: the first two 10-day steps from sub-steps of 0.25 d, FP64
    at tol_res 1e-10, agree with the oracle's to 1e-8 per field."""
    pf = _pf()
    case = I.case_paper_low()
    g, G = _golden_root("paper_low", case)
    opts = pf.default_opts(tol_res=G.TOL_RES, tol_upd=G.TOL_UPD, dt_init=G.DT_INIT, max_newton=20)
    states = _gpu_schedule(pf, case, 2, opts)
    _compare_golden(case, g, states, 1e-8, "paper 95x192x5")


def test_c3_slice_mixed_precision_error_against_the_oracle():
    """A 3-layer slice of the 200x200x50 field (120,000 cells, the 25-well
    line drive at the same rate per perforated layer): the first 5-day step
    (sub-steps from 0.25 d) at tol_res 1e-10 with the FP32/BF16 preconditioner
    inside FP64 FGMRES, and in FP64.  Per field against the oracle's root:
    mixed within 1e-6 (the bar for reduced precision), FP64 within 1e-8."""
    pf = _pf()
    case = I.case_c3(nz_override=3)
    g, G = _golden_root("c3_nz3", case)
    errs = {}
    for name, prec, tol in (("fp64", pf.PREC_FP64, 1e-8), ("mixed", pf.PREC_MIXED, 1e-6)):
        opts = pf.default_opts(precision=prec, tol_res=G.TOL_RES, tol_upd=G.TOL_UPD, dt_init=G.DT_INIT,
                               max_newton=20)
        states = _gpu_schedule(pf, case, 1, opts)
        errs[name] = _compare_golden(case, g, states, tol, f"c3 slice {name}")
    print("c3 slice per-field error against the oracle:", errs)
