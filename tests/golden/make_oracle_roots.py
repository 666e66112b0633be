"""Writes the oracle's roots of three workloads too large for the oracle to
solve inside a GPU test run: the first two scheduled steps of the smallest
serving realisation (40,326 cells) and of the paper's 95x192x5 reservoir
(91,200 cells), and the first step of a 3-layer slice of the 200x200x50
field (120,000 cells).  Calls only the oracle and the input generator.

    python tests/golden/make_oracle_roots.py [name ...]

Each file holds the states after every scheduled step (P, S, C planes and
Pb), the sub-steps taken, the Newton options and a digest of the inputs; the
GPU tests regenerate the inputs, check the digest and compare their own
states with these."""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1807_05298_amd import inputs as I  # noqa: E402

TOL_RES, TOL_UPD = 1e-10, 1e-9
DT_INIT = 0.25 * I.DAY


def cases():
    return {
        "c4_r17": (lambda: I.serving_realisation(17), 2),
        "paper_low": (I.case_paper_low, 2),
        "c3_nz3": (lambda: I.case_c3(nz_override=3), 1),
    }


def input_digest(case) -> str:
    h = hashlib.sha256()
    for a in (case.poro, case.kx, case.ky, case.kz, case.P0, case.S0, case.C0, case.Pb0, case.dts):
        h.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    for w in case.wells:
        h.update(repr((w.ix, w.iy, w.k_top, w.k_bot, w.injector, w.control, float(w.target), float(w.c_inj),
                       float(w.bhp_limit), w.direction, w.ix_last)).encode())
    h.update(repr((case.nx, case.ny, case.nz, case.dx, case.dy, case.dz, case.top, case.cr, case.p_ref)).encode())
    return h.hexdigest()


def path(name: str) -> str:
    return os.path.join(HERE, f"oracle_root_{name}.npz")


def main(names):
    import oracle
    from threadpoolctl import threadpool_limits
    for name in names:
        make, n_steps = cases()[name]
        case = make()
        t0 = time.time()
        o = oracle.Oracle(case)
        with threadpool_limits(limits=1):
            states, log = o.run(oracle.NewtonOpts(tol_res=TOL_RES, tol_upd=TOL_UPD, dt_init=DT_INIT), n_steps=n_steps)
        P = np.stack([o.unpack(x)[0] for x in states])
        S = np.stack([o.unpack(x)[1] for x in states])
        C = np.stack([o.unpack(x)[2] for x in states])
        Pb = np.stack([o.unpack(x)[3] for x in states])
        np.savez_compressed(path(name), P=P, S=S, C=C, Pb=Pb, sub_dts=np.array(log.dts),
                            newton_its=np.array(log.newton_its), tol=np.array([TOL_RES, TOL_UPD, DT_INIT]),
                            digest=np.array(input_digest(case)))
        print(f"{name}: {case.n} cells, {n_steps} steps, sub-steps {[round(d / I.DAY, 4) for d in log.dts]}, "
              f"Newton {log.newton_its}, {time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(cases()))
