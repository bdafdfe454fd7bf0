"""Write oracle_checkpoints_w2.npz: states of the FP64 oracle's LM trajectory
on problem 0 of the 250-camera workload (the one oracle_costs.json holds
under "2") at a few iterations, with the damping used there and the
oracle's trial cameras and trial cost of that iteration's step.  The GPU
tests start the library from these cameras (povar_set_state) and compare
one step with the oracle's.  Calls only oracle/ and the seeded generator.

    python tests/golden/make_oracle_checkpoints.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import povar_oracle as O  # noqa: E402
from paper_2405_05079_amd import synth  # noqa: E402

OUT = os.path.join(HERE, "oracle_checkpoints_w2.npz")
# the first iteration at the smallest damping (8), two at it, and later ones
# at dampings from 1e-9 to 1e-1
CHECKPOINTS = (0, 8, 11, 20, 33, 60, 83)


def main():
    from threadpoolctl import threadpool_limits
    prob = synth.workload(2, 0)
    opts = O.Options(order=prob.order, max_iters=1, ftol=0.0)
    P, X, f = O.initial_state(prob, prob.cams0)
    lam = opts.lambda0
    out = {k: [] for k in ("iter", "cams", "lam", "cost", "p_trial", "cost_trial")}
    it = 0
    with threadpool_limits(limits=1):
        for k in CHECKPOINTS:
            if k > it:   # run the LM loop to iteration k (resuming is exact: it is memoryless given P, lambda)
                res = O.lm_solve(prob, opts=O.Options(order=prob.order, max_iters=k - it, ftol=0.0), lam=lam, P=P)
                P, lam, it = res.P, res.lam, k
            X, _ = O.solve_landmarks(P, prob)
            f = O.cost(P, X, prob)
            lin = O.linearize(P, X, prob)
            Pn = O.retract(P, O.camera_step(P, lin, lam, prob.order))
            Xn, _ = O.solve_landmarks(Pn, prob)
            for key, v in (("iter", k), ("cams", P), ("lam", lam), ("cost", f), ("p_trial", Pn),
                           ("cost_trial", O.cost(Pn, Xn, prob))):
                out[key].append(v)
            print(k, lam, f, out["cost_trial"][-1], flush=True)
    np.savez(OUT, **{k: np.asarray(v) for k, v in out.items()})


if __name__ == "__main__":
    main()
