"""Write oracle_step_w3.npz and oracle_step_w5.npz: one damped camera step of
the FP64 oracle at the initial cameras of the 1,800-camera workload (order
20) and of the 13,700-camera workload (order 30), lambda = 1e-3: the ambient
step of every camera, the trial cameras, the cost there and at the start.
Calls only oracle/ and the seeded generator (the memory-bounded step:
about 30 GB of host memory and ten minutes for the larger workload).

    python tests/golden/make_oracle_steps_large.py [3] [5]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import povar_oracle as O  # noqa: E402
from paper_2405_05079_amd import synth  # noqa: E402

LAMBDA = 1e-3


def main(number: int):
    t0 = time.time()
    prob = synth.workload(number)
    P = prob.cams0 / np.linalg.norm(prob.cams0, axis=1, keepdims=True)
    dp, X, f = O.camera_step_large(P, prob, LAMBDA, prob.order)
    Pn = O.retract(P, dp)
    Xn, _ = O.solve_landmarks(Pn, prob)
    ft = O.cost(Pn, Xn, prob)
    np.savez(os.path.join(HERE, f"oracle_step_w{number}.npz"), dp=dp, p_trial=Pn, cost=f, cost_trial=ft,
             lam=LAMBDA, order=prob.order, n_obs=prob.n_obs, seeds=np.array([prob.seeds["data"], prob.seeds["init"]]))
    print(number, prob.n_obs, f, ft, round(time.time() - t0, 1), flush=True)


if __name__ == "__main__":
    for a in sys.argv[1:] or ["3", "5"]:
        main(int(a))
