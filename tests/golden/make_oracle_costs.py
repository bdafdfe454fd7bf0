"""Write oracle_costs.json: the FP64 oracle's LM trajectory on the seeded
synthetic workloads (initial cost, trial cost of every iteration, accept
flags, final cost).  Calls only oracle/ and the seeded generator.

    python tests/golden/make_oracle_costs.py [workload ...]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import povar_oracle as O  # noqa: E402
from paper_2405_05079_amd import synth  # noqa: E402

OUT = os.path.join(HERE, "oracle_costs.json")


def run(number: int) -> dict:
    prob = synth.workload(number)
    t0 = time.time()
    res = O.lm_solve(prob, opts=O.Options(order=prob.order, max_iters=prob.iters, ftol=0.0))
    return dict(workload=prob.name, n_cams=prob.n_cams, n_pts=prob.n_pts, n_obs=prob.n_obs,
                seeds=prob.seeds, eta=prob.eta, order=prob.order, iters=prob.iters,
                cost0=res.cost0, cost_final=res.cost, trace_cost=res.trace_cost,
                trace_accept=res.trace_accept, oracle_seconds=time.time() - t0)


if __name__ == "__main__":
    numbers = [int(a) for a in sys.argv[1:]] or [1, 2]
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for n in numbers:
        data[str(n)] = run(n)
        json.dump(data, open(OUT, "w"), indent=1)
        print(n, data[str(n)]["cost0"], data[str(n)]["cost_final"], data[str(n)]["oracle_seconds"], flush=True)
