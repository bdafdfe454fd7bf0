"""Write oracle_costs.json: the FP64 oracle's LM trajectory on the seeded
synthetic workloads (initial cost, trial cost, damping and accept flag of
every iteration, final cost).  Calls only oracle/ and the seeded generator.

    python tests/golden/make_oracle_costs.py [workload[.k] ...]

"2" is problem 0 of workload 2; "2.3" is its problem 3 (data seed 2003).
A trailing "p" ("2p", "2.3p") runs the same problem from initial cameras
perturbed by one rounding unit (each entry times 1 +- 2^-52, signs from a
fixed seed): how far two FP64 runs of the same method drift apart.
Each key runs in a process of its own (one BLAS thread each), so several
keys on the command line run in parallel.
"""
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

OUT = os.path.join(HERE, "oracle_costs.json")


def run(key: str) -> dict:
    from threadpoolctl import threadpool_limits

    from oracle import povar_oracle as O
    from paper_2405_05079_amd import synth
    import numpy as np
    perturbed = key.endswith("p")
    number, _, k = key.rstrip("p").partition(".")
    prob = synth.workload(int(number), int(k or 0))
    cams0 = prob.cams0
    if perturbed:
        signs = np.random.default_rng(1).choice([-1.0, 1.0], size=cams0.shape)
        cams0 = cams0 * (1.0 + signs * 2.0 ** -52)
    t0 = time.time()
    with threadpool_limits(limits=1):
        res = O.lm_solve(prob, cams0=cams0, opts=O.Options(order=prob.order, max_iters=prob.iters, ftol=0.0))
    return dict(workload=prob.name, n_cams=prob.n_cams, n_pts=prob.n_pts, n_obs=prob.n_obs,
                seeds=prob.seeds, eta=prob.eta, order=prob.order, iters=prob.iters,
                cost0=res.cost0, cost_final=res.cost, trace_cost=res.trace_cost,
                trace_accept=res.trace_accept, trace_lambda=res.trace_lambda,
                oracle_seconds=time.time() - t0)


if __name__ == "__main__":
    keys = sys.argv[1:] or ["1", "2"]
    with ProcessPoolExecutor(max_workers=min(len(keys), 6)) as ex:
        results = dict(zip(keys, ex.map(run, keys)))
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for key, r in results.items():
        data[key] = r
        print(key, r["cost0"], r["cost_final"], round(r["oracle_seconds"], 1), flush=True)
    json.dump(data, open(OUT, "w"), indent=1)
