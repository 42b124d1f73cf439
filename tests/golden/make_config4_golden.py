"""Writes tests/golden/config4_oracle.json: the FP64 oracle's solutions of an
8-member subset of the 64-QP batch (qpsynth.config4_instance, seed 4000): the
four smallest members and four more drawn at random from the rest (seeded,
below).  Every entry of x, the objective, the iteration count and the KKT
certificate of each member.

Calls only ``oracle/`` and the input generator.  Run from the repository root:
    python tests/golden/make_config4_golden.py
(dense Cholesky of an n x n matrix per IPM iteration, n up to 20,000: tens of
minutes on 8 cores).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import qpsynth  # noqa: E402

SUBSET_SEED = 4099


def subset():
    """The four smallest members, then four drawn without replacement from
    the other 60 with numpy.random.default_rng(SUBSET_SEED)."""
    sizes = qpsynth.config4_sizes()
    order = np.argsort(sizes, kind="stable")
    small = [int(i) for i in order[:4]]
    rest = np.array(sorted(int(i) for i in order[4:]))
    rng = np.random.default_rng(SUBSET_SEED)
    drawn = [int(i) for i in rng.choice(rest, size=4, replace=False)]
    return small, drawn


def main(out=os.path.join(ROOT, "tests", "golden", "config4_oracle.json")):
    small, drawn = subset()
    members = []
    for idx in small + drawn:
        t0 = time.time()
        prob = qpsynth.config4_instance(idx)
        res = oracle.solve(prob)
        yx = oracle.lambda_x_combined(res, prob)
        yA = oracle.lambda_A_combined(res, prob)
        cert = oracle.kkt_certificate(prob, res.x, yx, yA)
        rec = {"index": idx, "n": prob.n, "m": prob.m, "nnz_J": int(prob.J.nnz),
               "converged": bool(res.converged), "ipm_iters": int(res.iters), "zeta": res.zeta,
               "objective": res.objective,
               "certificate": {"eps_d": cert.eps_d, "eps_p": cert.eps_p, "eps_c": cert.eps_c,
                               "gap": cert.gap},
               "x": [float(v) for v in res.x], "seconds": time.time() - t0}
        members.append(rec)
        print(json.dumps({k: rec[k] for k in ("index", "n", "converged", "ipm_iters", "objective",
                                               "certificate", "seconds")}), flush=True)
    doc = {"about": "FP64 dense-Cholesky oracle on 8 members of the 64-QP batch (qpsynth.config4_instance, "
                    "seed 4000): the 4 smallest, then 4 drawn at random from the rest",
           "written_by": "tests/golden/make_config4_golden.py",
           "smallest": small, "drawn": drawn, "subset_seed": SUBSET_SEED,
           "members": members}
    with open(out, "w") as f:
        json.dump(doc, f, indent=0)


if __name__ == "__main__":
    main()
