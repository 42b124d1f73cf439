"""Writes tests/golden/config2_oracle.json: the FP64 oracle's solution of the
n=20,000 banded-dose QP (seed 2000), every entry of x.

Calls only ``oracle/`` and the input generator.  Run from the repository root:
    python tests/golden/make_config2_golden.py
(about 10-30 minutes on 8 cores; dense Cholesky of a 20,000 x 20,000 matrix
per IPM iteration).
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


def main(out=os.path.join(ROOT, "tests", "golden", "config2_oracle.json")):
    t0 = time.time()
    prob = qpsynth.config2()
    t1 = time.time()
    H = oracle.hessian_dense(prob)
    t2 = time.time()
    res = oracle.solve(prob, H=H, record=True)
    t3 = time.time()
    del H
    yx = oracle.lambda_x_combined(res, prob)
    yA = oracle.lambda_A_combined(res, prob)
    cert = oracle.kkt_certificate(prob, res.x, yx, yA)
    rec = {
        "about": "FP64 dense-Cholesky oracle on the banded-dose QP n=20000 (qpsynth.config2, seed 2000)",
        "written_by": "tests/golden/make_config2_golden.py",
        "converged": bool(res.converged), "ipm_iters": int(res.iters), "zeta": res.zeta,
        "objective": res.objective, "mu_final": res.mu,
        "certificate": {"eps_d": cert.eps_d, "eps_p": cert.eps_p, "eps_c": cert.eps_c, "gap": cert.gap},
        "x_inf_norm": float(np.abs(res.x).max()),
        "n_at_lower": int(np.sum(res.x < 1e-6)), "n_at_upper": int(np.sum(res.x > 50 - 1e-6)),
        "n_rows_active": int(np.sum(yA > 1e-9 * np.abs(yA).max())),
        "x": [float(v) for v in res.x],
        "seconds": {"generate": t1 - t0, "hessian": t2 - t1, "ipm": t3 - t2},
        "history": res.history,
    }
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps({k: rec[k] for k in ("converged", "ipm_iters", "objective", "certificate", "seconds")}))


if __name__ == "__main__":
    main()
