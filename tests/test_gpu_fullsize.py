"""Full-size parity of the batch and the large single QP.

* The 64-QP batch (n_k from 2,000 to 20,000, J at 0.5% in 64-voxel bands,
  m_k = n_k/10): solved by qp_solve_batch in chunks of eight, in FP64 on the
  persistent batched path (batch_mode = 1) and in FP32 on host workers
  (the default).  Every member is certified (KKT certificate <= 1e-9, from the device
  and from the oracle at the returned point); the eight members the oracle
  solved (tests/golden/config4_oracle.json, written by
  tests/golden/make_config4_golden.py from oracle/ only) are compared entry
  by entry at the bars of the precision (tests/bars.py).
* The n = 60,000 QP (J 2,000,000 x 60,000 with 200M BF16-valued nonzeros,
  rank-20 term, A 6,000 x 60,000): FP64 and BF16 solves certified at 1e-9;
  no dense oracle fits at this size (a 29 GB Hessian), so the certificate
  is the pin.
"""
import json
import os

import numpy as np
import pytest

import qpsynth
from bars import check_certificate, check_solve
from paper_2405_03584_amd import qpgpu

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
CHUNK = 8


def _golden4():
    with open(os.path.join(HERE, "golden", "config4_oracle.json")) as f:
        return {m["index"]: m for m in json.load(f)["members"]}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("chunk", range(64 // CHUNK))
def test_config4_batch_certified_and_oracle_members(chunk, prec):
    gold = _golden4()
    idx = list(range(chunk * CHUNK, (chunk + 1) * CHUNK))
    print(f"config4 members {idx[0]}..{idx[-1]} {prec}", flush=True)
    probs = [qpsynth.config4_instance(i) for i in idx]
    s = qpgpu.qp_default_settings(precision=prec, batch_mode=1 if prec == "fp64" else 0)
    hs = [qpgpu.qp_create_from_problem(p, settings=s) for p in probs]
    st, xs, infos = qpgpu.qp_solve_batch(hs)
    assert st == qpgpu.QP_OK, [f["status"] for f in infos]
    for i, p, h, x, inf in zip(idx, probs, hs, xs, infos):
        # the multipliers come from a single solve of the same handle, which
        # gives the batch's bits
        single = qpgpu.qp_solve(h)
        assert np.array_equal(single.x, x), i
        for k in ("eps_d", "eps_p", "eps_c", "gap"):
            assert inf[k] == single.info[k], (i, k)
        cert = check_certificate(p, single)
        line = f"  member {i} n={p.n} ipm={inf['ipm_iters']} pcg={inf['pcg_iters']} cert={cert.worst():.1e}"
        if i in gold:
            g = gold[i]
            dx, _ = check_solve(p, single, np.array(g["x"]), g["objective"], g["zeta"], prec)
            line += f" |x - x_oracle| = {dx:.2e}"
        print(line, flush=True)
        h.close()


@pytest.fixture(scope="module")
def config5_full():
    print("generating the n=60000 QP (200M nonzeros)", flush=True)
    return qpsynth.config5()


@pytest.mark.parametrize("prec", ["fp64", "bf16"])
def test_config5_full_size_certified(config5_full, prec):
    prob = config5_full
    print(f"config5 full size {prec}: create", flush=True)
    h = qpgpu.qp_create_from_problem(prob, settings=qpgpu.qp_default_settings(precision=prec))
    res = qpgpu.qp_solve(h)
    print(f"config5 {prec}: status {res.status} ipm {res.info['ipm_iters']} pcg {res.info['pcg_iters']} "
          f"{res.info['t_solve_ms']:.0f} ms", flush=True)
    assert res.status == qpgpu.QP_OK, res.info
    cert = check_certificate(prob, res)
    print(f"config5 {prec}: certificate {cert}", flush=True)
    h.close()
