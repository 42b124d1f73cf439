"""qp_solve_batch on its persistent path (batch_mode = 1): QPs on the line
format, solved together by batched PCG launches over global work lists
(batch_kernels.hpp); and on host workers (the default) for comparison.

Each QP's result must be the bits of its own qp_solve (the batched launches
run every QP's kernels with that QP's arguments), with the same IPM and PCG
iteration counts, and its minimiser the oracle's at the precision's bars.
The members are uneven on purpose: the four smallest QPs of the 64-QP batch
(n = 2000-2400), a scaled banded QP, and the ragged-lines QP, whose lines
cover the line format's edge cases and whose low-precision directions take
the FP64 fallback (the refinement cannot converge there), so QPs leave the
PCG work lists at different iterations and the IPM at different points."""
import numpy as np
import pytest

import oracle
import qpsynth
from bars import check_solve_vs_oracle
from paper_2405_03584_amd import qpgpu

pytestmark = pytest.mark.gpu


def _members():
    sizes = qpsynth.config4_sizes()
    small = [int(i) for i in np.argsort(sizes, kind="stable")[:4]]
    return [qpsynth.config4_instance(i) for i in small] + [qpsynth.config2(scale=0.02), qpsynth.ragged_lines()]


@pytest.fixture(scope="module")
def members():
    probs = _members()
    return probs, [oracle.solve(p) for p in probs]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_persistent_batch_equals_single_solves_and_oracle(members, prec):
    probs, refs = members
    print(f"persistent batch {prec}: " + ", ".join(f"{p.name} n={p.n}" for p in probs), flush=True)
    s = qpgpu.qp_default_settings(precision=prec, batch_mode=1)
    hs = [qpgpu.qp_create_from_problem(p, settings=s) for p in probs]
    st, xs, infos = qpgpu.qp_solve_batch(hs)
    assert st == qpgpu.QP_OK, [i["status"] for i in infos]
    # the same batch on host workers (batch_mode 0 on every handle)
    hw = [qpgpu.qp_create_from_problem(p, settings=qpgpu.qp_default_settings(precision=prec)) for p in probs]
    st_w, xs_w, infos_w = qpgpu.qp_solve_batch(hw)
    assert st_w == qpgpu.QP_OK
    for p, ref, h, x, inf, xw, infw in zip(probs, refs, hs, xs, infos, xs_w, infos_w):
        single = qpgpu.qp_solve(h)
        assert xw.tobytes() == x.tobytes(), p.name
        assert infw["pcg_iters"] == inf["pcg_iters"], p.name
        print(f"  {p.name}: batch ipm {inf['ipm_iters']} pcg {inf['pcg_iters']} | single ipm "
              f"{single.info['ipm_iters']} pcg {single.info['pcg_iters']}", flush=True)
        assert x.tobytes() == single.x.tobytes(), p.name
        for k in ("ipm_iters", "pcg_iters", "pcg_solves", "objective", "eps_d", "eps_p", "eps_c", "gap"):
            assert inf[k] == single.info[k], (p.name, k, inf[k], single.info[k])
        check_solve_vs_oracle(p, single, ref, prec)
        h.close()
    for h in hw:
        h.close()


def test_persistent_batch_twice_on_the_same_handles(members):
    """A second batch solve of the same handles (graphs and tables rebuilt)
    gives the same bits."""
    probs, _ = members
    hs = [qpgpu.qp_create_from_problem(p, settings=qpgpu.qp_default_settings(batch_mode=1)) for p in probs[:3]]
    st1, xs1, _ = qpgpu.qp_solve_batch(hs)
    st2, xs2, _ = qpgpu.qp_solve_batch(hs)
    assert st1 == st2 == qpgpu.QP_OK
    for a, b in zip(xs1, xs2):
        assert a.tobytes() == b.tobytes()
    for h in hs:
        h.close()
