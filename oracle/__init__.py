"""FP64 CPU oracle for the IPM search-direction path.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call or execute anything here.
It shares no code with the GPU library (``paper_2405_03584_amd``) and never
imports it.
"""
from .ipm_dense import (OracleSettings, OracleResult, solve, hessian_dense, hessian_apply,
                        objective, condensed_operator_dense, newton_solve_dense,
                        lambda_A_combined, lambda_x_combined, make_groups, GROUPS)
from .certificate import kkt_certificate, bruteforce_qp, Certificate

__all__ = ["OracleSettings", "OracleResult", "solve", "hessian_dense", "hessian_apply",
           "objective", "condensed_operator_dense", "newton_solve_dense",
           "lambda_A_combined", "lambda_x_combined", "make_groups", "GROUPS",
           "kkt_certificate", "bruteforce_qp", "Certificate"]
