"""Writes workloads/coeffs.json: the fixed coefficient vectors used by the workloads.

Run from the repository root: ``python -m oracle.write_coeffs``. Calls only the
oracle's fitting routines (test infrastructure: nothing runs it at run time; the benchmark
and the tests read the stored vectors through ``workloads/configs.py`` and hand them to
the library as ordinary coefficients).

* gform_v1      exponents {0,1,2,4,8,16}: least-squares fit of sum_k c_k x^(2e_k+1) to 1
                on x ~ U(0,1) with sum_k c_k = 1 (the paper's objective, Sec. 2.4, moved
                to the Gram basis).
* gform_v1_e8   the same for exponents {0,1,2,4,8}.
* paper_L14     the paper's complement-basis polynomial, depth L = 14 (ablation study),
                w_1..w_13 minimising the expected loss of Eq. (overall_polynomial) and w_14
                from Eq. (b_approximation); stored as (exponents, coefficients) of
                Y = X + sum_l w_l (I - XX^T)^(2^(l-1)) X, Eq. (newnew_formula).

Newton-Schulz step schedules of the baselines (one (a, b, c) per step of
X <- a X + b (XX^T) X + c (XX^T)^2 X, and the input scaling: gelfand_q = 0 for ||A||_F,
q >= 1 for Gelfand's bound ||(AA^T)^q||_F^(1/(2q))):

* original_ns8  the cubic of Eq. (one_iteration_matrix), eight steps.
* muon_ns5      Muon's quintic of Eq. (iteration_jordan), five steps.
* cesista_ns5   five quintics in Cesista's (gamma, r, u) form, fitted by the oracle.
* cans_ns5_q2   five minimax quintics for singular values in [1e-3, 1] (2 % margin at the top of
                each interval), Gelfand q = 2.
"""
import json
import os

from oracle.baselines import cans_schedule, cesista_fit
from oracle.coeffs import gform_ls_fit, tform_ls_fit, tform_exponents

PAPER_L = 14
MUON_ABC = (3.4445, -4.7750, 2.0315)  # Eq. (iteration_jordan)
CUBIC_ABC = (1.5, -0.5, 0.0)  # Eq. (one_iteration_matrix)


def main():
    out = {}
    for name, exps in (("gform_v1", [0, 1, 2, 4, 8, 16]), ("gform_v1_e8", [0, 1, 2, 4, 8])):
        out[name] = {"exponents": exps, "coeffs": [float(x) for x in gform_ls_fit(exps)],
                     "basis": "gram", "norm": "frobenius"}
    w = tform_ls_fit(PAPER_L)
    out["paper_L14"] = {"exponents": tform_exponents(PAPER_L), "coeffs": [1.0] + [float(x) for x in w],
                        "basis": "complement", "norm": "gram_frobenius"}
    sched = {
        "original_ns8": ([CUBIC_ABC] * 8, 0),
        "muon_ns5": ([MUON_ABC] * 5, 0),
        "cesista_ns5": (cesista_fit(5)[1], 0),
        "cans_ns5_q2": (cans_schedule(5, 1e-3, 5)[0], 2),
    }
    for name, (steps, q) in sched.items():
        out[name] = {"schedule": [[float(v) for v in abc] for abc in steps], "gelfand_q": q}
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "workloads", "coeffs.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
