"""Writes workloads/coeffs.json: the fixed coefficient vectors used by the workloads.

Run from the repository root: ``python -m oracle.write_coeffs``. Calls only the
oracle's fitting routines.

* gform_v1      exponents {0,1,2,4,8,16}: least-squares fit of sum_k c_k x^(2e_k+1) to 1
                on x ~ U(0,1) with sum_k c_k = 1 (the paper's objective, Sec. 2.4, moved
                to the Gram basis).
* gform_v1_e8   the same for exponents {0,1,2,4,8}.
* paper_L14     the paper's complement-basis polynomial, depth L = 14 (ablation study),
                w_1..w_13 minimising the expected loss of Eq. (overall_polynomial) and w_14
                from Eq. (b_approximation); stored as (exponents, coefficients) of
                Y = X + sum_l w_l (I - XX^T)^(2^(l-1)) X, Eq. (newnew_formula).
"""
import json
import os

from oracle.coeffs import gform_ls_fit, tform_ls_fit, tform_exponents

PAPER_L = 14


def main():
    out = {}
    for name, exps in (("gform_v1", [0, 1, 2, 4, 8, 16]), ("gform_v1_e8", [0, 1, 2, 4, 8])):
        out[name] = {"exponents": exps, "coeffs": [float(x) for x in gform_ls_fit(exps)],
                     "basis": "gram", "norm": "frobenius"}
    w = tform_ls_fit(PAPER_L)
    out["paper_L14"] = {"exponents": tform_exponents(PAPER_L), "coeffs": [1.0] + [float(x) for x in w],
                        "basis": "complement", "norm": "gram_frobenius"}
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "workloads", "coeffs.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
