"""Write oracle_floors.json: where the oracle itself stops being exact.

For each parity grid, the forward map is solved twice by the oracle's two
independent direct solvers (pivoted banded LU after reverse Cuthill-McKee,
and SuperLU) with the oracle's own RKFIT poles, and the per-channel
difference of u(t_k) = Re sum_j c_jk x_j is recorded in the M-norm, relative
to ||u(t_k)||_M and to the size of the residue-sum terms
S_k = sum_j |c_jk| ||x_j||_M (Sec. 3.2 product S R, Sec. 3.3 M-norm).
A channel whose oracle-vs-oracle difference exceeds 1e-9 ||u(t_k)||_M cannot
pin a 1e-8 relative GPU parity claim: the GPU tests check it only through
the per-shift bound (error <= eta S_k).

    python tests/golden/make_oracle_floors.py      (about a minute on 8 cores)

Calls only the oracle and the seeded input generators.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import tem_workloads as W  # noqa: E402
from oracle import direct, rkfit, yee  # noqa: E402


def floors(wl, degree):
    fit = rkfit.rkfit(wl.t, degree)
    s, C = rkfit.shifts_and_coefficients(fit)
    P = yee.Problem(wl)
    out = []
    for src in range(len(wl.loops)):
        Xb = direct.solve_shifted(P, s, P.F[:, src], "banded")
        Xs = direct.solve_shifted(P, s, P.F[:, src], "splu")
        xn = direct.m_norm(P, Xs)
        Sk = np.abs(C).T @ xn
        Us = direct.contract(Xs, C)
        un = direct.m_norm(P, Us)
        eu = direct.m_norm(P, direct.contract(Xb, C) - Us)
        out.append({"source": src,
                    "shift_rel": (direct.m_norm(P, Xb - Xs) / xn).tolist(),
                    "eu_over_Sk": (eu / Sk).tolist(),
                    "eu_over_un": (eu / un).tolist(),
                    "Sk_over_un": (Sk / un).tolist()})
    return out


def grids():
    return {"plain16": (W.cfg_plain16(), W.cfg_plain16().degree),
            "ragged37": (W.ragged37(), 16),
            "ragged70": (W.ragged70(), 16)}


def main():
    res = {name: floors(wl, m) for name, (wl, m) in grids().items()}
    with open(os.path.join(HERE, "oracle_floors.json"), "w") as fh:
        json.dump({"note": "oracle banded LU vs SuperLU, per channel (M-norm); written by make_oracle_floors.py",
                   "grids": res}, fh, indent=1)
    for name, per in res.items():
        for r in per:
            print(name, r["source"], "max eu/Sk %.2e" % max(r["eu_over_Sk"]),
                  "channels within 1e-9 relative: %d of %d"
                  % (sum(v <= 1e-9 for v in r["eu_over_un"]), len(r["eu_over_un"])))


if __name__ == "__main__":
    main()
