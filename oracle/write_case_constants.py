"""Writes ``paper_1912_12059_amd/case_constants.json``: the thermodynamic
numbers the synthetic initial conditions need, computed by the oracle only.

- Maxwell (binodal) densities at T = 0.85 (Sec. 2.1; the paper prints
  0.3197 and 1.8071 in Sec. 4.1.1).
- The gradient-theory surface-tension integral I(T): sigma = sqrt(kappa) I.
- Young-Laplace adjusted droplet densities (Sec. 4.3.1) for the droplet radii
  the 3D collision workloads use, at kappa = 1e-5.

Run:  python oracle/write_case_constants.py
"""
import json
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from oracle import oracle as O  # noqa: E402

T = 0.85
KAPPA = 1e-5
RADII = [0.1, 0.125, 0.15, 0.175, 0.2]


def main() -> None:
    rv, rl, ps, mus = O.maxwell(T)
    sv, sl = O.spinodal(T)
    I = O.surface_integral(T)
    sigma = math.sqrt(KAPPA) * I
    yl = {}
    for r in RADII:
        l, v = O.young_laplace(T, sigma, r)
        yl[f"{r:.3f}"] = {"rho_l": l, "rho_v": v}
    out = {
        "T": T,
        "maxwell": {"rho_v": rv, "rho_l": rl, "p_sat": ps, "mu_sat": mus},
        "spinodal": {"rho_sv": sv, "rho_sl": sl},
        "surface_integral": I,
        "kappa": KAPPA,
        "sigma": sigma,
        "young_laplace": yl,
        "provenance": "written by oracle/write_case_constants.py from the CPU oracle",
    }
    path = os.path.join(os.path.dirname(HERE), "paper_1912_12059_amd", "case_constants.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path)


if __name__ == "__main__":
    main()
