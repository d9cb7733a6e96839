"""Write laplace_tension.json: the interface tension of the capillary
workload's scheme (D2Q9, the eta = 1 force, beta 0.1, kappa 0.08, phases 1
and 0.5, all rates 1) measured by mechanics on the oracle -- drops of three
radii relaxed at kT = 0, sigma = R (p_in - p_out) (2-D Young-Laplace) -- and
its large-radius limit from a fit sigma(R) = sigma_inf + c / R.

Calls the oracle only.  Run from the repository root:
    python tests/golden/make_laplace_tension.py
"""

import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import capillary as cap  # noqa: E402
from oracle import flb  # noqa: E402

RHO_L, RHO_V, KAPPA, BETA = 1.0, 0.5, 0.08, 0.1
DROPS = ((96, 24.0, 8000), (128, 32.0, 10000), (160, 40.0, 12000))


def main():
    p = flb.Params(lattice="D2Q9", rho0=0.75, kT=0.0, force_model=1,
                   a=-0.5 * BETA * (RHO_L - RHO_V) ** 2, b=BETA, rho_c=0.5 * (RHO_L + RHO_V),
                   kappa=KAPPA, eta=1)
    w = cap.interface_width(RHO_L, RHO_V, KAPPA, BETA)
    rows = []
    for L, R0, n in DROPS:
        d = cap.laplace_drop(p, L, R0, n, RHO_L, RHO_V, w)
        d.update(L=L, R0=R0, steps=n)
        print(json.dumps(d), flush=True)
        rows.append(d)
    R = np.array([d["R"] for d in rows])
    sig = np.array([d["sigma"] for d in rows])
    A = np.stack([np.ones_like(R), 1.0 / R], 1)
    s_inf, c = np.linalg.lstsq(A, sig, rcond=None)[0]
    out = dict(
        workload="d2q9_capillary scheme: D2Q9, eta = 1, beta 0.1, kappa 0.08, rho_L 1, "
                 "rho_V 0.5, all rates 1, kT = 0",
        drops=rows, sigma_inf=float(s_inf), curvature_coefficient=float(c),
        sigma_eq_surf_tension=float(cap.surface_tension(RHO_L, RHO_V, KAPPA, BETA)))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "laplace_tension.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(path)


if __name__ == "__main__":
    main()
