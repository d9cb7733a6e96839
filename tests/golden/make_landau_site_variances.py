"""Write landau_site_variances_24.json: the stationary per-site variance of
every mode of the square-gradient fluid of the d3q19_256_landau workload
(a -0.01, b 0.1, rho_c 1, kappa 0.05, eta 0, all rates 1, kT 1e-6) on a
24^3 periodic box, from the exact stationary spectra of the step linearized
about rest (oracle.spectra.stationary_spectrum): the variance of mode a over
sites is sum_k <|m_a(k)|^2> / V^2.  Wavevectors where the linearized
stationary state is not unique (k = 0, where the conserved modes keep their
initial values, and a few Nyquist points) take the value G_a = rho0 kT N_a /
cs2 for the non-conserved modes and 0 for the conserved ones (a run from
rest); they weigh 1/V each.

Calls the oracle only.  Run from the repository root (about 90 s):
    python tests/golden/make_landau_site_variances.py
"""

import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import flb_workloads as W  # noqa: E402
from oracle import flb, lattice, spectra  # noqa: E402

N = 24


def main():
    kw = W.params_of("d3q19_256_landau", nx=N, ny=N, nz=N)
    p = flb.Params(**{k: v for k, v in kw.items() if k in flb.Params.__dataclass_fields__})
    lat = lattice.get("D3Q19")
    q = lat.q
    spec = spectra.stationary_spectrum(p)[:q].reshape(q, -1)
    G = p.rho0 * p.kT * np.asarray(lat.N) / lattice.CS2
    cons = np.array([c in (lattice.RHO, lattice.MOM) for c in lat.classes])
    V = N ** 3
    bad = np.isnan(spec)
    fill = np.where(cons, 0.0, G * V)[:, None] * np.ones_like(spec)
    spec = np.where(bad, fill, spec)
    var = spec.sum(1) / V ** 2
    out = dict(workload="d3q19_256_landau parameters on 24^3 (eta 0, kT 1e-6, all rates 1)",
               n=N, kT=p.kT, variance=var.tolist(), G=G.tolist(),
               ratio_to_G=(var / G).tolist(), undetermined_wavevectors=int(bad[0].sum()))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "landau_site_variances_24.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(path, np.round(var / G, 5))


if __name__ == "__main__":
    main()
