"""FP64 CPU oracle of the fluctuating lattice Boltzmann (FLB) time step.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference the HIP
library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  The product path
(``paper_1012_3632_amd``) never imports, links or calls anything here, and this
package imports nothing from the product path.

What it computes (Gross, Cates, Varnik, Adhikari, "Langevin theory of
fluctuations in the discrete Boltzmann equation"):

* ``lattice``  -- velocity sets, weights and the w-orthogonal moment basis
  (Sec. III eqs. moments, moments-inv, T-orthog, T-complete; App. B table
  tab:modes-d2q9 and eq. TD2Q9; a constructed D3Q19 basis, since the paper
  only cites one).
* ``philox``   -- Philox4x32-10 (Salmon et al., SC'11) and Box-Muller normals:
  the per-site, per-mode independent Gaussian draws of Sec. VI.
* ``flb``      -- the moment-space fluctuating LB update, Sec. V eq. lbe-mom,
  with relaxation rates of Sec. V (lambda^LB), the ideal-gas equilibrium
  (Sec. III eq. feq), the forcing term (Sec. III eq. forcing-term, read as the
  Guo form), the lattice-corrected velocity (Sec. V eq. lbe-moments), the LB
  noise covariance (Sec. V eq. noise-lbe) and the non-ideal force
  F = -rho grad mu (App. A eq. he-force, Sec. VI eq. f0-bulk).
* ``spectra``  -- the equilibration analysis of Sec. VI: per-mode equal-time
  spectra, the paper's G(k) (Sec. IV eq. g-mat-forcing with the OZ structure
  factor of App. A) and the exact stationary spectra of the linearized
  lattice step.
* ``capillary`` -- the capillary-fluctuation analysis of Sec. VI: interface
  heights by fitting the mean-field profile (eqs. height-def, denprof), their
  spectrum, eq. surf-tension and the capillary structure factor
  (eq. capill-static), and the scheme's interface tension by mechanics
  (Young-Laplace drops at kT = 0).
* ``modeq``    -- the modified-equilibrium (Swift) model of Sec. IV.B,
  linearized about rest on D2Q9: equilibrium moments of eq. meq-yeo, the
  correlations of eq. f-correl-yeo, the noise covariance fixed by the lattice
  FDT (its DBE limit against eq. noise-yeo), white normals filtered in
  Fourier space for the k-dependent (e, eps) block.
* ``grad``     -- reference gradients of a scalar loss of the final density
  w.r.t. the initial populations, the shear rate and kT, by reverse-mode
  automatic differentiation of ``flb`` (plain definition of the derivative).

Every function is pinned by the CPU tests ``tests/test_oracle_*.py`` against
closed forms, printed values, invariants or brute force (each module's
docstring names its pins).
"""
