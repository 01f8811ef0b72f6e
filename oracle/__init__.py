"""CPU FP64 oracle for the dual messenger Wiener filter on the sphere.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy implementation of what the GPU library computes.  Only the test suite,
the smoke check in ``__graft_entry__`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with the HIP library and
imports nothing from the product package.

What it follows (Kodi Ramanah, Lavaux & Wandelt 2018, arXiv:1801.05358):

* the data model and Wiener filter equation (Sec. 1, eqs 1-3);
* the messenger chi^2 and its reduced two-equation form (Sec. 2, eqs 4, 8, 9);
* the cooling of xi and the Heaviside truncation of the signal covariance
  (Sec. 2, text after eq 9);
* the per-ell 3x3 signal covariance and per-pixel noise, diagonal or the
  full correlated 3x3 block (Sec. 2.1, eqs 10-11);
* distinct temperature and polarization masks (Appendix B);
* Algorithm 1 (the polarized dual messenger loop);
* constrained realizations (Sec. 2.2, eq 19);
* the residual ||A x - y|| / ||y|| with A = 1 + S^1/2 N^-1 S^1/2 (Appendix C)
  and the chi^2 of eq 3 as diagnostics.

The paper works on the flat sky with 2D FFTs (eqs 12-16).  Here the basis
change is the spin-0 / spin-2 spherical harmonic transform on a ring grid
(HEALPix or Gauss-Legendre); every SHT convention is textbook mathematics:
Wigner-d three-term recurrence, Goldberg et al. (1967) spin harmonics, and
the Zaldarriaga & Seljak (1997) E/B convention.

Modules
-------
geometry   ring grids (HEALPix RING, Gauss-Legendre)
harmonics  Wigner-d functions and spin-weighted Legendre functions
sht        synthesis Y, adjoint Y^T, analysis A = Y^T W (full -lmax..lmax m)
dm         setup, filters, schedule, the iteration, diagnostics, CR
dense      dense matrices for tiny maps: exact WF, messenger fixed point
"""
