"""FP64 CPU oracle for the partial-sky box simulator (test infrastructure only).

This package is the plain, slow reference against which the HIP path is checked. It is
imported only by ``tests/``, by ``__graft_entry__.smoke()`` and by the ``cpu_baseline``
leg of ``bench.py``; the product path never imports, calls or links it, and it imports
nothing from the product package. The two sides share only the seeded input generators
(``paper_2507_15703_amd.workloads``), which hold none of the method's arithmetic.

What it computes (Giner Mascarell & Bunn, arXiv:2507.15703):

* ``philox``    -- the Philox4x32-10 counter-based generator (Salmon et al., SC'11).
* ``normal``    -- the canonical Box-Muller transform of two 32-bit words into a pair of
                   unit normals, written with +, -, x and bit operations only.
* ``spectrum``  -- the box power spectrum P_box = P_inf (2 pi / L)^3 (Sec. II C, eq.
                   finalpbox with M = N) and the per-|k|^2 weight tables.
* ``noise``     -- complex Gaussian modes of variance P_box on the Hermitian half grid
                   (Sec. II D 1, the 3-D Fourier method).
* ``field``     -- the unnormalised inverse 3-D DFT of the half grid to the real field.
* ``gather``    -- interpolation of the field at the pixel positions c + r n (Sec. II D 1,
                   sampling onto the sphere): trilinear, or Keys cubic convolution.
* ``simulate``  -- the three stages chained: the map the simulator must produce.
* ``inversion`` -- the C_l -> P_inf linear programme (Sec. II B) and the closed forms that
                   tie C_l, xi and P together (eqs. harmonics, rtheta, xiinfpinf).
* ``sht``       -- a Gauss-Legendre spherical-harmonic C_l estimator for full shells.
* ``mlp``       -- FP64 forward/backward of the spectrum surrogate network.
"""
