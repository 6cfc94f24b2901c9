"""FP64 CPU oracle for the local-line-of-sight power-spectrum multipole estimator.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this package.  The
GPU product path never calls it, and this package never imports the GPU package.

Everything is plain numpy / scipy in float64, written from the paper
(Hand, Li, Slepian & Seljak 2017, arXiv:1704.02357):

* ``legendre``  - Legendre polynomials, wedge means Lbar (Sec. 2.2, eq. Lbar).
* ``ylm``       - real spherical harmonics (Sec. 2.1, eq. real-Ylm).
* ``catalog``   - FKP scalars alpha, I and the shot noise S (Sec. 2.1, eq. FKP-density).
* ``mesh``      - mass assignment, interlacing, compensation (Sec. 2.3).
* ``estimator`` - O3: the FFT estimator, eq. Pell-ours / eq. Fell on the mesh.
* ``direct``    - O1: brute-force Legendre-weighted DFT; O2: galaxy-direct Yamamoto sums
                  (eq. Pell-yama).
* ``cartesian`` - O4: the Cartesian decomposition with (l+1)(l+2)/2 transforms per l.
* ``wedges``    - eq. wedge-est with eq. Lbar.
* ``global_los``- P(k, mu) and multipoles for one fixed line of sight.
* ``systematics`` - delta_l (eq. delta-ell), response R(mu) (eq. response) and the
                  non-uniform mu edges (eq. nonuniform-bins).

Conventions (points the paper leaves open, read the same way by the GPU library):
node c of an N^3 mesh sits at o + c H (H = L/N); forward DFT uses exp(-2 pi i n.c/N);
integer frequencies n_a lie in [-N/2, N/2); modes with any n_a = -N/2 (the Nyquist
planes) are zero in the combined field and belong to no k bin; k = 0 belongs to no bin.
"""
