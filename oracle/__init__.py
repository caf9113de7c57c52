"""CPU oracle for the Fourier-slice Radon NUFFT (test infrastructure only).

This package is TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it. The product path
(the HIP library and its Python binding) never imports, links or calls it, and
it shares no code with that path: the only common module is ``radon_inputs``,
which generates seeded inputs and contains none of the method's arithmetic.

Paper: Maia et al., *Compressive Phase Contrast Tomography* (LBNL-3899E),
section "fast radon transform". The transform is a 2D FFT on a regular
grid, then interpolation of that transform onto a polar grid ("gridding", a
non-uniform FFT that convolves with a kernel evaluated at regular positions),
then 1D inverse FFTs along each radial line. The inverse (adjoint) runs the
same steps reversed ("gridding and inverse gridding", abstract). The paper
fixes none of the numerical details; the readings taken here are:

  * O-exact (``exact``): the discrete Fourier-slice Radon transform with exact
    (non-uniform DFT) interpolation, and its exact transpose;
  * O-grid (``grid``): FP64 gridding with a Kaiser-Bessel kernel of width W,
    oversampling sigma, Beatty's shape parameter, analytic deapodization;
  * ``binning``: uniform-tile sample keys and their stable sort.

Every function is plain FP64 NumPy/SciPy written for readability, not speed.
Pins for each function live in ``tests/test_oracle_*.py``.
"""
