"""FP64 CPU oracle for the particle-mesh hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, links or
runs this code; only ``tests/``, the build entry's smoke check and the bench's
CPU-baseline leg may use it.  It shares no code with the HIP path: every
operation here is written out again from the paper's definitions and from
textbook cosmology, in plain PyTorch CPU float64 ops (``torch.fft`` serves as
the DFT primitive; autograd serves as the reference vector-Jacobian product).

Module map (paper passages in each function's docstring):
  cosmology   -- background, linear growth, kick/drift integrals, P(k) models
  cic         -- cloud-in-cell counting density and interpolation, the wrap rule
  fourier     -- DFT conventions, wavenumber grids, brute-force DFT for pins
  solve       -- Newtonian Poisson solve and the Poisson-gauge weak-field solve
  ics         -- Zel'dovich initial conditions (Newtonian and Poisson-gauge sets)
  integrate   -- kick-drift-kick leapfrog loop
  combine     -- GR-minus-Newton displacement and its addition to a fine run
  estimators  -- power spectrum and FFT bispectrum estimators
  adjoint     -- loss on P(k) and its reference gradient
  planar      -- the Newtonian cycle of a plane-parallel lattice reduced to one
                 dimension (expected values of full-size runs, sampled per particle)

Parity status: every function is pinned by a closed form, an invariant, a
brute-force evaluation or a statistical expectation in ``tests/test_oracle_*``,
except the Eisenstein-Hu no-wiggle transfer-function constants, which are
recalled from the published fitting formula and only pinned by their limits
("parity unpinned" for the constants themselves).
"""
from . import cosmology, cic, fourier, solve, ics, integrate, combine, estimators, adjoint, planar  # noqa: F401
