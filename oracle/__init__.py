"""FP64 CPU oracle for altGDmin (test infrastructure only).

This package is the plain, slow, obviously correct reference that the GPU
library is checked against.  It is test infrastructure: only the test suite,
the smoke check and the benchmark's CPU-baseline leg may import it.  The
product path never calls it, and it shares no code with the HIP library
(neither imports the other; the only common module is the seeded input
generator ``datagen``, which holds none of the method's arithmetic).

Everything is complex128.  The method is an iteration, so the oracle takes
the steps of the auto-altGDmin algorithm (Algorithm 2 of the paper) in the
paper's order and notation:

* ``operators``  -- the measurement operator A_k = [H_k F D_c]_c and the
  padded stacking of Sec. II-A, with an FFT backend and a dense-matrix
  backend built from the DFT definition;
* ``altgdmin``   -- truncation, scaled back-projection, spectral
  initialisation and the alternating loop (LS for b_k, gradient, step size,
  GD step, QR, exit rule), literally, frame by frame and coil by coil;
* ``variants``   -- FP64 restatements of the algebra the GPU path uses
  (hybrid ky/x form, folded gradient, Gram + Cholesky LS), checked against
  the literal forms;
* ``metrics``    -- subspace distance, NMSE and the scale-invariant N-S-MSE;
* ``mri``        -- the steps around the loop (Algorithm 1: the mean image by
  CGLS and the residuals; Algorithm 2's automatic rank; Algorithm 3: MEC-1
  and MEC-2) and the tracking drivers of Sec. IV (Algorithms 4 and 5).

Each function cites the passage it follows.  Readings chosen where the paper
is silent or ambiguous are stated at the function that applies them.
"""
from . import operators, altgdmin, variants, metrics, mri  # noqa: F401
