"""FP64 CPU oracle for BOAC candidate evaluation — TEST INFRASTRUCTURE ONLY.

A plain, slow, single-threaded NumPy/SciPy implementation of what the GPU path computes, written from
the paper (Eqs. 1-5, the MLEM step of BOAC, the simulation study) under the readings stated in each
module's header. It shares no code with the HIP library and never imports it. Only the test suite,
the smoke check and the bench's CPU-baseline leg may import it; the product path must not.

Modules:
  geometry   scanner geometry, bilinear sampling matrix W            (Eqs. 1-2)
  head       Legendre outline, partial-volume attenuation map         (Eqs. 3-4)
  projector  attenuation scan, attenuated projector, exact transpose  (Eqs. 1-2)
  mlem       MLEM iterations, Poisson negative log-likelihood         (Eq. 5, BOAC step 3)
  adjoint    exact reverse-mode gradient of J wrt (c_0..c_5, mu_b, mu_c) and dR, the envelope
             gradient (reconstruction held fixed), finite differences
  phantom    synthetic phantom and noisy sinogram                     (simulation study)
  bo         GP surrogate, expected improvement, chaotic search       (Eqs. 7-10, BOAC steps 4-6)
  metrics    SSIM, CNR, PSNR of the simulation study                  (Table I)

Pins: every function is checked by tests/test_oracle_*.py against closed forms, exact special cases,
library routines and brute force. The comparison of BOAC with the paper's own Table I is
"parity unpinned" (the paper's phantoms are not published).
"""
from .geometry import Geometry, angles, sampling_matrix, sample_image, sample_image_transpose  # noqa: F401
from .head import coverage_fractions, head_radius, legendre_all, rasterize_mu, rasterize_mu_adjoint  # noqa: F401
from .projector import attenuation, backproject, line_integrals, project, sensitivity  # noqa: F401
from .mlem import evaluate, mlem, neg_log_likelihood  # noqa: F401
from .adjoint import (central_difference, envelope_objective, objective_and_envelope_grad,  # noqa: F401
                      objective_and_grad)
