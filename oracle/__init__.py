"""Plain FP64 CPU oracle for one MPPI iteration on a jump-diffusion process.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
executes anything in this package; only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark do.  The oracle shares no code with the
HIP library: it implements the counter-based generator, the noise transform,
the dynamics, the costs, the weights and the update on its own, from the paper
(Wang, Williams, Theodorou, "Information Theoretic Model Predictive Control on
Jump Diffusion Processes", arXiv 1807.06108) and from the published definition
of Philox (Salmon et al., "Parallel random numbers: as easy as 1, 2, 3", SC'11).

Modules
  philox   - Philox4x32-10 / Philox4x64-10 block function (SC'11, Sec. 3-4).
  noise    - words -> uniforms -> Box-Muller normals, jump counts by inversion
             of the Poisson / zero-one law (Sec. IV-B, Algorithm 1 jump timer).
  models   - discrete-time dynamics (explicit Euler of eqs. (2),(4)) and the
             state costs q, phi for the three systems.
  mppi     - the iteration itself: modified path cost (eqs. (34)-(35)),
             weights (eq. (37) with the min-shift), update (eqs. (36)/(49)),
             receding-horizon shift (Algorithm 1, Sec. V); plus the separately
             written reference forms used as pins (Gaussian-only MPPI,
             brute-force argmin).

Parity status per function is listed in each module header.  Every function
here is pinned by a CPU test (tests/test_oracle_*.py) except where a header
says "parity unpinned".
"""

from . import philox, noise, models, mppi  # noqa: F401
