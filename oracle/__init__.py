"""Plain FP64 CPU oracle for the TV-Stokes dual iterations and their
overlapping Schwarz decomposition.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, headers, helpers or tables); the only module both sides
use is ``synth`` (seeded synthetic images, none of the method's arithmetic).

Everything here is written from the paper (Langer, Runft, Rahman, Tai, Wu,
"Functional Analysis and Parallel Domain Decomposition for the TV-Stokes
Model", arXiv 2602.17494) in plain numpy/scipy, float64, with no blocking,
fusion or reordering beyond what the paper's definitions state:

* ``operators``  -- Section 4.1 (Notations): finite differences, Neumann
  differences (eq. def:backdiffNeumann), gradient / divergence (eqs.
  defGradDis, defDivDis), the DCT matrix (eq. form:DCTmat), the inverse
  Laplacian (eqs. form:DiscInvLapl, form:DiscInvLaplTild) and the projection
  onto divergence-free fields (eq. formula:PKh).
* ``solvers``    -- Section 4.2: the discrete dual problems (eqs. tfsdualdis,
  ir2dualdis, ir1dualdis), Algorithm 1 (alg:chambTfs), Chambolle's iteration
  for the ROF dual of IRV2, the IRV2 potential g, the primal maps, energies,
  stopping residuals and duality gaps.
* ``schwarz``    -- Section 6: subdomains, the partition of unity, Algorithm 2
  (alg:disalgsubsp), the generic inner loop Algorithm 3 (alg:tfsparinner),
  the TFS inner loop with global arrays Algorithm 4 (alg:tfsparinnertfs) and
  its localized form Algorithm 5 (alg:tfsparinnertfsloc).
* ``quality``    -- Section 5.2: PSNR, MSSIM and the tangent-field measure
  Perf used to pick the TFS weight.

Readings of passages the paper leaves open are listed in each function's
docstring.  Pins (independent checks) live in ``tests/test_oracle_*.py``.
"""
