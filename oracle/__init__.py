"""FP64 CPU oracle for the TNSLQ logarithmic-negativity hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path; both take their inputs from ``tnslq_inputs``.

What it computes (Gray, "Fast Computation of Many-Body Entanglement"):

* ``exact``    -- the plain definition: regroup psi into (A, B, C), form
                  rho_AB, partially transpose B, diagonalise, and take
                  log2 of the trace norm (Sec. II Eq. 1, Sec. V).  Also the
                  explicit and the lazily contracted matvec of Eq. 4.
* ``probes``   -- the complex-Rademacher probe law drawn from SplitMix64,
                  the counter-based generator both sides implement.
* ``slq``      -- stochastic Lanczos quadrature in the order of Algorithm 1
                  (Sec. III): Hutchinson probes, Lanczos, Gauss quadrature of
                  |x| from the tridiagonal T_k, error on the mean (Sec. VIII).
* ``analytic`` -- the random-state closed form, Eq. 6 (Sec. VII.A).
* ``mlp``      -- FP64 forward/backward/Adam of the early-stopping surrogate,
                  rounding to BF16 at the points where the kernels do.
"""
