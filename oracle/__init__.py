"""Oracle: plain, slow, obviously-correct CPU reference for the batched
arithmetic-circuit (AC) evaluation path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import or run anything here.  The
product path (``paper_2103_17226_amd``) never imports it, and this package
never imports the product path; the two share only the seeded input
generators in ``workloads``.

Everything is complex128 / float64.  The pieces, each with the passage it
follows:

* ``sim``      -- state-vector, Kraus-branch state-vector and density-matrix
                  simulators (Sec. 2.1 state vectors and unitaries, Sec. 2.2
                  density matrices and Kraus channels, Table "noise models").
                  A branch amplitude f(x, k) is the amplitude the AC root
                  yields for output evidence x and noise-event evidence k
                  (Sec. 3.3.1, Table "inference"); P(x) = sum_k |f(x,k)|^2 is
                  the density-matrix diagonal (Sec. 3.3.1, the two density
                  matrix components summed to the final rho).
* ``grad``     -- exact derivatives of amplitudes by the product rule, the
                  parameter-shift rule for expected cost, and central finite
                  differences (gradients via model counting are listed among
                  the queries in Sec. 5).
* ``gibbs``    -- the counter-based SplitMix64 generator, single-site Gibbs
                  conditionals, a reference systematic-scan chain and the
                  exact t-sweep distribution on tiny spaces (Sec. 3.3.2).
* ``stats``    -- Pearson chi-square with pooling, KL divergence (Sec. 3.3.3).
* ``pathsum``  -- brute-force Feynman path sum for noise-free QAOA p=1
                  (Sec. 3.2.1: each model of the CNF is one Feynman path and
                  their weighted count is the amplitude), in plain C.
"""
