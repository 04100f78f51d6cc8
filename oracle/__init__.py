"""FP64 CPU oracle for the Fourier-accelerated volume integral method
(Frerot, Bonnet, Molinari, Anciaux, arXiv 1811.11558).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, headers, tables or constant generators); the two meet
only through the seeded input generators in ``synth/``, which hold none of
the method's arithmetic.

The oracle is written to be read against the paper, not to be fast:

* ``elastic``      -- isotropic constants, Voigt/tensor helpers (Sec. 1).
* ``fundamental``  -- partial-Fourier Kelvin (Table 1), Boussinesq-Cerruti
                      (B00, B10), the gradient recurrence and the jump term
                      (Sec. 2.2-2.3).
* ``depth``        -- exact P1 element integrals of g0/g1 (Sec. 3.2,
                      eqns int_g0 / int_g1), no cutoff; dense element-pair
                      matrices, and the same sums by depth recurrences
                      (the fast mode, pinned to the dense one).
* ``operators``    -- mindlin_apply / boussinesq_apply: DFT per layer
                      (Sec. 3.1), dense O(N3^2) depth sums per mode
                      (eqn full_discrete_convolution, eqn 2gradient),
                      Mindlin superposition (eqn mindlin_B_U), k = 0 and
                      Nyquist readings.
* ``plasticity``   -- J2 radial return (Sec. 4.1) and the DF-SANE fixed
                      point on the incremental residual (Sec. 4.2-4.3).
* ``contact``      -- Polonsky-Keer projected CG on the Kalker dual with
                      the total-load constraint (Sec. 5.1).
* ``coupling``     -- Algorithm 1 (Sec. 5.2), and Newton's method with the
                      consistent tangent (the alternative of Sec. 4.3).
* ``friction``     -- tangential (Coulomb, partial-slip) contact under a
                      given pressure, the friction Sec. 5.1 says can be
                      added: projected gradient with momentum on the
                      complementary energy; the normal-tangential coupling
                      through the Boussinesq-Cerruti cross terms.

Every function is pinned by ``tests/test_oracle_*.py`` against things the
oracle does not compute itself: an independent high-precision state-space
ODE solve, textbook closed forms, brute-force DFT sums, reciprocity and
invariances.  Functions without such a pin say "parity unpinned".
"""
