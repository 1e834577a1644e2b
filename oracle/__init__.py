"""CPU FP64 oracle for the SLAR / LoMaC time step -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, deliberately unoptimised restatement of what
the paper computes, written in NumPy double precision.  It exists to check
the GPU library, never to serve it:

  * only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
    of ``bench.py`` may import it;
  * it shares no code with the HIP path (no kernels, headers, helpers,
    tables or constant generators) and imports nothing from the product
    package; the only thing both sides consume is ``slar_inputs`` (seeded
    synthetic inputs, no arithmetic of the method);
  * every function cites the passage of the paper it restates.

Parity status per module (see each module header):
  grid        pinned (closed-form weights, printed grid values)
  feet        pinned (exact shifts, closed-form flows)
  ht          pinned (brute-force tensor-product interpolation)
  cross       pinned (exact low-rank recovery, SVD error bound, brute force);
              the pivot sequence itself is a free heuristic choice
  spectral    pinned (closed-form Poisson solution, discrete identities)
  lomac       pinned (orthogonality, moment preservation, idempotence)
  macro       pinned (conservation identities, Newton residual)
  cnn         pinned (central finite differences)
  step        pinned end to end (Landau damping rate, amplification factor)
"""
