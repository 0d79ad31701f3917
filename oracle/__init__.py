"""Plain FP64 CPU oracle for the adaptive sketching-based solvers of Lacotte & Pilanci,
"Fast Convex Quadratic Optimization Solvers with Adaptive Sketching-based Preconditioners"
(arXiv 2104.14101).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code, constants or helpers with the HIP library; the only
thing both sides consume is the seeded input generator in ``synth/`` (which holds none of the
method's arithmetic) and the published definition of the Philox4x64-10 counter-based
generator, which each side implements on its own.

Modules
  philox     Philox4x64-10 (Salmon et al., SC'11) and the random streams the method draws.
  sketch     SRHT (Sec. 2.1 and the SRHT proof section) and Gaussian embeddings (Sec. 2.1).
  factor     cached factorisation of H_S: Cholesky of H_S when m >= d, Woodbury form when
             m < d (Sec. 4.1, "Sketching and factorization costs").
  solvers    adaptive PCG (Algorithm 2), adaptive IHS (Algorithm 1 with the IHS update,
             Theorem "rate IHS"), the improvement test, stop rules, matrix variables.
  reference  x*_ref by direct Cholesky + extended-precision iterative refinement; effective
             dimension d_e (Sec. 1.1, Notations).
  adjoint    dense FP64 gradients of a loss of x* w.r.t. b, A and log(nu).

Parity status of each function is stated in its docstring; functions without an
independent pin say "parity unpinned".
"""
