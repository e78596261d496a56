"""CPU oracle for the brickwall Hilbert-Schmidt cost, gradient and HVP.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package; only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark use it.  It shares no code with the
HIP library (no kernels, headers, tables or helpers); the two meet only in
the seeded inputs drawn by `paper_2604_20384_amd.inputs`.

Everything is plain numpy in complex128 / float64, written from the paper
(arXiv 2604.20384, "Hessian-vector products for tensor networks via
recursive tangent-state propagation"):

* `circuit`  - brickwall layout, gate application, dense unitaries,
               product states (Sec. III, Sec. IV).
* `dense`    - the definition by substitution: overlaps, environments
               (Eq. environment) and their directional derivatives
               (one gate replaced by a unit matrix, another by its
               variation, Sec. III "HVP via recursive tangent-state
               propagation"), with no recursion.
* `sv`       - the statevector recursion of Alg. 1 (HVP kernel) with the
               environment accumulated before the backward update.
* `hs`       - the post-processing of Alg. 2 (cost, gradient, HVP of the
               Hilbert-Schmidt test) averaged over samples (Eq. costHS).
* `riem`     - projections onto the tangent space of U(4), Riemannian
               gradient and HVP (App. F), polar retraction, Pauli tangent
               basis (App. G).

Pins (tests/test_oracle_*.py) tie each function to something other than
itself: brute-force substitution against the recursion, central finite
differences, Hessian symmetry, real linearity, cut invariance, Euler
identities of the multilinear overlap, the optimum at G = U_ref, and
hand-derived two-qubit cases.  The retraction is one valid choice among
several (the paper does not fix one); it is pinned by its defining
properties only.
"""
