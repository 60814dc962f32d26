"""FP64 CPU oracle for proximal-distance convex clustering.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously-correct
reference that the GPU path is checked against.  Only the test suite, the
package's smoke check and the benchmark's CPU-baseline leg may import it; the
product path (the HIP library and its Python binding) never does, and shares
no code with it.  The two meet only through the seeded input generators in
``gen``, which contain none of the method's arithmetic.

Modules
  prep      observed-column means, mean imputation, standardisation
  weights   k-nearest-neighbour Gaussian-kernel weights   (eq_weighting)
  graph     incidence matrix, degrees, connected components
  mm        the proximal-distance MM iteration and solver (eq_proxdist,
            first_surrogate, sqrt_root_majorization, second_surrogate, the U
            and V updates, block-descent projection, eq_missing_analog)
  certify   independent certificates: the convex objective (eq_lindsten), a
            dual solver with a duality-gap bound, brute force over partitions,
            and closed forms

Parity status per function is stated in each module's header.
"""
from . import prep, weights, graph, mm, certify  # noqa: F401
