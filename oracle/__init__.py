"""Oracle for the periodic KIFMM evaluation pass -- TEST INFRASTRUCTURE ONLY.

A plain, slow, double-precision CPU implementation written from the paper:
  * ``periodic``: the periodic sums themselves (lattice sums, Ewald sums), the
    definition the method approximates;
  * ``kifmm``: a plain periodic kernel-independent FMM with the same
    discretisation as the product (surfaces, tree, lists, operators);
  * ``tree``: the Morton-sorted adaptive octree and periodic U/V/W/X lists.
Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
it.  It shares no code with the GPU library.
"""
from . import kernels, tree, periodic, kifmm  # noqa: F401
from ._native import build  # noqa: F401
