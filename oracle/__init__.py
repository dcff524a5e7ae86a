"""CPU oracle for colored peeling (test infrastructure only).

Plain, slow, FP64 reference of what the GPU path computes, written from
Levitt & Martinsson, "Randomized compression of rank-structured matrices
accelerated with graph coloring" (arXiv 2205.03406).  Only ``tests/``, the
smoke check and the benchmark's CPU-baseline leg may import it; the product
library never does, and the two share no code.

* ``comb.c`` (plain C, built with gcc): tree, lists, constraint graphs, DSatur.
* ``numeric.py`` (numpy/scipy, FP64): counter-based Gaussian test matrices,
  the dense kernel black box, compression (alg:h1_pseudocode with the
  per-pair recovery of alg:compress_double_random), hmatvec, error measures.
* ``uniform.py``: uniform H^1 compression (per-box bases, two stages).
* ``product.py``: compressed operators and their products as black boxes.
* ``h2.py``: H^2 compression (nested bases) and its upward / downward apply.
"""
from .comb import OTree, dsatur, build as build_comb  # noqa: F401
from .numeric import (  # noqa: F401
    philox4x32_10, gaussian_block, test_matrix, leaf_test_matrix,
    KernelBlackBox, DenseBlackBox, CountingBlackBox, compress, HMatrix,
    rel_fro_error_dense, probe_error, kernel_matrix,
)
from .uniform import (  # noqa: F401
    UniformGraph, uniform_test_matrix, compress_uniform, uniform_floats,
)
from .product import HMatrixBlackBox, ProductBlackBox, assemble  # noqa: F401
from .h2 import H2Matrix, compress_h2, augment_gaussian, svd_basis  # noqa: F401
