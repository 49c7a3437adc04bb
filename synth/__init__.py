"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and
the benchmark.

This package only draws random sparse matrices, orthonormal factors and update
streams with the shapes and value distributions of the paper's workloads
(Section 4 "Datasets"; Appendix "Experiments on Synthetic Matrices").  It holds
none of the update method's arithmetic: no projection, orthogonalisation or
SVD of an update lives here.  Orthonormal starting factors are produced by a
QR of a Gaussian matrix (a random-matrix recipe, not a step of the method), and
the initial truncated SVD of a workload's starting matrix is a randomized
range finder — the paper leaves the initial factorisation unspecified and
only the result ``A~ = U S V^T`` matters for every comparison downstream.
"""
from .sparse import (CSR, bernoulli_uniform, chung_lu_weights, chung_lu_graph,
                     zipf_ratings, lognormal_values, random_orthonormal,
                     synthetic_factors, randomized_init)
from .workloads import (seed_children, config1_rows, config2_graph, config2_initial_matrix,
                        config3_ratings, config4_weights, config4_weights_r2, config5_stream,
                        materialise_matrix, materialise_request, small_case)

__all__ = [
    "CSR", "bernoulli_uniform", "chung_lu_weights", "chung_lu_graph",
    "zipf_ratings", "lognormal_values", "random_orthonormal",
    "synthetic_factors", "randomized_init", "seed_children", "config1_rows",
    "config2_graph", "config2_initial_matrix", "config3_ratings", "config4_weights_r2", "config4_weights", "config5_stream",
    "materialise_matrix", "materialise_request", "small_case",
]
