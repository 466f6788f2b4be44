"""CPU oracle (test infrastructure only).

Only the tests, the package smoke check and the benchmark's CPU-baseline leg
may import anything under this directory.  The product path never does, and
the oracle never imports the product package.
"""
from .reff_oracle import (GROUNDED, FLOATING, laplacian, grounded, diag,
                          pairs, edge_list, edge_list_fast, pad_nodes)
from . import selinv

__all__ = ["GROUNDED", "FLOATING", "laplacian", "grounded", "diag", "pairs",
           "edge_list", "edge_list_fast", "pad_nodes", "selinv"]
