"""CPU FP64 oracle (test infrastructure only; see ``spamm_oracle``)."""
from .spamm_oracle import *  # noqa: F401,F403
from .spamm_oracle import (TRUNCMUL, SPAMM, HYBRID, Tree, Truncation, Result,  # noqa: F401
                           build, build_from_blocks, truncate, truncate_elementwise,
                           kept_flat, kept_recursive, multiply, exact_product,
                           tie_triples, spamm_elementwise, morton_key, grid_size,
                           pyramid, count_candidates, with_leaves_dropped)
