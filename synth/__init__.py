"""Seeded synthetic inputs shared by the oracle and the GPU library.

This package only *generates inputs*: data graphs in CSR form and small
pattern graphs.  It holds none of the estimator's arithmetic (no proposal
weights, no random draws of the sampler, no pattern analysis), so that the
oracle and the HIP path can both consume the same inputs while sharing no
code of the method itself.

The paper evaluates on real graphs (LiveJournal, UK-2002, Twitter,
Friendster, GSH-2015; Table 1 of the evaluation section) which are not
available here; the generators below stand in for them with the same
scale-free degree skew (Chung-Lu power law, R-MAT).
"""

from .graphs import CSR, chung_lu, rmat, csr_from_edges, tiny_graph, complete_graph, ring_graph, star_graph, complete_bipartite
from .patterns import Pattern, named_pattern, NAMED_PATTERNS, random_pattern_set

__all__ = [
    "CSR", "chung_lu", "rmat", "csr_from_edges", "tiny_graph", "complete_graph",
    "ring_graph", "star_graph", "complete_bipartite",
    "Pattern", "named_pattern", "NAMED_PATTERNS", "random_pattern_set",
]
