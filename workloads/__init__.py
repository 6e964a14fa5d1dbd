"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.  Nothing in this package performs any step of the multigrid
method: it produces box coordinates, boundary data and right-hand sides."""
from .configs import (Workload, c1, c2, c2_head_sequence, c3, c5, paper_setup, streamer_small, forest,
                      rhs_zero, DIRICHLET, NEUMANN)
from .octree import BoxList, uniform_boxes, refine_boxes_explicit, refine_by_score
from .transport import EMAX, synthetic_n2_table, constant_table

__all__ = ["Workload", "c1", "c2", "c2_head_sequence", "c3", "paper_setup", "c5", "streamer_small", "forest", "rhs_zero", "DIRICHLET", "NEUMANN",
           "BoxList", "uniform_boxes", "refine_boxes_explicit", "refine_by_score",
           "EMAX", "synthetic_n2_table", "constant_table"]
