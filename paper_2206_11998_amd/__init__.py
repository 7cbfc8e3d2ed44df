"""MI355X (gfx950) implementation of the hot path of the Lagrangian particle
method (arXiv 2206.11998): neighbour search, GFD least-squares fits and the
blended upwind / Lax-Wendroff update, behind the C ABI of include/lp.h.

``paper_2206_11998_amd.lp`` is the Python binding of liblp.so;
``paper_2206_11998_amd.workloads`` builds seeded synthetic particle sets.
"""
__all__ = ["lp", "workloads", "build"]
