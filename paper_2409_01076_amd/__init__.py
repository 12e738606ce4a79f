"""MI355X (gfx950) D2Q9 lattice Boltzmann library for the single MRT-featured
collision (SmrtLBM) and the SRT collision (Zhou, arXiv:2409.01076).

``paper_2409_01076_amd.smrt`` is the binding of the HIP library
(``libsmrt.so``, C ABI in ``include/smrt.h``); ``paper_2409_01076_amd.inputs``
draws seeded synthetic initial fields.  Importing the package loads nothing.
"""
__all__ = ["smrt", "inputs", "build"]
