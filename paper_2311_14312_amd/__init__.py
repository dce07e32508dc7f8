"""MI355X-native diffusion curves: hybrid BEM/BIEM densities, FMM render.

The compute path lives in libdcfmm.so (HIP, gfx950); ``dcfmm`` is its
Python binding.  Import it explicitly: ``from paper_2311_14312_amd import
dcfmm``.
"""
