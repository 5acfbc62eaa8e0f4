"""gfx950 (MI355X) 2D constrained Delaunay refinement: the gDP2d round loop of
Chen, Tan and Ong as HIP kernels behind a C ABI (include/gdp2d.h).

The binding lives in ``paper_2007_00324_amd.gdp2d``; importing the package
does not load the library.
"""
