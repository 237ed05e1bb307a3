"""Mass-consistent wind downscaling (Mandel et al.) on AMD Instinct MI355X.

The solver lives in libmcwind.so (HIP for gfx950, C ABI in include/mcwind.h);
``paper_2101_08453_amd.mcwind`` is its Python binding and
``paper_2101_08453_amd.inputs`` builds the synthetic workloads.  Nothing is
imported eagerly, so importing the package never loads the GPU library.
"""
