"""MI355X (gfx950) D3Q7 reactive-diffusion lattice Boltzmann solver for
catalyst-layer structures (Chen et al., arXiv 1410.1914), behind the C ABI of
``include/lbm.h``.  ``lbm`` is the ctypes binding; ``build`` compiles the HIP
libraries in-tree."""
