"""MI355X-native Brownian hard-disk time step (arXiv:1703.02484).

The simulation runs in hand-written HIP kernels behind the C-ABI declared in
``include/bd.h``; this package only marshals arguments to that library.
"""
