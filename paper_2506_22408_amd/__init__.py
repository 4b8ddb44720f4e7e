"""MI355X-native matchgate-shadow overlap estimator for QC-AFQMC.

Implements, as hand-written HIP kernels for gfx950 behind a C ABI
(``include/shadowov.h``), the classical post-processing hot path of
Zhao et al., arXiv:2506.22408: for every AFQMC walker Slater determinant
phi_w and every matchgate shadow (Q_s, b_s), the estimate of
<Psi_T|phi_w> from Pfaffians of the Majorana-basis matrices A(z) at the
interpolation nodes, reduced over shadows; and its first derivative.

Submodules: ``binding`` (ctypes binding of the built library; importing it
fails if the library is missing), ``workload`` (seeded synthetic inputs),
``build`` (hipcc build of the library).
"""
