"""MI355X-native hot path of the inertial-coupling (IC) method for
compressible Brownian particles (Balboa Usabiaga & Delgado-Buscalioni,
arXiv:1307.0702): one explicit step of the fluctuating isothermal
Navier-Stokes equations on a periodic staggered grid, coupled to particles
through the 3-point kernel, as HIP kernels for gfx950 behind a C ABI.

The binding lives in `paper_1307_0702_amd.ic` and loads `libic.so`; importing
this package does not load it, so the seeded input generators in
`paper_1307_0702_amd.workloads` can be used without a built library.
"""
