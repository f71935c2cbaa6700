"""MI355X-native sketched plug-and-play fan-beam CT (arXiv:2203.07308).

Modules:
  fbpnp  - ctypes binding of the HIP library libfbpnp.so (include/fbpnp.h)
  synth  - seeded synthetic inputs (phantoms, noise draws, view subsets, workloads)
  build  - compiles libfbpnp.so for gfx950 with hipcc
"""
