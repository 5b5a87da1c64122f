"""ENUF hot path for AMD MI355X: HIP kernels behind a C ABI (libenuf.so).

Submodules:
  enuf    ctypes binding of include/enuf.h (Enuf context, EnufEnergy autograd)
  inputs  seeded synthetic workloads
  build   in-tree hipcc build of libenuf.so
Nothing is imported eagerly, so the input generators load without torch.
"""
