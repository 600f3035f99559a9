"""MI355X-native NFFT-boosted Sinkhorn: the hot path of entropy-regularized
optimal transport between point clouds (Lakshmanan, Pichler, Potts,
arXiv 2201.07524) as hand-written HIP kernels for gfx950 behind a C ABI.

Importing the package is cheap; the binding in ``nfs`` loads the compiled
library ``lib/libnfs.so`` on first use and raises if it is missing.
"""
__all__ = ["nfs", "workloads"]
