"""MI355X-native colour-gradient lattice Boltzmann step with the improved geometric wetting
boundary (arXiv:1707.00198): HIP kernels behind the C-ABI of include/lbmcg.h, a ctypes
binding (``lbm``), the Sec. III measures on top of the device reductions (``diagnostics``) and
synthetic workload generators (``workloads``)."""

__all__ = ["lbm", "diagnostics", "workloads", "build"]
