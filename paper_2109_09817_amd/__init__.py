"""MI355X-native exact Gaussian-process training with never-materialised kernel-matrix products.

The compute path is libgpkmm.so (HIP kernels for gfx950 behind the C ABI of
include/gpkmm.h); ``gp`` holds thin PyTorch-facing wrappers.  Importing the
package does not load the library; the first call does, and raises if the
library has not been built.
"""
__all__ = ["gp"]
