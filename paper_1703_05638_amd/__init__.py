"""lrpost: low-rank posterior covariance for the space-time heat-equation
inverse problem on MI355X.  The compute path lives in liblrpost.so (HIP for
gfx950, C-ABI in include/lrpost.h); `paper_1703_05638_amd.lrpost` is its
ctypes binding and `paper_1703_05638_amd.build` builds it."""
__all__ = ["lrpost", "build"]
