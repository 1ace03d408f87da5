"""MI355X (gfx950) stochastic local-Newton 3DGS training step (arxiv 2501.13975).

The compute path is the HIP library libgsn.so behind the C ABI in
include/gsn.h; ``gsn`` is its ctypes binding and ``train`` the sweep driver.
"""
