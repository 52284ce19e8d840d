"""MI355X (gfx950) photometric bundle adjustment with proxy-template inverse
compositional Gauss-Newton: HIP kernels behind the C ABI of include/pba.h
(csrc/), built into libpba.so, and its ctypes binding (pba.py)."""
