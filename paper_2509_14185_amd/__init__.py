"""MI355X (gfx950) damped Gauss-Newton step for physics-informed profile networks.

- csrc/: hand-written HIP kernels and the C ABI (include/gn.h), built into
  libgn.so by build.py.
- gn: ctypes binding (argument marshalling only) and the differentiable
  residual (torch.autograd.Function).

Import `paper_2509_14185_amd.gn` explicitly; importing the package itself
loads nothing.
"""
