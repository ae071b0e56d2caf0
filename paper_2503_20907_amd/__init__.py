"""MI355X-native x-ray transform of tensor-product B-spline images.

The operator (forward projection over arbitrary lines and its exact adjoint)
runs in the HIP library ``libxrt.so`` built from ``csrc/`` for gfx950; this
package only exposes it to Python (``_lib``: ctypes, ``ops``: torch tensors).
Importing ``ops`` loads torch first so that the library binds to the HIP
runtime torch already uses.
"""
__all__ = ["ops", "build"]
__version__ = "0.1.0"
