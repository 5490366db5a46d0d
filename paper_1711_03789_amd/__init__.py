"""MI355X-native one-level Schwarz (AS / RAS / ORAS) preconditioned GMRES for the lowest-order
Nedelec discretisation of curl curl E - (k^2 + i xi) E = F (arXiv:1711.03789).

The solver is the C-ABI library libmx.so (include/mx.h); `mx` is its ctypes binding.
"""
from . import mx  # noqa: F401
