"""MI355X H^2 VIE hot path: Python binding of libh2vie.so.

PyTorch supplies device memory and streams; every step of the product and
the solver runs in the library's HIP kernels.  Importing this package does
not need a GPU; constructing an operator does, and fails loudly when the
library is missing.
"""

from ._lib import H2Error, load  # noqa: F401
from .api import H2Operator, H2Group, GmresResult, LeafMLP, leaf_neighbors  # noqa: F401
