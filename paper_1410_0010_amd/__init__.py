"""APM nested-grid gravity solve for AMD MI355X (gfx950).

The hot path (TSC deposit, FFT convolution with the optimal influence function,
Fourier-space differencing, level composition, TSC interpolation) runs in the HIP
library libapm.so behind the C ABI of include/apm.h; this package is its thin
Python binding.  The library is loaded on first use (Plan, Context, lib()); a
missing or stale library raises ImportError there.  There is no fallback path.
"""

from ._apm import APMError, lib  # noqa: F401
from .solver import Context, Plan  # noqa: F401

__all__ = ["Plan", "Context", "APMError", "lib"]
