"""MI355X-native damped Chebyshev wave-packet propagation (arXiv 2412.10167 hot path).

The compute path is the HIP library libtdwp.so (C ABI in include/tdwp.h);
`tdwp` is its thin ctypes binding.
"""
from .tdwp import (Plan, TdwpError, library_path, load_library,  # noqa: F401
                   PRECISIONS, EXPORTED_SYMBOLS, jshift, jshift_interpolate,
                   cumulative_probability, cross_section, fit_jshift_b, energy_content,
                   photo_cross_section)
