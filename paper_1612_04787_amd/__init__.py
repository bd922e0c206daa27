"""MI355X-native signal-whitened FFT window matching (SWiFT-IR hot path).

The compute lives in libswift.so (HIP for gfx950, C ABI in include/swift.h);
this package is its thin Python binding.
"""
from .swift import (  # noqa: F401
    FLAG_CONCURRENT_SIZES,
    FLAG_JAC_TRANSLATION,
    FLAG_PEARSON,
    ST_NEAR_TIE,
    ST_DEGENERATE,
    ST_CLAMPED,
    SIZES,
    Swift,
    SwiftError,
    SwiftMatchFn,
    theta6_to_theta8,
    load_library,
    make_params,
    parse_records,
)
