"""MI355X (gfx950) stabilizer-tableau simulator core.

The hot path (tableau evolution under fused gate passes and CHP Z-measurement)
runs in hand-written HIP kernels behind the C ABI in include/sq.h; this
package is the Python binding (``binding``) and the build step (``build``).
"""
from .binding import (  # noqa: F401
    Program, SqError, Tableau, Tuning, batch_sample, bytes_required, load, ops_array, parse_qasm, version,
    words_to_bits,
    I, H, S, SDG, X, Y, Z, CX, CZ, CY, SWAP, ISWAP, MEASURE, COLLAPSE_ROWSUM, COLLAPSE_INJECT,
    LAYOUT_COLUMNS, LAYOUT_ROWS,
)
