"""MI355X-native K-S change-point detection (the evaluation hot path of MT4G, arXiv 2511.05958).

The public surface is the C ABI of ``include/ks.h`` (``libks.so``) and this
package's ctypes binding of it with the same names. ``synth`` is the seeded
input generator.
"""

from ._binding import *  # noqa: F401,F403
from ._binding import KsError, lib  # noqa: F401
