"""MI355X-native FM-index engine: Occ8 over an interleaved 2-bit BWT with checkpoint
counts, exact and z-mismatch backward search, batching and serving (libfmocc)."""
from .fm import *  # noqa: F401,F403
