"""MI355X-native (gfx950) per-object NeRF training step of PRENOM
(arXiv 2503.01582, Sec. III-B): prior-based probabilistic ray sampling,
hash-grid encoding, MLP on the matrix cores, volume rendering, losses, the
hand-written backward and Adam, as HIP kernels behind the C ABI of
include/prenom.h.  The HIP library (libprenom.so) must be built; nothing here
falls back to another implementation."""

from ._lib import FLAG_ESCAPED, FLAG_MISS, FLAG_UNIFORM, LIB_PATH, PrenomError  # noqa: F401

__all__ = ["FLAG_ESCAPED", "FLAG_MISS", "FLAG_UNIFORM", "LIB_PATH", "PrenomError"]
