"""MI355X-native continuous-field DQMC sweep for the projected SO(5) model
(arXiv 2605.03700): HIP kernels for gfx950 behind the C ABI of include/cfqmc.h."""
from .cfqmc import CFQMC, Batch, Slmc, FP64, MIXED, MIXED_ALL, Q_BZ, Q_LIST, Q_PAPER, Q_RADIUS, Q_SPHERE, load  # noqa: F401
