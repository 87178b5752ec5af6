"""MI355X-native calibrated O(N log N) FFT-correlator (Gorthi, Parsons &
Dillon 2020): HIP kernels for gfx950 behind the C-ABI of include/rrcal.h,
with a thin PyTorch/ctypes binding."""
from ._lib import (RRCError, load_library, EXPORTS, LIB_PATH, RRC_C64, RRC_CI4)  # noqa: F401
from .api import (Plan, Batch, ChiSq, chisq, select_subset, degeneracy_count, default_opts,  # noqa: F401
                  wall_clock_hz, gain_variance, lowcad_schedule, LowCadence, hex_mask, select_subset_masked,
                  degeneracy_count_masked, chisq_full)

__all__ = ["Plan", "Batch", "ChiSq", "chisq", "select_subset", "degeneracy_count", "default_opts",
           "wall_clock_hz", "gain_variance", "lowcad_schedule", "LowCadence", "hex_mask",
           "select_subset_masked", "degeneracy_count_masked", "chisq_full",
           "load_library", "RRCError", "EXPORTS", "LIB_PATH"]
