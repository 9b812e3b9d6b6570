"""MI355X-native DF-DSRG-PT2 virtual natural-orbital pass (arXiv 2312.07008).

The computation lives in libdfpt2.so (hand-written HIP for gfx950, C ABI in
include/dfpt2.h).  This package only loads it and marshals torch device
tensors into its entry points; there is no CPU fallback.
"""
from ._lib import (BF16_SLICED, FP8_SLICED, FP64, INT8_SLICED, DfptError, Opts, LIB_PATH, load,  # noqa: F401
                   TRUNC_CUMULATIVE, TRUNC_CUTOFF, TRUNC_FIXED, TRUNC_FRACTION)
from .api import (pairscreen_adam_step, pairscreen_build_mask, pairscreen_features,  # noqa: F401
                  pairscreen_mlp_backward, pairscreen_mlp_forward, pairscreen_num_params, pairscreen_targets,
                  pairscreen_train)
from .api import (add_active_particle_density, add_cumulant_singles_density, build_vv_density, build_vv_density_noalloc, eigh_sym, fno_truncate, fno_truncate_rule, naf_compress,  # noqa: F401
                  fno_truncate_workspace_size,
                  make_opts, pp_ladder, pp_ladder_workspace_size, profile_enable, profile_read,
                  pt2_correction_workspace_size,
                  pt2_energy_correction, upload_inputs,
                  workspace_size)
