"""MI355X (gfx950) lattice-BGK lid-driven cavity library (D2Q9 cavities and
batches, the D3Q19 box, the learned warm start).

The HIP library ``liblbm.so`` (C ABI in include/lbm.h) does all the work;
``paper_2211_05009_amd.lbm`` is its ctypes binding.
"""
from .lbm import (Batch, Cavity, Cube, Surrogate, LbmError, LBM_F32_SHIFTED, LBM_F64,  # noqa: F401
                  LBM_OPT_GRAPH_STEPS, LBM_OPT_NUM_VARIANTS, LBM_OPT_STEP_VARIANT,
                  LBM_OPT_USE_GRAPH)

__all__ = ["Batch", "Cavity", "Cube", "Surrogate", "LbmError", "LBM_F64", "LBM_F32_SHIFTED",
           "LBM_OPT_USE_GRAPH", "LBM_OPT_STEP_VARIANT", "LBM_OPT_NUM_VARIANTS",
           "LBM_OPT_GRAPH_STEPS"]
