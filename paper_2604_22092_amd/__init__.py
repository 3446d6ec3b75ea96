"""MI355X (gfx950) renewal tau-leap SEIR step of FlashSpread (arXiv 2604.22092).

The step runs in hand-written HIP kernels inside ``libflashspread.so``; this
package is the thin Python binding of its C ABI (``include/fs.h``).  Importing
the package does not load the library; the first call does, and raises if it
is not built.
"""
from ._capi import (FS_DIST_ERLANG, FS_DIST_EXP, FS_DIST_LOGNORMAL, FS_DIST_WEIBULL, FS_E,
                    FS_I, FS_R, FS_S, FS_STORAGE_COMPACT, FS_STORAGE_FP32, EXPORTS, FsError,
                    Graph, LIB_PATH, Sim, VARIANT_AUTO, VARIANT_RESIDENT, VARIANT_STREAM, fs_counts, fs_eval_hazard, fs_eval_philox,
                    fs_get_rates, fs_get_state, fs_graph_create, fs_graph_destroy,
                    fs_graph_get_info, fs_history, fs_set_state, fs_sim_create,
                    fs_sim_destroy, fs_sim_get_bins, fs_sim_seed, fs_sim_set_bins, fs_sim_tune, fs_step, fs_step_index, fs_sync, fs_version,
                    lib, make_dist)

__all__ = [n for n in dir() if not n.startswith("_")]
