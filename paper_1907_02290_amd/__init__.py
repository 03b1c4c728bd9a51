"""MI355X-native (gfx950, HIP) Barnes-Hut step with index interaction lists,
one multiwalk force launch and list reuse, after "Accelerated FDPS"
(Iwasawa et al. 2019).  The work happens in ``libnbody_hip.so``; this
package only binds it (``nbody``), builds it (``_build``), and sequences
its calls for the learned list refresh (``learn``) and the autotuner
(``tune``)."""
from .nbody import (Context, NbError, NB_MAKE_LIST, NB_MAKE_LIST_FOR_REUSE,
                    NB_REUSE_LIST, NB_REUSE_REFRESH, NB_REUSE_CHECK, NB_OK,
                    NB_ERR_INPUT, NB_ERR_OOM, NB_ERR_LIST, NB_ERR_STATE,
                    NB_ERR_HIP, NB_FLAG_TIMING, NB_FLAG_GRAPH,
                    NB_FLAG_REFRESH, NB_FLAG_PERSISTENT, NB_FLAG_COPIED_LISTS,
                    NB_FLAG_LEVEL_MOMENTS, MLP_NIN,
                    MLP_NPARAM, MLP_STATIC_MAX_ROWS, PHASES, load,
                    version, LIB_PATH)

__all__ = ["Context", "NbError", "NB_MAKE_LIST", "NB_MAKE_LIST_FOR_REUSE",
           "NB_REUSE_LIST", "NB_REUSE_REFRESH", "NB_REUSE_CHECK", "NB_OK",
           "NB_ERR_INPUT", "NB_ERR_OOM", "NB_ERR_LIST", "NB_ERR_STATE",
           "NB_ERR_HIP", "NB_FLAG_TIMING", "NB_FLAG_GRAPH", "NB_FLAG_REFRESH",
           "NB_FLAG_PERSISTENT", "NB_FLAG_COPIED_LISTS", "NB_FLAG_LEVEL_MOMENTS",
           "MLP_NIN", "MLP_NPARAM", "MLP_STATIC_MAX_ROWS", "PHASES", "load", "version", "LIB_PATH"]
