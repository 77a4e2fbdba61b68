"""MI355X-native evaluation Y = K~ W of compressed H^2 kernel matrices
(the evaluation phase of MatRox, arXiv 1812.07152).

The compute path is libhm.so (HIP kernels for gfx950) behind the C ABI of
include/hm.h; this package is its Python binding.
"""
from .hm import (HM_BATCH_AUTOTUNE, HM_BATCH_NO_GRAPH, HM_BATCH_TILE, Batch, hm_batch_check, hm_batch_create,  # noqa: F401
                 hm_batch_eval, hm_batch_free, hm_batch_info, hm_eval_batched)
from .hm import (Server, hm_poll, hm_server_add, hm_server_create, hm_server_destroy,  # noqa: F401
                 hm_server_stats, hm_submit)
from .hm import (HM_F32, HM_F64, HM_FAR_FROM_POINTS, HM_LOAD_NO_FAR_BLOCKS, HM_LOAD_NO_NEAR_BLOCKS, HM_LOAD_SYMMETRIC, HM_NEAR_FROM_POINTS, HM_PREC_BF16X3, HM_PREC_FP32, HM_PREC_FP64,  # noqa: F401
                 HM_LEVEL_LAUNCHES, HM_NOALLOC_SCRATCH_BYTES, HM_PROFILE, HM_TREE_ORDER, HMError, Matrix, Repr, hm_check, hm_compress, hm_eval, hm_eval_noalloc, hm_free,
                 hm_info, hm_last_error, hm_load_compressed, hm_load_compressed_mem, hm_profile_read,
                 hm_profile_reset, hm_repr_free, hm_repr_write, hm_set_points, precbit)
from .hm import Structure, hm_inspect_p1, hm_inspect_p2, hm_inspect_p2_load  # noqa: F401
