"""Fisher-vector encoding on AMD MI355X (gfx950): thin Python binding of libfv.

Every step of the encoder runs in the HIP kernels of ``libfv.so``; this package only
marshals arguments (numpy arrays for host memory, torch tensors for device memory and
streams).  If the library has not been built, :func:`load` raises -- there is no fallback.
"""
from .fv import (  # noqa: F401
    FvError, Gmm, load, lib_path, limits, gmm_load, gmm_free, gmm_info, encode, encode_batch,
    strerror, last_device_error, kernel_timing, kernel_timing_read,
    OK, PENDING, E_INVAL, E_NOMEM, E_DEVICE, E_BUDGET, E_AGAIN, E_NOTFOUND, E_TIMEOUT,
    E_UNSUPPORTED, PREC_FP32, PREC_BF16_SPLIT, PREC_FP16_SPLIT, PREC_BF16, X_DEVICE, OUT_DEVICE,
    NO_POWER_NORM, NO_L2_NORM, ASYNC, THRESHOLD, THRESHOLD_TAU, PROJ_SPLIT16, EXPORTED_SYMBOLS, EXEC_HIP,
    EXEC_FAKE, Server, ServerConfig,
    server_config, set_tuning, get_tuning, Tuning, Pca, pca_load, project, encode_projected,
    encode_batch_projected, em_step, em_fit, stream_release, DSIFT_DIM, dsift_rows, dsift,
    encode_images, encode_noalloc, graph_counters,
)
