"""MI355X (gfx950) PairHMM forward library: Python binding.

The compute path is the C-ABI library ``libphmm.so`` built from ``csrc/``
(hand-written HIP for gfx950); this package only marshals arguments to it.
There is no CPU fallback: importing works anywhere, but every compute call
needs the built library and a gfx950 device and raises otherwise.
"""
from ._binding import (  # noqa: F401
    PHMM_OK, PHMM_EINVAL, PHMM_ERANGE, PHMM_ENOMEM, PHMM_EDEVICE, PHMM_ETIMEOUT,
    PHMM_FP32_RERUN, PHMM_FP64_PLAIN, PHMM_FLAG_FP32, PHMM_FLAG_RERUN, PHMM_FLAG_LONG,
    PHMM_FLAG_RESCALED, PHMM_FLAG_FP64, PHMM_PENDING, PhmmError, Context, Server, lib, lib_path,
    phmm_num_classes, phmm_class_n, phmm_validate_batch, phmm_forward_batch,
    phmm_forward_one, phmm_workspace_bytes, phmm_forward_batch_async, phmm_device_status,
    phmm_forward_batch_noalloc, phmm_forward_batch_graph,
    phmm_last_counts, phmm_last_timing, phmm_vector_peak, phmm_copy_calib, DeviceBatch,
    genotype_offsets, phmm_genotype_batch, phmm_genotype_batch_async,
)
