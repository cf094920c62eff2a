"""MI355X (gfx950) hot path for real-time detection of dispersed radio
transients in image cubes (Ruhe et al., arXiv:2103.15418).

The computation lives in the HIP library liblpf.so (C ABI: include/lpf.h);
this package is its thin binding.  Importing it does not touch the GPU;
using a Context or Model without the built library raises.
"""

from ._abi import (DBG, EVENT_ENDED, EVENT_NEW, KERNEL_BOX, KERNEL_DISK, KERNEL_GAUSS, LIB_PATH,  # noqa: F401
                   LPF_EFULL, LPF_EINVAL, LPF_OK, PEAK_DTYPE, PREC_BF16, PREC_FP16, PREC_FP32,
                   SOURCE_DTYPE, Config, Context, LpfError, Model, Server, default_config, detect_batch,
                   extract_flux_batch, ingest_batch, lib, now_ns, pack_weights, select_candidates,
                   workspace_size)
