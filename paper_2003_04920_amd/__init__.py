"""MI355X (gfx950) implementation of PI-RRT#'s exploitation phase (Replan) behind a
C ABI (include/pirrt.h), after "GPU Parallelization of Policy Iteration RRT#"
(arXiv 2003.04920).  The Python side is a ctypes binding only."""
from .binding import (Graph, Batch, Rrg, Mlp, PirrtError, load, pirrt_config, pirrt_stats, LIB_PATH, EXPORTS,  # noqa: F401
                      PIRRT_OK, PIRRT_EINVAL, PIRRT_ENOMEM, PIRRT_EDEVICE, PIRRT_ENOTCONVERGED,
                      PIRRT_MEM_HOST, PIRRT_MEM_DEVICE, PIRRT_NO_PRUNE, PIRRT_TIMING, PIRRT_LOOKAHEAD,
                      PIRRT_TRUNCATED, PIRRT_MLP_NOALLOC_MAX_BATCH)
