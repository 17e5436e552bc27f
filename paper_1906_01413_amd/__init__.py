"""MI355X-native RIOT inner loop of incremental 4D-Var (arXiv 1906.01413).

The compute path is the HIP library ``libriot.so`` (C ABI in include/riot.h);
``riot`` is its ctypes binding. Importing this package does not touch the GPU.
"""

from .riot import (ProposalNet, Riot, RiotBatch, RiotError, Sketch, Tracer, load_library, colmajor,  # noqa: F401
                   empty_colmajor, exp_corr_sqrt, gaussian_taps)
