"""MI355X-native periodic thermal homogenization: the design-iteration hot
path of the OpenTM method (arXiv 2405.19991) over hand-written gfx950 HIP
kernels, exposed through a C ABI (include/opentm_amd.h).

The library is loaded lazily on first use and must have been built
(``paper_2405_19991_amd/build.py``); there is no CPU fallback.
"""
from .api import (Batch, Homogenization, Network, apply_device, apply_device_tiled, init_density,  # noqa: F401
                  oc_update_noalloc, run_instance, time_apply_device, version)
