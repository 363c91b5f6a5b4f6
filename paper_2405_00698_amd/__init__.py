"""MI355X (gfx950) soft-robot co-design hot path: a C-ABI HIP library
(libsoftrobot.so) with a thin Python binding.  See include/softrobot.h."""
from ._lib import (SR_NO_ACTUATION, SR_NO_GRAVITY, SR_NO_GROUND, SR_QUERY_BF16, SR_QUERY_FP32,  # noqa: F401
                   SR_STEP_AUTO, SR_STEP_PERSISTENT, SR_STEP_PLAIN, SR_WEIGHT_ACTUATION, GENOME_LEN,
                   SoftRobotError, default_params, table2_params, load)


def __getattr__(name):
    if name in ("Population",):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
