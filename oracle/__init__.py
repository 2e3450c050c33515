"""Plain FP64 CPU oracle of the differential-BEM hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import it.  The product (the HIP library and
its Python binding) never calls it; it shares no code with the GPU path.
"""
from .bem_oracle import *  # noqa: F401,F403
from . import straight  # noqa: F401,E402
from . import regularizers  # noqa: F401,E402
