"""FP64 CPU oracle (test infrastructure only; never used by the product path)."""
from .bri_oracle import *  # noqa: F401,F403
from .bri_oracle import __all__  # noqa: F401
