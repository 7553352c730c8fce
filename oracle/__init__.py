"""FP64 CPU oracle (test infrastructure only; see mpmi_oracle's header)."""
from .mpmi_oracle import *  # noqa: F401,F403
from . import mpmi_oracle  # noqa: F401
