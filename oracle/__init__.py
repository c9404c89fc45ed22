"""FP64 CPU oracle (test infrastructure only; never imported by the product path)."""
from .ibp_oracle import *  # noqa: F401,F403
