"""CPU FP64 oracle (test infrastructure only; never imported by the product path)."""
from .fcgle_oracle import *  # noqa: F401,F403
