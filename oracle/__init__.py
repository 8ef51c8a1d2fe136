"""FP64 CPU oracle (test infrastructure; not part of the product path)."""
from .qtt_oracle import *  # noqa: F401,F403
