"""FP64 CPU oracle of live WDD.  Test infrastructure only: imported by tests, the smoke
check and the benchmark's CPU baseline leg, never by the product path."""
from .wdd import *  # noqa: F401,F403
