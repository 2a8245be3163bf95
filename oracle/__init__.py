"""FP64 CPU oracle (test infrastructure only; see :mod:`oracle.sfista64`)."""

from .sfista64 import *  # noqa: F401,F403
