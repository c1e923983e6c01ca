"""Seeded synthetic inputs shared by the CPU oracle and the GPU library (data only)."""
from .problems import *  # noqa: F401,F403
