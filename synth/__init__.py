"""Seeded synthetic inputs shared by the oracle tests and the GPU path (no solver arithmetic)."""
from .problems import *  # noqa: F401,F403
