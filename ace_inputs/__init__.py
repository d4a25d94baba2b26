"""Seeded synthetic workloads (inputs only; no ACE arithmetic)."""
from .generators import *  # noqa: F401,F403
