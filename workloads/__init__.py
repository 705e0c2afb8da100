"""Seeded synthetic inputs (circuits, channels, Hamiltonians, uniforms) shared by the oracle,
tests and benchmark. Holds no arithmetic of the low-rank method itself."""
from .circuits import *  # noqa: F401,F403
