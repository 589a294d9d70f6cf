"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This package holds no arithmetic of the reconstruction method: it draws
specimens, sampling masks and noise, and lists the workload presets.  Anything
that needs the system operator (noise scaled to the signal, lambda scaled to
lambda_max) is composed by the caller.
"""
from .generators import *  # noqa: F401,F403
