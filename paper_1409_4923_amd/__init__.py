"""libbmotor: Monte Carlo integration of Brownian-motor Langevin equations on MI355X.

The compute path is the HIP library ``libbmotor.so`` (C ABI in include/bmotor.h);
``bmotor`` is its ctypes binding and ``workloads`` holds seeded parameter sets.
"""
from . import workloads  # noqa: F401

__all__ = ["bmotor", "workloads"]
