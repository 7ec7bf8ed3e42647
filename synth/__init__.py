"""Seeded synthetic inputs shared by the oracle and the GPU library: physics
data stand-ins (``physics``) and workload generators (``workloads``)."""
from . import physics, workloads  # noqa: F401
