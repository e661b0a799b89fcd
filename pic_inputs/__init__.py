"""Seeded synthetic inputs shared by the simulation library's callers and the
test oracle: workload parameter sets, cross-section tables and initial
particle states. Nothing here performs a step of the PIC/MCC method."""
from . import state, workloads, xsec  # noqa: F401
