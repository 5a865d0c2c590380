"""SDF photon random walk (McMillan, Bruce & Dholakia 2021) for MI355X.

The GPU path lives in ``paper_2112_08035_amd.smcrt`` (ctypes binding of
``libsmcrt.so``); seeded synthetic inputs in ``paper_2112_08035_amd.workloads``.
Importing this package loads nothing.
"""
__version__ = "0.1.0"
