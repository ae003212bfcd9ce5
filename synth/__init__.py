"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package builds inputs only (Gaussian sets, cameras, transfer-function tables,
perturbed copies, sampled pixel lists).  It holds none of the renderer's arithmetic:
no projection, no compositing, no gradients.
"""
from .generators import *  # noqa: F401,F403
