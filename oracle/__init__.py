"""CPU oracle for the VEG splatting rasterizer.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
may import this package.  The library (``paper_2504_13339_amd``) never imports it and
shares no code with it.
"""
from .veg_oracle import *  # noqa: F401,F403
