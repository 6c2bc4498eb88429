"""FP64 CPU oracle for one evaluation of the FFT-based electrostatic placer.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path.
"""
from .fftpl_oracle import *  # noqa: F401,F403
from .fftpl_oracle import __all__  # noqa: F401
