"""MI355X-native hybrid-PIC step (kinetic ions, massless fluid electrons).

The compute path lives in ``libhvpic.so`` (hand-written HIP for gfx950 behind
the C-ABI declared in ``include/hvpic.h``); :mod:`.hvpic` is its thin ctypes
binding and :mod:`.sim` sequences the calls of one time step.
"""
