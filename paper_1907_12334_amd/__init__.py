"""MI355X-native batched Multiple Semi-Coarsened Multigrid (MSG) solves.

The compute path is the HIP shared library ``libmsg.so`` (built from
``csrc/``) behind the C-ABI declared in ``include/msg.h``; ``msg`` is the thin
ctypes binding over it.  Importing this package loads nothing; the library is
loaded on first use and its absence is an error, never a fallback.
"""
