"""MI355X-native correction-function KFBI (arXiv 2309.05965).

The compute path lives in the HIP library ``libkfbi.so`` (C ABI declared in
include/kfbi.h); ``paper_2309_05965_amd.kfbi`` is the thin ctypes binding.
Importing this package loads nothing: the library is opened on first use of
the binding, and the binding raises if it is missing.
"""
