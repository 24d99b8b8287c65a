"""MI355X-native Basic Scheme for FFT-based homogenisation on patterns P(M).

The compute path is the C-ABI library ``liblsh.so`` (hand-written HIP for
gfx950, declared in ``include/lsh.h``); ``lsh`` is its thin ctypes binding.
"""
