"""MI355X-native LOBPCG eigensolver for real-space Kohn-Sham DFT.

The compute path is the HIP library ``libksh.so`` (sources in ``csrc/``,
C ABI in ``include/ksh.h``); ``binding`` marshals torch device tensors into
it.  There is no CPU fallback: without the built library the binding raises.
"""
