"""MI355X-native reaction + SDC stage of the partitioned bidomain strategy.

The numerical work runs in hand-written HIP kernels for gfx950 behind the C ABI
of include/ionic_sdc.h (libionic_sdc.so); ``paper_2510_27447_amd.ionic`` is
the thin ctypes binding with the same entry-point names, using PyTorch only
for device memory and streams.  ``workloads`` builds the seeded synthetic
inputs and ``serve`` the continuous-batching request loop.
"""
