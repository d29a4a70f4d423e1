"""MI355X-native PEPS-VMC hot path: amplitude, local energy and log-derivative.

The compute lives in the HIP library ``libpeps_hip.so`` behind the C ABI of
``include/peps.h``; ``peps`` holds the ctypes binding and the autograd wrapper.
The binding is imported lazily so that ``workloads`` works without a GPU.
"""
__all__ = ["workloads"]
