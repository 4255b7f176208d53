"""MI355X-native exact max-flow / min-cut by parallel augmented-path region
discharge (P-ARD).  The solver is the HIP library libmfard.so behind the C ABI
of include/mf.h; ``paper_1109_1146_amd.mf`` is its ctypes binding."""

__all__ = ["mf"]
