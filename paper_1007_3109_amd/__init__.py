"""lbrd: MI355X-native reacting-species D2Q9 lattice Boltzmann.

The compute path is the HIP library ``liblbrd.so`` behind the C ABI declared
in ``include/lbrd.h``; ``paper_1007_3109_amd.lbrd`` is its ctypes binding.
Importing this package does not load the library (the host-only helpers in
``analysis`` and ``workloads`` work without a GPU); importing the binding
does, and fails loudly if the library was not built.
"""
__all__ = ["analysis", "workloads"]
