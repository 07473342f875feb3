"""MI355X-native vertex-vs-SDF contact queries and contact reduction.

The compute path is the HIP library ``libfactory_sdf.so`` built from
``csrc/``; ``fc`` is its ctypes binding and ``autograd`` wraps the adjoint in
a ``torch.autograd.Function``.  ``workloads`` builds seeded synthetic inputs.
Submodules are imported lazily so that input generation works without the
library.
"""
__all__ = ["fc", "autograd", "workloads", "autotune", "build"]
