"""MI355X-native next-best-view scoring for object-aware 3D Gaussian Splatting.

The compute path is the HIP library ``_build/libngs.so`` (C ABI in ``include/ngs.h``);
``binding`` marshals torch device tensors into it. Build with ``build.build()``.
"""
__all__ = ["binding", "build"]
