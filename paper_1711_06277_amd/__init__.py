"""MI355X-native adaptive ray tracing (ART) sweep.

``inputs``  seeded synthetic workloads (no method arithmetic);
``_abi``    ctypes binding of libart.so (the C ABI of include/art.h);
``api``     ArtTracer / ArtTrace (torch.autograd.Function) on top of the ABI.

``api`` and ``_abi`` are imported on demand: they need the built HIP library.
"""
__all__ = ["inputs"]
