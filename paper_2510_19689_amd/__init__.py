"""MI355X-native batched TabNet inference: predictions plus per-step feature masks.

The compute path is the HIP library ``libtabnet.so`` (C ABI, declared in
include/tabnet.h); ``paper_2510_19689_amd.tabnet`` is its thin Python binding.
``paper_2510_19689_amd.synth`` draws seeded models and inputs.
"""
__all__ = ["synth"]
