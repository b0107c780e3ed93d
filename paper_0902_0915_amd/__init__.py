"""MI355X-native convolutional gridding of radio visibilities, FFT imaging and adjoints.

The compute path is a C-ABI HIP library (``libmwagrid.so``, declared in include/mwagrid.h);
``paper_0902_0915_amd.mwagrid`` is its thin ctypes binding, which fails loudly if the
library has not been built. ``paper_0902_0915_amd.synth`` produces seeded synthetic inputs.
"""
__all__ = ["mwagrid", "synth"]
