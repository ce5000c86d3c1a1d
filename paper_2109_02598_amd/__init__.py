"""MI355X-native semi-implicit Fourier spectral step (HIP, gfx950).

The compute path lives in the C-ABI library ``libspecstep.so`` built from
``csrc/``; ``specstep`` is the thin Python binding over it.  Importing the
package does not load the library: ``inputs`` (seeded synthetic data) is
usable without a GPU or a build.
"""
__all__ = ["inputs"]
