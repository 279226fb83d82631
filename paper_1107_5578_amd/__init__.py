"""MI355X-native scalar diffraction by FFT convolution (angular spectrum and
Fresnel convolution form), hand-written HIP for gfx950 behind a C ABI.

Importing the package loads nothing native; ``paper_1107_5578_amd.cwo`` loads
the HIP library and raises if it is missing.
"""
__all__ = ["cwo", "workloads"]
