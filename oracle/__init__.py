"""FP64 CPU oracle for scalar diffraction by FFT convolution.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import, call, link or execute anything in
this package. The product library never depends on it, and this package never
imports the product.

Contents:
* ``dft``         direct DFT by DFT-matrix products (exact twiddle arguments)
* ``fft64.c``     textbook radix-2 FP64 FFT, pinned against the direct DFT
* ``diffraction`` the ASM and Fresnel (convolution form) pipelines written out
* ``gs``          one step of the amplitude-constrained ping-pong iteration
"""
from . import dft, diffraction  # noqa: F401
