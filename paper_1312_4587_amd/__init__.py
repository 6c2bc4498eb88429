"""MI355X (gfx950) hot path of FFTPL, the FFT-based electrostatic placer of
Lu et al., "FFTPL: An Analytic Placement Algorithm Using Fast Fourier
Transform for Density Equalization".

``libfftpl.so`` (HIP, built by ``paper_1312_4587_amd.build``) holds every
kernel behind the C ABI of ``include/fftpl.h``; ``paper_1312_4587_amd.fftpl``
is its thin Python binding (torch for device memory and streams only).
"""
__all__ = ["fftpl"]
