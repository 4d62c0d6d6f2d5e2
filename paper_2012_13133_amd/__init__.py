"""MI355X (gfx950) implementation of the Kryging hot path: masked BTTB
covariance products by circulant embedding and FFT, and the Krylov
iterations that consume them (Lanczos quadrature log-determinants, CG and
generalized Golub-Kahan solves, kriging and the parametric bootstrap).

The compute lives in the HIP library ``libkryging.so`` (C ABI in
``include/kryging.h``); ``paper_2012_13133_amd.kryging`` is its ctypes
binding.  ``paper_2012_13133_amd.synth`` holds seeded synthetic inputs.
"""
