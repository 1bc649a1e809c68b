"""Plain FP64 CPU oracle for polarised A x W-projection gridding and degridding.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only the tests, the smoke check and the benchmark's CPU-baseline leg use it.
It shares no code with the HIP library; the two meet only at the seeded input
generators in `synth`.

Every function is a direct, unblocked transcription of what the paper (arXiv
2206.15117) says the imager computes, or of the textbook definition it relies
on, written in float64 / complex128 with numpy and scipy primitives:

  geometry   uv -> oversampled grid position, footprint, w-plane choice
  pswf       the order-0 prolate spheroidal anti-aliasing function
  mueller    Jones -> Mueller -> Stokes Mueller (Eqs. 3-5), null
             regularisation (Eq. 6) and the per-pixel inverse (Sec. 3.2-3.3)
  kernels    image-domain A x W x anti-aliasing screens and their DFT into
             oversampled uv kernel tables (Sec. 3.2)
  gridding   grid / degrid with 4x4 Mueller kernels (the exact adjoint pair)
  imaging    FFT + taper correction, the predict direction, and brute-force
             direct Fourier transforms used as truth
  plan       the visibility binning (plane, uv tile, oversampling phase)
  mlp        FP64 forward/backward of the kernel-surrogate network
  uvmosaic   UV-domain mosaics: per-field beam kernels on one grid and the
             image correction gamma of Eq. 1 (Sec. 2.2)

Readings of passages the paper leaves open are listed in the module that
takes them.  Functions without an independent pin say "parity unpinned".
"""
