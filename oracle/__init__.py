"""Plain, slow, obviously-correct CPU oracle for scene-space gathering and filtering.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import or run anything in this package; the
product path (the HIP library and its Python binding) never does, and the
oracle never imports the product package. The two share no code.

Arithmetic is float64 throughout. Inputs are taken the way the GPU stores them
("mode Q": colour and depth rounded to IEEE binary16, then widened exactly to
float64), or unquantised ("mode F": u8/255 and float32 depth in float64) for
error reports.

Modules and the passages they follow (Klose et al., Sampling Based Scene-Space
Video Processing):
  staging    -- colour/depth storage rounding (the stored input planes)
  poses      -- camera matrices C^f, their inverses and relative products (Sec. 3, Sec. 4 Eq. 1-2)
  gather     -- sample sets S^f(p) with the depth-guided frustum test (Sec. 4)
  filters    -- weighted mean O(p) = sum w(s) s_rgb / W (Sec. 5 Eq. 3) with the
                Gaussian denoising weight around the reference sample (Sec. 5 Eq. 4);
                the per-frame factors of deblurring (Sec. 5 Eq. 5) and computational
                shutters (Eq. 10); inpainting by masked mean-shift (Eq. 8-9)
  frustum    -- the paper's depth-agnostic frustum gather (Sec. 4, Eq. 1-2) by its
                definition, and the hull-rasterisation algorithm that pins it
  depth      -- data-term-only multi-view depth over a temporal window (Sec. 3,
                preprocessing: 3x3 RGB SSD along the epipolar lines, lowest mean cost)
  bruteforce -- all-pairs twin of `gather` for tiny inputs (pure Python loops)
  metrics    -- PSNR (Sec. 5, the denoising PSNR figure)

Parity unpinned: nothing in this package is unpinned; see the test suite for
the pin of each function.
"""
