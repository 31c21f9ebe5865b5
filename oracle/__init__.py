"""FP64 CPU oracle of the adaptive-sampling hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct reference written from the paper.  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it; the product
path never does.  It shares no code with the HIP library: its only common dependency is
the seeded input generator `procgen`, which holds none of the method's arithmetic.

Modules (each function cites the passage it follows):
  philox    -- Philox4x32-10 counter-based generator (Salmon et al., SC'11), the u draws
  density   -- sampler CNN and budget normalisation (Sec. 3, Overview)
  sampling  -- stochastic rounding mask, s-normalised scatter, relaxed holdout, pyramid
               (Sec. 4.2 eqs. holdout/stoch_rnoisy, Sec. 4.3 eqs. relaxed_holdout/h_factor,
               App. A eq. app-pyramid)
  filt      -- joint softmax, gather G, learnable upsampling U, warp W, coarse-to-fine
               reconstruction (App. A)
  unet      -- the kernel-predictor U-Net
  tmo       -- differentiable filmic tonemapper and training loss (Sec. 5, Sec. 6.3)
Gradients of the differentiable stages are taken with torch.autograd on these FP64
forward definitions and pinned by central finite differences in the tests.
"""
