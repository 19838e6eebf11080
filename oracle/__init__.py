"""CPU oracle for the seam-matched exposure / white-balance correction.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
HIP path is checked against.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never does.
It shares no code with the HIP kernels or their C-ABI: integers are exact
(numpy int64 / Python int) and floating point is IEEE binary64 with every
operation written out, so that a reader can check it against the paper by eye.

Modules
  ringcorr   -- the correction method of section 3.1 ("White balance and
                exposure correction") and the seam gradient cost of
                section 4.2 (the gradient-cost equation).
  crossmap   -- the cross-channel 3x3 linear maps that section 5 proposes:
                cross sums of the bands, Cholesky-factor midway fit, Q16
                matrix maps and their blend with the identity.
  attention  -- the difference approach of section 3.3's attention
                mechanisms: thresholded frame difference, on-pixel counts per
                cell and per sliding window, windows over a threshold.
  surrogate  -- the learned estimator: feature vector, MLP forward/backward,
                MSE loss, Adam and the fallback rule.  The paper has no such
                network; it is specified by the project and pinned by finite
                differences and closed forms only.
"""
