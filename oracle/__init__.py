"""FP64 CPU oracle for complex-valued Frequency Selective Extrapolation.

TEST INFRASTRUCTURE ONLY. This package exists to check the GPU library, and
nothing in the product path may import, call, link or execute it: only the
test suite, the smoke check and the CPU-baseline leg of the benchmark use it.
It shares no code with the GPU path; both take their inputs from ``synth``.

Modules:
  cfse    plain cFSE by direct spatial projection (Section III, eqs. (3),
          (8)-(10), (13), (14), (17)); the reference the GPU results are checked against.
  spectral the frequency-domain form of Section III in FP64 (eqs. (11),
          (12), (15), (18)); a pin for the oracle and a CPU speed reference.
  cfse3   the same in three dimensions (video; Section II and the
          Conclusion), by direct spatio-temporal projection.
  rfse    real-valued FSE, the model of eq. (2), with selection and
          estimation derived as a weighted least-squares fit of each pair.
  fixed   a fixed-point integer encoding of Algorithm 1 with one division
          per block (the Conclusion's argument), defined bit for bit.
  cnn     FP64 forward/backward of the warm-start network (not in the paper).
  metrics PSNR over lost pixels.
"""
