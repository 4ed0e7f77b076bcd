"""FP64 CPU oracle for learned digital backpropagation (LDBP) and the split-step method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call or
execute anything under ``oracle/``; only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP path.

The code is deliberately plain: NumPy complex128, direct sums, ``numpy.fft`` as
the only library primitive, no blocking, no fusion, no reordering beyond what the
paper's definitions state.  Each function cites the passage it follows
(section / equation of Haeger & Pfister, "Physics-Based Deep Learning for
Fiber-Optic Communication Systems", arXiv 2010.14258).

Modules
  units    physical constants and unit conversions (Table I)
  ldbp     the LDBP model (eq. model, Sec. III-B) and its adjoint
  ssm      time-discretised NLSE, split-step channel and FFT-based DBP (Sec. III-A)
  txrx     transmitter, receiver DSP, MSE and effective SNR (Sec. IV-A, IV-B)
  design   log step sizes, half-step merging, least-squares taps, Kerr coefficients (Sec. IV-C)
  train    Adam update and the progressive pruning schedule (Sec. IV-B, IV-C)
  philox   counter-based Philox4x32-10 generator + Box-Muller (Salmon et al., SC'11)

Parity status of each function is listed in its module docstring; functions
without an independent pin say "parity unpinned" there.
"""
