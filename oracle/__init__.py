"""Plain, slow FP64 CPU oracle of the semi-implicit Fourier spectral step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call
or execute this package: only the test suite, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP
library (no kernels, headers, tables or helpers); its inputs come from
the seeded generator module, which holds none of the method's
arithmetic.

Contents
  spectral.py   the exponential (ETD1) spectral scheme of Sec. 2.4.2,
                Eqs. 1-4 and the update rule Eq. 8, for the models of
                Sec. 3 (Eqs. 9-13) and Gray-Scott.
  fd_euler.py   the explicit forward-Euler finite-difference solver of
                Sec. 2.4.1 with the 5/7-point Laplacian of Sec. 2.2.2,
                used as an independent discretisation to pin the scheme.
  adjoint.py    the discrete adjoint of the spectral map for Gray-Scott,
                with checkpoint-and-recompute (no counterpart in the paper;
                it is the exact transpose of the map in spectral.py).
  structure.py  the radially averaged structure factor of Sec. 3
                (Eq. 14, Porod's law).
  operator_split.py  the procedure of Sec. 2.4.2 that builds the scheme
                from equation text (linear/nonlinear split, derivative
                pairing, A and B_i), with the ETD1 and the linearly
                implicit factors.

The FFT is numpy's (a library primitive); the oracle uses full complex
transforms over every axis, never a real-to-complex layout.
"""
