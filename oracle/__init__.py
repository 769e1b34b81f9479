"""Plain, slow FP64 CPU oracle for the all-electron RPA screening path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports this; only
the tests, the smoke check and the CPU-baseline leg of the benchmark do.  It
shares no code with the HIP path (its inputs come from the seeded generator
in `synth`, which holds none of the method's arithmetic).

What it computes, in the paper's order (Sec. II.D, Eq. RPA, Eq. eps_LFE,
Eq. eps_noLFE), with readings of unstated points listed in each module:

  gto.py   Gaussian basis, primitive Fourier integrals (binomial expansion
           about the product centre plus the Gaussian moment recursion), the
           27-cell Bloch-summed AO matrix M(k; q+G) and S(k) = M(k; 0).
  rpa.py   pair densities, transition weights, chi0_GG'(q, w), the
           symmetrised eps_GG', its inverse (LAPACK), eps_M and the loss.
  mlp.py   the FP64 reference network for the loss surrogate.

Parity status of each function is stated in its docstring.
"""
