"""Plain FP64 CPU oracle for the approximate inverse-CDF method.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check of the entry
module and the CPU-baseline leg of the benchmark may import this package.  The
product (the HIP library and its Python binding) never imports, links or runs
anything here, and nothing here imports the product.

Every function is a slow, direct statement of what the paper defines, in FP64,
with the passage it follows named in its docstring (Giles & Sheridan-Methven,
"Approximating inverse cumulative distribution functions to produce approximate
random variables", arXiv:2012.09715).  Library primitives (erfc, the regularised
incomplete gamma function, a dense linear solve, adaptive quadrature) serve as
single steps; there is no blocking, fusion or reordering beyond the paper's own
definitions.

Modules
  normal     Phi, phi, Phi^-1 (bisection on erfc)                 Section 2
  tables     piecewise-constant and dyadic piecewise-polynomial    Sections 2.2, 2.3
             coefficient tables, their L2 errors
  transform  applying a table to uniforms (Code 1, Algorithm 1)   Sections 3.2, 3.3
  dtypes     IEEE rounding to FP32 / FP16 / BF16
  rng        Philox-4x32-10 and the uniform grids built from it
  gbm        coupled fine/coarse GBM level replay (EM, Milstein)   Section 4
  mlmc       optimal allocation, costs, savings                    Section 4.1
  ncx2       non-central chi-squared CDF and inverse               Section 5
  cir        CIR transition and level replay                       Section 5.2
  mlp        FP64 forward/backward of the surrogate network

Functions with no independent pin say "parity unpinned" in their docstring.
"""
