"""Error bounds of the GPU parity tests (E_inf of Eq. (Einf) against the direct oracle).

FP64 path, leg2cheb: 1e-13 at every size and rank >= 18 (the requirement on the FP64
path).  Measured on the configuration inputs: 1e-16 .. 2e-15.

FP64 path, cheb2leg: 1e-13 on the configurations' decaying inputs f_j = z_j/(j+1)^r,
r = 1/2 or 1.  The reverse kernel of Eq. (Lxymod) is less smooth near the diagonal than
the forward one, and at rank 18 one submatrix carries ~3e-13 relative Chebyshev
truncation error (measured against mpmath), but on decaying inputs the error relative to
max|z| stays at 1e-15 .. 1e-14 (measured: 2.3e-15 at N = 10^6, 8.4e-15 on the ragged
batch).  The uniform-input protocol of Table 1 (r = 0) is held to its own printed values
instead (Table 1 reports cheb2leg errors up to 2e-13 for the paper's code).

FP32 form (rank 16): every product in FP32 (unit roundoff u = 2^-24) with FP32
accumulation; inputs rounded once, outputs scaled and stored in FP64.  An output row is
a sum of at most 2s near-field terms plus a far-field value built through L upward and L
downward transfers of M-term sums: random signs give about sqrt(2s + 2LM) u ~ 1e-6 at
s = 32, L = 9, M = 16, a worst-case sign pattern (2s + 2LM) u ~ 2e-5.  Measured maximum
over every configuration: 7.4e-7 (the ragged batch of configuration 4); the bound is about
3x that.

BF16 hi+lo form: each product is ah bh + ah bl + al bh (al bl dropped, lo parts rounded)
with FP32 accumulation, about 2^-17 relative per product: random signs give
sqrt(352) 2^-17 ~ 1.4e-4 as a model bound.  Measured maximum over every configuration:
1.14e-5 (n = 1024, cheb2leg); the bound is about 3x that.
"""

TOL64 = {(0, 18): 1e-13, (1, 18): 1e-13, (0, 20): 1e-13, (1, 20): 1e-13,
         (0, 24): 1e-13, (1, 24): 1e-13,
         # lower ranks: the rank's own truncation error
         (0, 16): 1e-12, (1, 16): 1e-11, (0, 12): 1e-9, (1, 12): 1e-8}
TOL32 = 2.5e-6
# FP16 hi+lo form: products of 22-bit operands (the lo parts' rounding and the dropped
# lo lo term leave about 2^-22 relative per product; the scaling by powers of two is
# exact), FP32 accumulation as in the FP32 form, so the FP32 form's error model applies.
# Measured maximum over every configuration: 5.9e-7 (the 256 x 65536 batch against the FP64
# path); the bound is about 3x that.
TOLF16 = 2e-6
TOLBF = 3.5e-5
