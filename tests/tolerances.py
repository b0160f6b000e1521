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

Batched forms (rank 16): the near field of step (6) (the dense near-diagonal leaf block)
and the final sum of near and far parts are FP64 in every form; the far part (steps
(1)-(5): T, B, Ahat products) runs in the form's precision with FP32 accumulation.  So the
error is the far part's: about u_form sqrt(2LM) times the far part's magnitude, which on
the decaying inputs f_j = z_j/(j+1) of the configurations is ~1e-3 .. 1e-2 of max|z|.

FP32 form: unit roundoff 2^-24.  Measured maximum over every configuration input (decaying):
5.6e-9 (n = 20000, leaf 32); the bound is about 3x that.  On undecayed inputs (uniform on
[0, 1), the protocol of Table 1) the far part is of the order of max|z|: TOL32_U and
its siblings below.

BF16 hi+lo form: each product is ah bh + ah bl + al bh (al bl dropped, lo parts rounded)
with FP32 accumulation, about 2^-17 relative per product.  Measured maximum (decaying):
2.5e-8 (n = 20000, leg2cheb); the bound is about 3x that.

FP16 hi+lo form: products of 22-bit operands (about 2^-22 relative per product; the
scaling by powers of two is exact), FP32 accumulation.  Measured maximum (decaying):
1.0e-9 (n = 129); the bound is about 3x that.  A tile whose transforms are scaled by
10^-30 .. 10^30 loses accuracy where the tiny ones' far-field products fall into FP32's
subnormal range: measured 2.5e-7, bound TOLF16_SCALED.
"""

TOL64 = {(0, 18): 1e-13, (1, 18): 1e-13, (0, 20): 1e-13, (1, 20): 1e-13,
         (0, 24): 1e-13, (1, 24): 1e-13,
         # lower ranks: the rank's own truncation error
         (0, 16): 1e-12, (1, 16): 1e-11, (0, 12): 1e-9, (1, 12): 1e-8}
TOL32 = 2e-8
TOLBF = 8e-8
TOLF16 = 3e-9
TOLF16_SCALED = 7.5e-7
# undecayed inputs (uniform on [0, 1)), n = 20000, 16 transforms, both directions
# (test_batched_forms_undecayed): measured 2.75e-7 (FP32), 8.3e-6 (BF16 hi+lo), 2.2e-7
# (FP16 hi+lo), all in leg2cheb; the bounds are about 3x those
TOL32_U = 8.5e-7
TOLBF_U = 2.5e-5
TOLF16_U = 6.5e-7

# DCTs of kinds 2 and 3 (the library's FFT, FP64), E_inf relative to max|y|: an FFT's
# rounding error grows like sqrt(log2 n) u in norm.  Measured maximum over n = 1 .. 2^20
# (one-, two- and three-pass lengths, radices 2 .. 8): 1.63e-15 (n = 3^11, kind 2); the
# bound is about 3x that.
TOL_DCT = 5e-15


# The grid pipeline (Sec. 1: leg2cheb then the DCT of kind 3, or the DCT of kind 2 then
# cheb2leg).  The FMM's error is about u times max|c| in every coefficient, also in the
# small ones, and the DCT of kind 3 sums n such errors with varying signs: the grid values
# carry about sqrt(n) u max|c| (the round trip the same again).  Measured E_inf / (sqrt(n) u),
# u = 2^-53: 0.4 (leg2grid, n = 6000), 2.0 (leg2grid, n = 65536), 1.6 (round trip,
# n = 10^6); the bound is 6 sqrt(n) u.
def TOL_GRID(n):
    return 6.0 * max(n, 1) ** 0.5 * 2.0 ** -53
