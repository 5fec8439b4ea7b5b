"""Error bars of the mixed-precision forms, derived from the arithmetic.

The low-precision Newton-Schulz iterations return the sign of a matrix
X + Delta with ||Delta|| about K u ||X|| (K = 21 scaled steps, u the unit
roundoff of the low precision).  Pi is 1-Lipschitz, so two effects bound the
error of the assembled projection:

* components with |lambda| below the resolution tau = c u ||X||_2 may be
  classified either way; each contributes at most |lambda|, so their share is
  at most band(tau) = sqrt(sum of lambda^2 over |lambda| < tau);
* the remaining components carry the first-order eigenvector error, which in
  the eigenbasis of X is (l_i + l_j)/(l_i - l_j) [X, S]_ij / 4 on entries
  coupling opposite signs, of modulus at most |[X, S]_ij| / 4, and the
  eigenvalue error of S, at most sqrt(||X||_F^2 - ||X S||_F^2) / 4: the
  library's est_rel_err combines the two relative to ||Pi||_F (first order,
  so a factor 2 of slack).

The stated bar of a mixed result is band(2 u ||X||_2) + 2 est ||Pi||_F.  For
FP32 there is also the fixed bar FP32_REL_BAR = 1e-5, from
K u sqrt(2) c = 21 * 2^-24 * 1.41 * 4 = 7.1e-6 (||X||_F / ||Pi||_F is about
sqrt(2) for spectra symmetric about 0), rounded up.  The split-BF16 form
("BF16x3", u = 2^-16) is held to the band at 2 u ||X||_2 plus twice its
estimate, like BF16.
"""
import numpy as np

U_BF16 = 2.0 ** -8
U_FP32 = 2.0 ** -24
# split BF16 products: an FP32 value as hi + lo (two BF16 terms) is within
# 2^-17 of itself relative, and dropping lo*lo costs at most 2^-16 of a
# product, so a split product carries the unit roundoff of a 16-bit format
U_BF16X3 = 2.0 ** -16
FP32_REL_BAR = 1e-5
BAND_C = 2.0


def unit_roundoff(mode: str) -> float:
    return {"mixed_bf16": U_BF16, "mixed_bf16x3": U_BF16X3}.get(mode, U_FP32)


def ns_l0(mode: str) -> float:
    """Lower end of the Newton-Schulz schedule the library uses in `mode`:
    max(1e-6, u/4) for the unit roundoff u of the iterates' format (BF16
    2^-8, split BF16 2^-16, FP32 2^-24)."""
    u = {"mixed_bf16": 2.0 ** -8, "mixed_bf16x3": 2.0 ** -16}.get(mode, 2.0 ** -24)
    return max(1e-6, 0.25 * u)


def band_norm(lam, mode: str, c: float = BAND_C) -> float:
    """sqrt(sum lambda^2 over |lambda| < c u ||X||_2)."""
    lam = np.asarray(lam, dtype=np.float64)
    tau = c * unit_roundoff(mode) * np.abs(lam).max()
    return float(np.sqrt(np.sum(lam[np.abs(lam) < tau] ** 2)))


def mixed_bar_abs(lam, mode: str, pi_norm: float, est: float) -> float:
    """Absolute Frobenius bar of a mixed result (band + first-order term)."""
    return band_norm(lam, mode) + 2.0 * est * pi_norm + 1e-12 * pi_norm
