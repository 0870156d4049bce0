"""Bessel function J_0 in FP64 for Example 2's Schloemilch kernel
K(g, w) = J_0(g w).  Test infrastructure: only tests, the package's smoke
check and the bench's CPU baseline use this module.

Entries are evaluated at z = fl(g * w), the FP64 product of the two points,
by two published methods chosen by the size of z:

* z < 25: Miller's normalized backward recurrence.  Starting from
  f_{n0+1} = 0, f_{n0} = 1e-30 at the even index n0 = 2 floor((z + 40) / 2),
  f_{n-1} = (2 n / z) f_n - f_{n+1} runs down to f_0; since
  J_0 + 2 sum_{k>=1} J_{2k} = 1, J_0(z) = f_0 / (f_0 + 2 sum_{k>=1} f_{2k})
  (Abramowitz & Stegun 9.12 and 9.1.46; the start index is measured against a
  40-digit reference to give 4e-16 absolute error on [0, 25)).  Values are
  rescaled by 1e-200 whenever |f| exceeds 1e200.
* z >= 25: Hankel's asymptotic expansion (A&S 9.2.5, 9.2.9, 9.2.10),
    J_0(z) = sqrt(2 / (pi z)) (P(z) cos chi - Q(z) sin chi),  chi = z - pi/4,
    P = sum_m (-1)^m b_{2m} / z^{2m},  Q = -sum_m (-1)^m b_{2m+1} / z^{2m+1},
    b_k = (1 3 ... (2k-1))^2 / (k! 8^k),
  with 11 terms each (the 22nd term is below 1e-17 from z = 25 on).  With
  cos chi = (cos z + sin z) / sqrt 2 and sin chi = (sin z - cos z) / sqrt 2
  this is J_0 = ((P + Q) cos z + (P - Q) sin z) / sqrt(pi z).  The argument
  is reduced as z = n pi/2 + r, n = rint(2 z / pi), by a three-part split of
  pi/2 (Cody and Waite): C1 and C2 are pi/2 and its remainder truncated to
  27 and 29 significant bits, so n C1 and n C2 are exact for n < 2^24, and
  C3 is the next 53 bits (C1 + C2 + C3 = pi/2 to 4e-35).

The HIP path implements the same two methods in the same operation order
without fused multiply-adds, so the two agree to rounding of the library
sin, cos and sqrt.
"""
from __future__ import annotations

import numpy as np

SMALL = 25.0           # Miller below, Hankel from here on
HANKEL_TERMS = 11      # terms of P and of Q
MILLER_EXTRA = 40.0    # n0 = 2 floor((z + extra) / 2)
PIO2_C1 = float.fromhex("0x1.921fb54000000p+0")
PIO2_C2 = float.fromhex("0x1.10b4611000000p-30")
PIO2_C3 = float.fromhex("0x1.4c4c6628b80dcp-59")
TWO_OVER_PI = 2.0 / np.pi


def hankel_coefficients() -> list[float]:
    """b_0 .. b_{2 HANKEL_TERMS - 1}: b_k = b_{k-1} (2k-1)^2 / (8k) in float64."""
    b = [1.0]
    for k in range(1, 2 * HANKEL_TERMS):
        b.append(b[-1] * float((2 * k - 1) * (2 * k - 1)) / float(8 * k))
    return b


def _miller(z: np.ndarray) -> np.ndarray:
    n0 = 2.0 * np.floor((z + MILLER_EXTRA) / 2.0)
    r = 2.0 / np.where(z > 0, z, 1.0)
    f = np.zeros_like(z)
    fn = np.zeros_like(z)
    s = np.zeros_like(z)
    for n in range(int(n0.max()) if z.size else 0, 0, -1):
        start = n0 == n
        f = np.where(start, 1e-30, f)
        fn = np.where(start, 0.0, fn)
        s = np.where(start, 1e-30, s)  # n0 is even: J_{n0} is the first term of the sum
        act = n <= n0
        fp = (n * r) * f - fn          # f_{n-1}
        fn = np.where(act, f, fn)
        f = np.where(act, fp, f)
        if (n - 1) % 2 == 0 and n - 1 >= 2:
            s = np.where(act, s + f, s)
        big = np.abs(f) > 1e200
        f = np.where(big, f * 1e-200, f)
        fn = np.where(big, fn * 1e-200, fn)
        s = np.where(big, s * 1e-200, s)
    return np.where(z > 0, f / (f + 2.0 * s), 1.0)


def _hankel(z: np.ndarray) -> np.ndarray:
    b = hankel_coefficients()
    u = 1.0 / (z * z)
    p = np.full_like(z, (-1.0) ** (HANKEL_TERMS - 1) * b[2 * HANKEL_TERMS - 2])
    q = np.full_like(z, (-1.0) ** (HANKEL_TERMS - 1) * b[2 * HANKEL_TERMS - 1])
    for m in range(HANKEL_TERMS - 2, -1, -1):
        p = p * u + (-1.0) ** m * b[2 * m]
        q = q * u + (-1.0) ** m * b[2 * m + 1]
    q = -q / z
    n = np.rint(z * TWO_OVER_PI)
    r = ((z - n * PIO2_C1) - n * PIO2_C2) - n * PIO2_C3
    sr, cr = np.sin(r), np.cos(r)
    quad = n.astype(np.int64) & 3
    cz = np.choose(quad, [cr, -sr, -cr, sr])
    sz = np.choose(quad, [sr, cr, -sr, -cr])
    return ((p + q) * cz + (p - q) * sz) / np.sqrt(np.pi * z)


def j0(z) -> np.ndarray:
    """J_0 of float64 arguments (any shape), |z| < 2^24 pi/2."""
    z = np.abs(np.asarray(z, dtype=np.float64))
    if np.any(z >= 2.0 ** 24 * PIO2_C1):
        raise ValueError("J_0 argument beyond the reduction's range")
    out = np.empty_like(z)
    small = z < SMALL
    if np.any(small):
        out[small] = _miller(z[small])
    if np.any(~small):
        out[~small] = _hankel(z[~small])
    return out
