"""Own FP64 transcendental routines and the Gaussian transform (oracle side).

The paper draws Theta_ir from a centred Gaussian with spread L^-0.5
(Sec. III-A, Eq. 5) and initialises the GCN weights at random (Sec. III-B).
For the two sides of the parity check to draw *identical* Gaussians, the
uniform -> normal map uses only IEEE basic operations (+, -, *, /, sqrt,
exact exponent split, exact rint), in a fixed order, with no fused
multiply-add.  NumPy ufuncs round every operation separately, so this file is
exactly that sequence.

* ln(x):  x = m * 2^e with m in [sqrt(1/2), sqrt(2));  ln m = 2 atanh(f),
  f = (m-1)/(m+1), by its odd power series through f^23;  ln x = e*ln2 + ln m.
* sincos(2*pi*u), u in (0,1):  k = rint(4u) (exact), r = 4u - k (exact),
  t = r * (pi/2), |t| <= pi/4;  Taylor series of sin through t^19 and of cos
  through t^20; quadrant k selects signs and swap.
* Box-Muller:  rho = sqrt(-2 ln u0), z0 = rho cos(2 pi u1), z1 = rho sin(2 pi u1).
* uniform:  u = ((x >> 12) + 0.5) * 2^-52, in (0, 1), exact.

Pinned in ``tests/test_oracle_random.py`` against ``math.log/sin/cos`` (a few
ulp) and by moment / Kolmogorov-Smirnov tests of the resulting normals.
"""
import math
import numpy as np

LN2 = float.fromhex("0x1.62e42fefa39efp-1")          # double nearest ln 2
HALF_PI = float.fromhex("0x1.921fb54442d18p+0")      # double nearest pi/2
SQRT_HALF = float.fromhex("0x1.6a09e667f3bcdp-1")    # double nearest sqrt(1/2)
TWO_M52 = 2.0 ** -52

# 1/(2j+1) for the atanh series, j = 1..11
_ATANH_C = [1.0 / float(2 * j + 1) for j in range(1, 12)]
# 1/n! for the Taylor series, n = 0..20 (n! is exact in binary64 for n <= 22)
_INV_FACT = [1.0 / float(math.factorial(n)) for n in range(0, 21)]


def ln(x):
    """Natural log of positive finite doubles (array), own routine."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                      # x = m * 2^e, m in [0.5, 1)
    small = m < SQRT_HALF
    m = np.where(small, m * 2.0, m)         # exact
    e = np.where(small, e - 1, e).astype(np.float64)
    f = (m - 1.0) / (m + 1.0)
    f2 = f * f
    s = _ATANH_C[-1]
    for c in reversed(_ATANH_C[:-1]):
        s = c + f2 * s
    s = f2 * s                              # f^2/3 + f^4/5 + ...
    lnm = 2.0 * f + (2.0 * f) * s
    return e * LN2 + lnm


def sincos_2pi(u):
    """(sin(2 pi u), cos(2 pi u)) for u in [0, 1], own routine."""
    u = np.asarray(u, dtype=np.float64)
    u4 = u * 4.0                            # exact
    k = np.rint(u4)                         # exact, round half to even
    r = u4 - k                              # exact, |r| <= 1/2
    t = r * HALF_PI
    t2 = t * t
    # sin t = t + t^3 * P(t^2),  P = -1/3! + t^2/5! - ... - t^16/19!
    ps = -_INV_FACT[19]
    for n in (17, 15, 13, 11, 9, 7, 5, 3):
        cn = _INV_FACT[n] if ((n - 1) // 2) % 2 == 0 else -_INV_FACT[n]
        ps = cn + t2 * ps
    s = t + (t * t2) * ps
    # cos t = 1 + t^2 * P(t^2),  P = -1/2! + t^2/4! - ... + t^18/20!
    pc = _INV_FACT[20]
    for n in (18, 16, 14, 12, 10, 8, 6, 4, 2):
        cn = _INV_FACT[n] if (n // 2) % 2 == 0 else -_INV_FACT[n]
        pc = cn + t2 * pc
    c = 1.0 + t2 * pc
    q = np.mod(k, 4.0).astype(np.int64)
    sin = np.select([q == 0, q == 1, q == 2, q == 3], [s, c, -s, -c])
    cos = np.select([q == 0, q == 1, q == 2, q == 3], [c, -s, -c, s])
    return sin, cos


def uniform52(x):
    """uint64 -> double in (0,1): ((x >> 12) + 0.5) * 2^-52, exact."""
    x = np.asarray(x, dtype=np.uint64)
    return ((x >> np.uint64(12)).astype(np.float64) + 0.5) * TWO_M52


def box_muller(u0, u1):
    """Two independent standard normals from two uniforms in (0,1)."""
    rho = np.sqrt(-2.0 * ln(u0))
    s, c = sincos_2pi(u1)
    return rho * c, rho * s


def normals_from_block(blk):
    """Philox block [..., 4] -> four standard normals [..., 4] (FP64).

    Words (0,1) give normals 0 and 1; words (2,3) give normals 2 and 3.
    """
    u = uniform52(blk)
    z0, z1 = box_muller(u[..., 0], u[..., 1])
    z2, z3 = box_muller(u[..., 2], u[..., 3])
    return np.stack([z0, z1, z2, z3], axis=-1)
