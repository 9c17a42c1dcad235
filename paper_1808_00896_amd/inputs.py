"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.

This module only draws random numbers and lays them out; it holds none of the
transform's arithmetic.  Coefficients are complex f°(l, m, m') in the l-major
layout (flat index l(4l^2-1)/3 + (m+l)(2l+1) + (m'+l), 0 <= l < B), grids are
complex [2B, 2B, 2B] arrays indexed [alpha_i, beta_j, gamma_k].  All
generators use numpy's PCG64 (``numpy.random.default_rng(seed)``).

The paper's own benchmark inputs are not stated, so these stand in for them:
  * uniform[-1, 1] real and imaginary parts (the small round-trip case),
  * i.i.d. normal parts scaled by (1 + l)^-p (band-limited data whose
    spectrum decays like that of smooth densities; p = 1 by default),
  * batches of bandwidths drawn uniformly from a set,
  * spherical-harmonic coefficient pairs a^l_m, b^l_m for rotational matching.
"""
import numpy as np


def num_coeffs(B):
    """Number of SO(3) coefficients of bandwidth B: B(4B^2 - 1)/3."""
    return B * (4 * B * B - 1) // 3


def degrees(B):
    """Degree l of every flat coefficient index (block l holds (2l+1)^2)."""
    return np.repeat(np.arange(B), [(2 * l + 1) ** 2 for l in range(B)])


def coeffs_uniform(B, seed):
    """Real and imaginary parts i.i.d. uniform[-1, 1]."""
    rng = np.random.default_rng(seed)
    n = num_coeffs(B)
    re = rng.uniform(-1.0, 1.0, n)
    im = rng.uniform(-1.0, 1.0, n)
    return re + 1j * im


def coeffs_decay(B, seed, power=1.0, rng=None):
    """Real and imaginary parts i.i.d. N(0, 1), scaled by (1 + l)^-power."""
    if rng is None:
        rng = np.random.default_rng(seed)
    n = num_coeffs(B)
    re = rng.standard_normal(n)
    im = rng.standard_normal(n)
    return (re + 1j * im) * (1.0 + degrees(B)) ** (-power)


def grid_random(B, seed):
    """A random (not band-limited) complex grid, parts i.i.d. N(0, 1)."""
    rng = np.random.default_rng(seed)
    N = 2 * B
    return rng.standard_normal((N, N, N)) + 1j * rng.standard_normal((N, N, N))


def uneven_batch(n, choices, seed, power=1.0):
    """n functions with bandwidths drawn uniformly from ``choices``.

    The bandwidths are drawn first, then the coefficients function by function
    from the same generator.  Returns (list of B, list of coefficient arrays).
    """
    rng = np.random.default_rng(seed)
    Bs = [int(b) for b in rng.choice(np.asarray(choices), size=n)]
    cs = [coeffs_decay(B, None, power, rng=rng) for B in Bs]
    return Bs, cs


def sh_pair_batch(n, B, seed, power=1.5):
    """n pairs of spherical-harmonic coefficient vectors a^l_m, b^l_m.

    Each vector has B^2 entries in the order (l, m) -> l^2 + (m + l), parts
    i.i.d. N(0, 1) scaled by (1 + l)^-power.  Returns arrays [n, B^2] x 2.
    """
    rng = np.random.default_rng(seed)
    l = np.repeat(np.arange(B), [2 * k + 1 for k in range(B)])
    scale = (1.0 + l) ** (-power)

    def draw():
        return (rng.standard_normal((n, B * B)) + 1j * rng.standard_normal((n, B * B))) * scale

    return draw(), draw()
