"""Independent brute-force evaluation used to pin the oracle (tests only).

Nothing here shares code with the oracle: the Wigner-d values come from the
paper's explicit Jacobi-polynomial definition (Sect. 2.2) through
``scipy.special.eval_jacobi``, extended to all order pairs with the three
same-angle symmetries of eq. "Wigner_symmetries"; the transforms are the plain
O(B^6) sums of eq. "fourier_representation" and eq. "quadrature"; the weights
are eq. "weights" in numpy.
"""
import math

import numpy as np
from scipy.special import eval_jacobi


def d_explicit(l, m, mp, beta):
    """d(l, m, m'; beta) by the explicit definition, valid for m' >= |m|."""
    assert mp >= abs(m) and l >= mp
    beta = np.asarray(beta, dtype=np.float64)
    norm = math.sqrt(math.factorial(l + mp) / math.factorial(l + m)
                     * math.factorial(l - mp) / math.factorial(l - m))
    sign = -1.0 if (m + mp) % 2 else 1.0
    return (sign * norm * np.sin(beta / 2) ** (mp - m) * np.cos(beta / 2) ** (m + mp)
            * eval_jacobi(l - mp, mp - m, m + mp, np.cos(beta)))


def d_any(l, m, mp, beta):
    """d(l, m, m'; beta) for any |m|, |m'| <= l via the explicit form and the
    same-angle symmetries (m,m') -> (-m,-m'), (m',m), (-m',-m)."""
    if abs(m) > l or abs(mp) > l:
        return np.zeros_like(np.asarray(beta, dtype=np.float64))
    s = -1.0 if (m - mp) % 2 else 1.0
    if mp >= abs(m):
        return d_explicit(l, m, mp, beta)
    if m >= abs(mp):
        return s * d_explicit(l, mp, m, beta)
    if -mp >= abs(m):
        return s * d_explicit(l, -m, -mp, beta)
    return d_explicit(l, -mp, -m, beta)


def weights_np(B):
    """eq. "weights" evaluated in numpy."""
    j = np.arange(2 * B)
    beta = (2 * j + 1) * np.pi / (4 * B)
    i = np.arange(B)[:, None]
    s = (np.sin((2 * i + 1) * beta[None, :]) / (2 * i + 1)).sum(0)
    return 2 * np.pi * np.sin(beta) / B ** 2 * s


def _tables(B):
    N = 2 * B
    ang = np.arange(N) * np.pi / B
    beta = (2 * np.arange(N) + 1) * np.pi / (4 * B)
    lmm = [(l, m, mp) for l in range(B) for m in range(-l, l + 1) for mp in range(-l, l + 1)]
    D = np.array([d_any(l, m, mp, beta) for (l, m, mp) in lmm])          # [c, j]
    M = np.array([m for (_, m, _) in lmm])[:, None]
    MP = np.array([mp for (_, _, mp) in lmm])[:, None]
    Ea = np.exp(-1j * M * ang[None, :])                                  # [c, i]
    Eg = np.exp(-1j * MP * ang[None, :])                                 # [c, k]
    L = np.array([l for (l, _, _) in lmm])
    return D, Ea, Eg, L


def inverse_brute(B, coeffs):
    """f_ijk = sum_{l,m,m'} f° e^{-i m alpha_i} d(l,m,m';beta_j) e^{-i m' gamma_k}."""
    D, Ea, Eg, _ = _tables(B)
    return np.einsum("c,ci,cj,ck->ijk", np.asarray(coeffs), Ea, D, Eg, optimize=True)


def forward_brute(B, grid):
    """f° = (2l+1)/(8 pi B) sum_{ijk} w_B(j) f_ijk conj(D(l,m,m';alpha_i,beta_j,gamma_k))."""
    D, Ea, Eg, L = _tables(B)
    w = weights_np(B)
    s = np.einsum("ijk,ci,cj,ck->c", np.asarray(grid), Ea.conj(), D * w[None, :], Eg.conj(),
                  optimize=True)
    return (2 * L + 1) / (8 * np.pi * B) * s
