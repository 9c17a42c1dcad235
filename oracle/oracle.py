"""ctypes binding of the CPU oracle (oracle/so3_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
CPU-baseline leg of bench.py.  Nothing in the GPU library imports it.

All arrays are numpy; complex data is complex128 (the C side sees interleaved
doubles).  ``prec`` selects the double build ("f64") or the x87 long-double
build ("f80"); both take and return doubles.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)

_SIGS = {
    "so3o_weights": [ctypes.c_int, _dp],
    "so3o_wigner_d": [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp],
    "so3o_wigner_d_grid": [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp],
    "so3o_dft2": [ctypes.c_int, ctypes.c_int, _dp],
    "so3o_forward": [ctypes.c_int, _dp, _dp],
    "so3o_inverse": [ctypes.c_int, _dp, _dp],
    "so3o_adjoint": [ctypes.c_int, _dp, _dp],
    "so3o_adjoint_inverse": [ctypes.c_int, _dp, _dp],
    "so3o_separation_forward": [ctypes.c_int, _dp, _dp],
    "so3o_idwt": [ctypes.c_int, _dp, _dp],
    "so3o_inverse_slice": [ctypes.c_int, _dp, ctypes.c_int, _dp],
    "so3o_forward_pairs": [ctypes.c_int, _dp, ctypes.c_int, _ip, _dp],
    "so3o_num_threads": [],
}


def lib():
    """Load (building on first use if needed) the oracle shared library."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _build
            _build.build()
        _lib = ctypes.CDLL(_LIB_PATH)
        for name, args in _SIGS.items():
            for suf in ("_f64", "_f80"):
                fn = getattr(_lib, name + suf)
                fn.argtypes = args
                fn.restype = ctypes.c_int
    return _lib


def _fn(name, prec):
    if prec not in ("f64", "f80"):
        raise ValueError("prec must be 'f64' or 'f80'")
    return getattr(lib(), f"{name}_{prec}")


def _ptr(a):
    return a.ctypes.data_as(_dp)


def _c128(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a


def _check(rc, name):
    if rc != 0:
        raise RuntimeError(f"oracle {name} failed with status {rc}")


def num_coeffs(B):
    """B(4B^2-1)/3 coefficients for bandwidth B (Sect. 2.4)."""
    return B * (4 * B * B - 1) // 3


def coeff_index(l, m, mp):
    """Flat index of f°(l, m, m') in the l-major layout."""
    return l * (4 * l * l - 1) // 3 + (m + l) * (2 * l + 1) + (mp + l)


def num_threads(prec="f64"):
    return int(_fn("so3o_num_threads", prec)())


def weights(B, prec="f64"):
    """Quadrature weights w_B(j), j < 2B (eq. "weights")."""
    w = np.empty(2 * B)
    _check(_fn("so3o_weights", prec)(B, _ptr(w)), "weights")
    return w


def wigner_d(B, m, mp, beta, prec="f64"):
    """d(l, m, m'; beta) for l < B by seeds + three-term recurrence."""
    d = np.empty(B)
    _check(_fn("so3o_wigner_d", prec)(B, m, mp, float(beta), _ptr(d)), "wigner_d")
    return d


def wigner_d_grid(B, m, mp, j, prec="f64"):
    """d(l, m, m'; beta_j) for l < B with beta_j = (2j+1)pi/(4B) formed in the
    oracle's working precision."""
    d = np.empty(B)
    _check(_fn("so3o_wigner_d_grid", prec)(B, m, mp, j, _ptr(d)), "wigner_d_grid")
    return d


def dft2(a, sign, prec="f64"):
    """Unnormalised 2-D DFT exp(sign 2 pi i (pq)/n) of a square complex array."""
    a = _c128(a).copy()
    n = a.shape[0]
    assert a.shape == (n, n)
    _check(_fn("so3o_dft2", prec)(n, sign, _ptr(a.view(np.float64))), "dft2")
    return a


def _grid_shape(B):
    return (2 * B, 2 * B, 2 * B)


def forward(B, grid, prec="f64"):
    """FSOFT: grid [2B,2B,2B] complex -> coefficients [B(4B^2-1)/3] complex."""
    g = _c128(grid).reshape(-1)
    assert g.size == (2 * B) ** 3
    c = np.empty(num_coeffs(B), np.complex128)
    _check(_fn("so3o_forward", prec)(B, _ptr(g.view(np.float64)), _ptr(c.view(np.float64))), "forward")
    return c


def inverse(B, coeffs, prec="f64"):
    """iFSOFT: coefficients -> grid [2B,2B,2B] complex."""
    c = _c128(coeffs).reshape(-1)
    assert c.size == num_coeffs(B)
    g = np.empty(_grid_shape(B), np.complex128)
    _check(_fn("so3o_inverse", prec)(B, _ptr(c.view(np.float64)), _ptr(g.view(np.float64))), "inverse")
    return g


def adjoint(B, coeffs, prec="f64"):
    """F^H = W I V: adjoint of the forward transform."""
    c = _c128(coeffs).reshape(-1)
    assert c.size == num_coeffs(B)
    g = np.empty(_grid_shape(B), np.complex128)
    _check(_fn("so3o_adjoint", prec)(B, _ptr(c.view(np.float64)), _ptr(g.view(np.float64))), "adjoint")
    return g


def adjoint_inverse(B, grid, prec="f64"):
    """I^H = V^-1 F W^-1: adjoint of the inverse transform."""
    g = _c128(grid).reshape(-1)
    assert g.size == (2 * B) ** 3
    c = np.empty(num_coeffs(B), np.complex128)
    _check(_fn("so3o_adjoint_inverse", prec)(B, _ptr(g.view(np.float64)), _ptr(c.view(np.float64))),
           "adjoint_inverse")
    return c


def separation_forward(B, grid, prec="f64"):
    """S(m, m'; j) unweighted, shape [2B-1, 2B-1, 2B] indexed [m+B-1, m'+B-1, j]."""
    g = _c128(grid).reshape(-1)
    P, N = 2 * B - 1, 2 * B
    S = np.empty((P, P, N), np.complex128)
    _check(_fn("so3o_separation_forward", prec)(B, _ptr(g.view(np.float64)), _ptr(S.view(np.float64))),
           "separation_forward")
    return S


def idwt(B, coeffs, prec="f64"):
    """S'(j; m, m') = sum_l d f°, shape [2B-1, 2B-1, 2B] indexed [m+B-1, m'+B-1, j]."""
    c = _c128(coeffs).reshape(-1)
    P, N = 2 * B - 1, 2 * B
    S = np.empty((P, P, N), np.complex128)
    _check(_fn("so3o_idwt", prec)(B, _ptr(c.view(np.float64)), _ptr(S.view(np.float64))), "idwt")
    return S


def inverse_slice(B, coeffs, j, prec="f64"):
    """f(alpha_i, beta_j, gamma_k) for all (i, k): one beta-slice of the inverse."""
    c = _c128(coeffs).reshape(-1)
    N = 2 * B
    s = np.empty((N, N), np.complex128)
    _check(_fn("so3o_inverse_slice", prec)(B, _ptr(c.view(np.float64)), int(j), _ptr(s.view(np.float64))),
           "inverse_slice")
    return s


def forward_pairs(B, grid, pairs, prec="f64"):
    """f°(l, m, m') for l < B of the listed (m, m') pairs: array [npairs, B]."""
    g = _c128(grid).reshape(-1)
    assert g.size == (2 * B) ** 3
    p = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    out = np.empty((p.shape[0], B), np.complex128)
    _check(_fn("so3o_forward_pairs", prec)(B, _ptr(g.view(np.float64)), p.shape[0],
                                           p.ctypes.data_as(_ip), _ptr(out.view(np.float64))),
           "forward_pairs")
    return out


# ---------------------------------------------------------------------------
# Rotational-matching head (correlation of two functions on the sphere,
# the application motivated in Sect. 1): plain definitions in numpy.
# ---------------------------------------------------------------------------

def sh_index(l, m):
    """Position of the spherical-harmonic coefficient (l, m) in a vector of
    B^2 entries ordered by degree, then order m = -l..l."""
    return l * l + m + l


def correlation_coeffs(B, a, b):
    """SO(3) coefficients of the correlation of two functions on the sphere:
    f°(l, M, M') = a(l, M) * conj(b(l, M')), for 0 <= l < B, |M|, |M'| <= l,
    in the layout of ``coeff_index``.  a, b: B^2 complex coefficients each."""
    a = _c128(a).reshape(-1)
    b = _c128(b).reshape(-1)
    assert a.size == b.size == B * B
    out = np.empty(num_coeffs(B), np.complex128)
    for l in range(B):
        al = a[l * l:(l + 1) * (l + 1)]
        bl = b[l * l:(l + 1) * (l + 1)]
        o = coeff_index(l, -l, -l)
        # row M, column M': a(l, M) conj(b(l, M'))
        out[o:o + (2 * l + 1) ** 2] = np.outer(al, np.conj(bl)).reshape(-1)
    return out


def correlation_coeffs_vjp(B, a, b, g):
    """Vector-Jacobian product of ``correlation_coeffs`` in the convention of
    complex autograd (gradients are conjugate Wirtinger derivatives):
    ga(l, M) = sum_M' g(l, M, M') b(l, M'),  gb(l, M') = sum_M conj(g(l, M, M')) a(l, M)."""
    a = _c128(a).reshape(-1)
    b = _c128(b).reshape(-1)
    g = _c128(g).reshape(-1)
    ga = np.empty(B * B, np.complex128)
    gb = np.empty(B * B, np.complex128)
    for l in range(B):
        n = 2 * l + 1
        o = coeff_index(l, -l, -l)
        G = g[o:o + n * n].reshape(n, n)
        ga[l * l:l * l + n] = G @ b[l * l:l * l + n]
        gb[l * l:l * l + n] = np.conj(G).T @ a[l * l:l * l + n]
    return ga, gb


def argmax_real(grid):
    """Flat index of the largest real part (the first one on exact ties)."""
    return int(np.argmax(np.asarray(grid).real.reshape(-1)))


# ---------------------------------------------------------------------------
# Functions on the sphere (the rotational-matching application of Sect. 1)
# ---------------------------------------------------------------------------

def sh_forward(B, f):
    """Spherical-harmonic coefficients of a function on the sphere sampled at
    (theta_j, phi_k) = ((2j+1) pi/(4B), k pi/B), j, k < 2B (the beta and
    alpha samples of the sampling theorem, Sect. 2.3, at m' = 0):
        a(l, m) = sum_{j,k} w_B(j) f[j, k] conj(Y(l, m; theta_j, phi_k)),
        Y(l, m; theta, phi) = sqrt((2l+1)/(4 pi)) e^{i m phi} d(l, 0, m; theta),
    d as defined in Sect. 2.2 (d(l, 0, m) is the textbook d^l_{m0}, so Y is
    the orthonormal spherical harmonic with the Condon-Shortley phase).  The
    quadrature is exact for functions of degree < B.  Returns B^2 complex
    values, (l, m) at l^2 + m + l."""
    f = _c128(f)
    N = 2 * B
    assert f.shape == (N, N)
    w = weights(B)
    phi = np.arange(N) * np.pi / B
    a = np.zeros(B * B, np.complex128)
    for m in range(1 - B, B):
        F = (f * np.exp(-1j * m * phi)[None, :]).sum(axis=1)
        for j in range(N):
            d = wigner_d_grid(B, 0, m, j)
            for l in range(abs(m), B):
                a[sh_index(l, m)] += np.sqrt((2 * l + 1) / (4 * np.pi)) * w[j] * d[l] * F[j]
    return a


def rotation_of_index(B, idx):
    """Euler angles (alpha, beta, gamma) of the rotation R = Rz(alpha) Ry(beta)
    Rz(gamma) read off the correlation grid of a = coefficients of f and
    b = coefficients of g: the grid point (alpha_i, beta_j, gamma_k) of flat
    index (i*2B + j)*2B + k is the rotation with g(w) = f(R^-1 w) at
    (alpha, beta, gamma) = (gamma_k, beta_j, alpha_i) (the roles of the
    outer angles swap because d(l, m, m') of Sect. 2.2 is the transpose of
    the textbook d^l_{m m'})."""
    N = 2 * B
    i, j, k = idx // (N * N), (idx // N) % N, idx % N
    return (k * np.pi / B, (2 * j + 1) * np.pi / (4 * B), i * np.pi / B)


def refine_quadratic(B, grid, idx):
    """Sub-grid refinement of a correlation maximum: along each grid axis a
    parabola through Re C at the maximum and its two neighbours (periodic in
    alpha and gamma; none at the first and last beta sample) moves the grid
    coordinate by (c- - c+) / (2 (c- - 2 c0 + c+)), clamped to [-1/2, 1/2],
    and the moved coordinates are read as in ``rotation_of_index``.  Returns
    (alpha, beta, gamma)."""
    N = 2 * B
    g = np.asarray(grid).reshape(N, N, N).real
    i, j, k = idx // (N * N), (idx // N) % N, idx % N
    c0 = g[i, j, k]

    def step(cm, cp):
        den = cm - 2.0 * c0 + cp
        if not den < 0.0:
            return 0.0
        return min(0.5, max(-0.5, (cm - cp) / (2.0 * den)))

    di = step(g[(i - 1) % N, j, k], g[(i + 1) % N, j, k])
    dk = step(g[i, j, (k - 1) % N], g[i, j, (k + 1) % N])
    dj = step(g[i, j - 1, k], g[i, j + 1, k]) if 0 < j < N - 1 else 0.0
    return ((k + dk) * np.pi / B, (2 * (j + dj) + 1) * np.pi / (4 * B), (i + di) * np.pi / B)


def corr_eval(B, fo, alpha, beta, gamma, prec="f64"):
    """The SO(3) function with coefficients fo at an arbitrary point:
        C(alpha, beta, gamma) = sum_{l,m,m'} fo(l,m,m') e^{-i m alpha}
                                d(l,m,m';beta) e^{-i m' gamma},
    the sum of eq. "fourier_representation" that the inverse transform
    evaluates at the grid points (alpha_i, beta_j, gamma_k); d by the seeds
    and recurrence of Sect. 2.2 at this beta.  A beta outside [0, pi] names
    the same rotation as (alpha + pi, beta', gamma - pi) with beta' = -beta
    or 2 pi - beta (Rz(pi) Ry(b) Rz(-pi) = Ry(-b)), so it is evaluated there."""
    fo = _c128(fo).reshape(-1)
    beta = float(np.mod(beta, 2 * np.pi))
    if beta > np.pi:
        alpha, beta, gamma = alpha + np.pi, 2 * np.pi - beta, gamma - np.pi
    tot = 0j
    for m in range(1 - B, B):
        for mp in range(1 - B, B):
            l0 = max(abs(m), abs(mp))
            ls = np.arange(l0, B)
            d = wigner_d(B, m, mp, beta, prec)[l0:]
            tot += np.exp(-1j * (m * alpha + mp * gamma)) * np.dot(d, fo[coeff_index(ls, m, ls * 0 + mp)])
    return tot


def _rz(a):
    c, s_ = np.cos(a), np.sin(a)
    return np.array([[c, -s_, 0.0], [s_, c, 0.0], [0.0, 0.0, 1.0]])


def _ry(b):
    c, s_ = np.cos(b), np.sin(b)
    return np.array([[c, 0.0, s_], [0.0, 1.0, 0.0], [-s_, 0.0, c]])


def _expso3(w):
    """Rotation matrix exp([w]x) (Rodrigues)."""
    t = np.sqrt(w @ w)
    K = np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])
    if t < 1e-300:
        return np.eye(3)
    return np.eye(3) + np.sin(t) / t * K + 2.0 * np.sin(0.5 * t) ** 2 / (t * t) * (K @ K)


def zyz_of(Q):
    """Angles (a, b, c), b in [0, pi], with Q = Rz(a) Ry(b) Rz(c); on the
    axis (sin b = 0) c = 0 and a carries the whole turn."""
    sb = np.hypot(Q[0, 2], Q[1, 2])
    b = np.arctan2(sb, Q[2, 2])
    if sb > 0.0:
        return np.arctan2(Q[1, 2], Q[0, 2]), b, np.arctan2(Q[2, 1], -Q[2, 0])
    if Q[2, 2] > 0:
        return np.arctan2(Q[1, 0], Q[0, 0]), b, 0.0
    return np.arctan2(-Q[1, 0], -Q[0, 0]), b, 0.0


def corr_at(B, fo, Q, prec="f64"):
    """C at the rotation Q: the rotation read off grid index (i, j, k) is
    Rz(gamma_k) Ry(beta_j) Rz(alpha_i) (rotation_of_index), so C is
    evaluated at (alpha, beta, gamma) = (c, b, a) of Q's angles (a, b, c)."""
    a, b, c = zyz_of(Q)
    return corr_eval(B, fo, c, b, a, prec)


def polish_rotation(B, fo, start, iters=8, prec="f64"):
    """Off-grid refinement of a correlation maximum by Newton steps on
    F(w) = Re C(Q0 exp([w]x)), local rotation-vector coordinates w around
    the current rotation Q0 (no pole of Euler angles on the way).  Q0 starts
    at Rz(a) Ry(b) Rz(c) for start = (a, b, c).  Each step samples F at w = 0,
    +-h e_i and h (e_i + e_j), i < j (ten points: the quadratic model through
    them is exact for quadratics), takes g_i = (F(h e_i) - F(-h e_i)) / 2h,
    H_ii = (F(h e_i) - 2 F(0) + F(-h e_i)) / h^2 and H_ij from F(h e_i + h e_j);
    steps by -H^-1 g when -H is positive definite (its Cholesky factor exists)
    and otherwise by -g_i / H_ii per axis (or h toward larger F where
    H_ii >= 0), clamps each component to [-h, h], sets Q0 = Q0 exp([step]x)
    and h = min(h, max(1e-5, 2 max|step|)); h starts at pi/(4B).  Returns the
    angles (a, b, c) of the final rotation (a, c in [0, 2 pi), b in [0, pi])
    and Re C there."""
    Q0 = _rz(start[0]) @ _ry(start[1]) @ _rz(start[2])
    h = np.pi / (4 * B)
    E = np.eye(3)
    val = 0.0
    for it in range(iters + 1):
        F0 = corr_at(B, fo, Q0, prec).real
        if it == iters:
            val = F0
            break
        Fp = [corr_at(B, fo, Q0 @ _expso3(h * E[i]), prec).real for i in range(3)]
        Fm = [corr_at(B, fo, Q0 @ _expso3(-h * E[i]), prec).real for i in range(3)]
        g = np.array([(Fp[i] - Fm[i]) / (2 * h) for i in range(3)])
        H = np.diag([(Fp[i] - 2 * F0 + Fm[i]) / (h * h) for i in range(3)])
        for i, j in ((0, 1), (0, 2), (1, 2)):
            Fij = corr_at(B, fo, Q0 @ _expso3(h * (E[i] + E[j])), prec).real
            H[i, j] = H[j, i] = (Fij - F0 - h * (g[i] + g[j]) - 0.5 * h * h * (H[i, i] + H[j, j])) / (h * h)
        A = -H
        ok = A[0, 0] > 0
        if ok:
            l00 = np.sqrt(A[0, 0])
            l10, l20 = A[1, 0] / l00, A[2, 0] / l00
            r11 = A[1, 1] - l10 * l10
            ok = r11 > 0
        if ok:
            l11 = np.sqrt(r11)
            l21 = (A[2, 1] - l20 * l10) / l11
            r22 = A[2, 2] - l20 * l20 - l21 * l21
            ok = r22 > 0
        if ok:
            l22 = np.sqrt(r22)
            y0 = g[0] / l00
            y1 = (g[1] - l10 * y0) / l11
            y2 = (g[2] - l20 * y0 - l21 * y1) / l22
            d2 = y2 / l22
            d1 = (y1 - l21 * d2) / l11
            d0 = (y0 - l10 * d1 - l20 * d2) / l00
            step = np.array([d0, d1, d2])
        else:
            step = np.array([-g[i] / H[i, i] if H[i, i] < 0 else (h if g[i] >= 0 else -h) for i in range(3)])
        step = np.clip(step, -h, h)
        Q0 = Q0 @ _expso3(step)
        h = min(h, max(1e-5, 2 * np.abs(step).max()))
    a, b, c = zyz_of(Q0)
    two_pi = 2 * np.pi
    return (float(np.mod(a, two_pi)), float(b), float(np.mod(c, two_pi))), float(val)
