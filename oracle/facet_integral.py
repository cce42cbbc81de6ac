"""Closed-form physical-optics integral over one flat triangle (test infrastructure).

Section 2.2 describes BART only as analytic ray tracing whose forward (from TX) and
backward (from RX) rays meet on a facet; the paper gives no formula for the facet
response. Reading used here (single-bounce physical optics with the exact flat-
triangle integral of Gordon's type):

    I_f(k) = integral over triangle T of exp(j k w . (r - c)) dA
           = 2 A * Phi(k b0, k b1, k b2),   b_i = w . (x_i - c),

where w = u_t + u_r is the sum of the unit vectors from the facet centroid c to the
Tx and Rx phase centres, A the area, x_i the vertices. By the Hermite-Genocchi
formula Phi is the second divided difference of F(x) = -exp(jx) at the three nodes
a_i = k b_i. Four equal forms are provided; `phi` picks the stable one.
"""
from __future__ import annotations

import math

import numpy as np


def _sinc(u):
    return np.sinc(np.asarray(u) / np.pi)  # sin(u)/u with sinc(0) = 1


def _first_dd(x, y):
    """First divided difference of -exp(jx): -j exp(j(x+y)/2) sinc((y-x)/2)."""
    return -1j * np.exp(0.5j * (x + y)) * _sinc(0.5 * (y - x))


def phi_sinc(a: np.ndarray) -> np.ndarray:
    """Divided-difference form with the largest-gap pair as divisor:
    Phi = (F[a_l, a_j] - F[a_l, a_i]) / (a_j - a_i), (i, j) the pair farthest apart.
    Undefined when all three nodes coincide."""
    a = np.asarray(a, np.float64)
    gaps = np.stack([np.abs(a[..., 1] - a[..., 2]), np.abs(a[..., 0] - a[..., 2]),
                     np.abs(a[..., 0] - a[..., 1])], -1)
    l = np.argmax(gaps, axis=-1)  # node left out of the widest pair
    i = np.where(l == 0, 1, 0)
    j = np.where(l == 2, 1, 2)
    al = np.take_along_axis(a, l[..., None], -1)[..., 0]
    ai = np.take_along_axis(a, i[..., None], -1)[..., 0]
    aj = np.take_along_axis(a, j[..., None], -1)[..., 0]
    return (_first_dd(al, aj) - _first_dd(al, ai)) / (aj - ai)


def phi_series(a: np.ndarray, order: int = 12) -> np.ndarray:
    """Taylor series about the node mean m: Phi = exp(jm) sum_n j^n h_n(b) / (n+2)!,
    b = a - m, h_n the complete homogeneous symmetric polynomial of degree n
    (written out as the sum of b0^p b1^q b2^r over p+q+r = n)."""
    a = np.asarray(a, np.float64)
    m = a.mean(axis=-1)
    b = a - m[..., None]
    out = np.zeros(a.shape[:-1], np.complex128)
    for n in range(order + 1):
        h = np.zeros(a.shape[:-1])
        for p in range(n + 1):
            for q in range(n + 1 - p):
                r = n - p - q
                h = h + b[..., 0] ** p * b[..., 1] ** q * b[..., 2] ** r
        out = out + (1j ** n) * h / math.factorial(n + 2)
    return np.exp(1j * m) * out


def phi_vertex(a: np.ndarray) -> np.ndarray:
    """Vertex form -sum_i exp(j a_i) / prod_{l != i} (a_i - a_l); needs distinct nodes
    and loses accuracy as they approach each other (near-specular facets)."""
    a = np.asarray(a, np.float64)
    out = np.zeros(a.shape[:-1], np.complex128)
    for i in range(3):
        den = np.ones(a.shape[:-1])
        for l in range(3):
            if l != i:
                den = den * (a[..., i] - a[..., l])
        out = out - np.exp(1j * a[..., i]) / den
    return out


def phi(a: np.ndarray, threshold: float = 1e-3, order: int = 12) -> np.ndarray:
    """Stable Phi: the sinc form when the widest node gap is >= threshold, otherwise
    the series (order 12 leaves a remainder far below FP64 rounding there)."""
    a = np.asarray(a, np.float64)
    gap = np.max(np.stack([np.abs(a[..., 1] - a[..., 2]), np.abs(a[..., 0] - a[..., 2]),
                           np.abs(a[..., 0] - a[..., 1])], -1), axis=-1)
    out = np.empty(a.shape[:-1], np.complex128)
    small = gap < threshold
    if np.any(~small):
        out[~small] = phi_sinc(a[~small])
    if np.any(small):
        out[small] = phi_series(a[small], order)
    return out


def facet_integral(k, beta: np.ndarray, area) -> np.ndarray:
    """I_f(k) = 2 A Phi(k beta_0, k beta_1, k beta_2) for wavenumbers k (any shape
    broadcasting against beta[..., 0])."""
    k = np.asarray(k, np.float64)
    a = k[..., None] * np.asarray(beta, np.float64)
    return 2.0 * np.asarray(area) * phi(a)


def gordon_integral(wvec: np.ndarray, tri: np.ndarray) -> complex:
    """Edge-sum (Gordon) form of the same integral for one triangle [3,3] and a
    phase-gradient vector w (rad/m): with n the unit normal, w_t the in-plane part
    of w, e_m the edge from vertex m to m+1 and r_m its midpoint,
        I = 1/(j |w_t|^2) sum_m ((n x w_t) . e_m) sinc(w . e_m / 2) exp(j w.(r_m - c)).
    From the divergence theorem in the facet plane; needs w_t != 0."""
    tri = np.asarray(tri, np.float64)
    w = np.asarray(wvec, np.float64)
    c = tri.mean(axis=0)
    nvec = np.cross(tri[1] - tri[0], tri[2] - tri[0])
    n = nvec / np.linalg.norm(nvec)
    wt = w - np.dot(w, n) * n
    s = 0.0 + 0.0j
    for m in range(3):
        e = tri[(m + 1) % 3] - tri[m]
        r = 0.5 * (tri[(m + 1) % 3] + tri[m])
        s += np.dot(np.cross(n, wt), e) * _sinc(0.5 * np.dot(w, e)) * np.exp(
            1j * np.dot(w, r - c))
    return s / (1j * np.dot(wt, wt))


def quadrature_integral(wvec: np.ndarray, tri: np.ndarray, n: int = 200) -> complex:
    """Brute-force quadrature of the same integral: Duffy map of the triangle onto
    the unit square, n x n Gauss-Legendre points."""
    tri = np.asarray(tri, np.float64)
    w = np.asarray(wvec, np.float64)
    c = tri.mean(axis=0)
    e1, e2 = tri[1] - tri[0], tri[2] - tri[0]
    two_a = np.linalg.norm(np.cross(e1, e2))
    x, wt = np.polynomial.legendre.leggauss(n)
    x = 0.5 * (x + 1.0)
    wt = 0.5 * wt
    s, u = np.meshgrid(x, x, indexing="ij")
    ws, wu = np.meshgrid(wt, wt, indexing="ij")
    t = (1.0 - s) * u
    pts = tri[0] + s[..., None] * e1 + t[..., None] * e2
    f = np.exp(1j * ((pts - c) @ w))
    return complex(two_a * np.sum(f * (1.0 - s) * ws * wu))
