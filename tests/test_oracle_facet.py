"""Pins of the oracle's facet integral against quadrature, closed forms and the
edge-sum form (no GPU)."""
import numpy as np
import pytest

import oracle


def _rand_tri(rng, size=0.05):
    return rng.normal(size=(3, 3)) * size


def _area(tri):
    return 0.5 * np.linalg.norm(np.cross(tri[1] - tri[0], tri[2] - tri[0]))


@pytest.mark.parametrize("k", [0.3, 30.0, 400.0, 1700.0])
def test_integral_matches_quadrature_and_edge_sum(k):
    rng = np.random.default_rng(int(k * 10))
    for _ in range(4):
        tri = _rand_tri(rng)
        w = rng.normal(size=3)
        w *= rng.uniform(0.2, 2.0) / np.linalg.norm(w)
        c = tri.mean(axis=0)
        beta = (tri - c) @ w
        val = complex(oracle.facet_integral(np.array(k), beta, _area(tri)))
        quad = oracle.quadrature_integral(k * w, tri, n=320)
        edge = oracle.gordon_integral(k * w, tri)
        scale = _area(tri)
        assert abs(val - quad) < 1e-11 * scale
        assert abs(val - edge) < 1e-11 * scale


def test_specular_limit_and_series():
    # all nodes equal: Phi = exp(ja)/2, so I = A when beta = 0
    a = np.array([[0.7, 0.7, 0.7]])
    assert np.allclose(oracle.phi(a), np.exp(0.7j) / 2, atol=1e-15)
    assert np.isclose(complex(oracle.facet_integral(np.array(5.0), np.zeros(3), 0.25)), 0.25)
    # series and sinc forms agree across the switch-over region
    rng = np.random.default_rng(5)
    for spread in (1e-3, 1e-2, 0.3):
        a = rng.normal(size=(50, 3)) * spread
        assert np.max(np.abs(oracle.phi_series(a, 24) - oracle.phi_sinc(a))) < 1e-12
    # well-separated nodes: vertex form agrees
    a = rng.normal(size=(50, 3)) * 20.0
    assert np.max(np.abs(oracle.phi_vertex(a) - oracle.phi(a))) < 1e-12


def _plate_tris(a, b, tilt):
    """Two triangles of an a x b plate in the x-z plane, rotated by tilt about z."""
    x = np.array([-a / 2, a / 2])
    z = np.array([-b / 2, b / 2])
    corners = np.array([[x[0], 0, z[0]], [x[1], 0, z[0]], [x[1], 0, z[1]], [x[0], 0, z[1]]])
    c, s = np.cos(tilt), np.sin(tilt)
    rot = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])
    corners = corners @ rot.T
    return np.array([corners[[0, 1, 2]], corners[[0, 2, 3]]]), rot @ np.array([0, -1.0, 0])


@pytest.mark.parametrize("tilt_deg", [0.0, 0.3, 2.0, 11.0])
def test_flat_plate_closed_form(tilt_deg):
    """Monostatic plane wave along -y on an a x b plate tilted by theta about its
    b-edge: |o I| = a b cos(theta) |sinc(k a sin(theta))|, i.e.
    sigma = 4 pi / lambda^2 (a b cos(theta) sinc(k a sin theta))^2 and 4 pi A^2 / lambda^2
    at normal incidence."""
    a, b = 0.31, 0.17
    th = np.deg2rad(tilt_deg)
    tris, n_plate = _plate_tris(a, b, th)
    u = np.array([0.0, -1.0, 0.0])  # unit vector from the plate to the radar
    w = 2 * u
    lam = 299792458.0 / 79e9
    k = 2 * np.pi / lam
    total = 0j
    for t in tris:
        cf = t.mean(axis=0)
        nf = np.cross(t[1] - t[0], t[2] - t[0])
        nf /= np.linalg.norm(nf)
        assert np.dot(nf, n_plate) > 0.999
        obl = 0.5 * np.dot(nf, w)
        beta = (t - cf) @ w
        # the facet integral is about the facet centroid: move it to the plate centre
        total += obl * complex(oracle.facet_integral(np.array(k), beta, _area(t))) * np.exp(
            1j * k * np.dot(w, cf))
    expect = a * b * np.cos(th) * np.sinc(k * a * np.sin(th) / np.pi)
    assert abs(abs(total) - abs(expect)) < 1e-12 * a * b
    sigma = 4 * np.pi * abs(total) ** 2 / lam ** 2
    if tilt_deg == 0.0:
        assert np.isclose(sigma, 4 * np.pi * (a * b) ** 2 / lam ** 2, rtol=1e-12, atol=0.0)
