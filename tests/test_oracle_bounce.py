"""Pins of the ground double bounce (image method, oracle/bounce.py): a point above the
road against path lengths from the law of reflection, reciprocity, and visibility of
the reflected legs on constructed geometry."""
import numpy as np
import pytest

import oracle
import scenes
from oracle import bounce
from scenes import Instance, Mesh, RadarArray, Scene

C = 299792458.0


def _reflected_length(a, b, z_g):
    """|a - S| + |S - b| with S on z = z_g where the angles of incidence and reflection
    are equal (similar triangles on the heights above the plane)."""
    ha, hb = a[2] - z_g, b[2] - z_g
    s = ha / (ha + hb)
    S = a + s * (b - a)
    S[2] = z_g
    return np.linalg.norm(a - S) + np.linalg.norm(S - b)


def test_point_above_ground_four_paths():
    wf = scenes.paper_waveform(64, 2)
    e_t = np.array([0.4, 0.0, 6.0])
    e_r = np.array([-0.3, 0.0, 5.5])
    arr = RadarArray(tx=e_t[None].copy(), rx=e_r[None].copy())
    x = np.array([3.0, 25.0, 1.2])
    amp = 1.5 - 0.5j
    sc = Scene(meshes=[], instances=[],
               points=scenes.Points(pos0=x[None], vel=np.zeros((1, 3)), amp=np.array([amp])))
    gamma = -0.8 + 0.1j
    z_g = 0.2
    H = bounce.synthesize_bounce(sc, wf, arr, z_g=z_g, gamma=gamma)[0]
    f = wf.f0 + np.arange(wf.n_samples) * wf.slope / wf.fs
    legs_t = [np.linalg.norm(e_t - x), _reflected_length(e_t, x, z_g)]
    legs_r = [np.linalg.norm(e_r - x), _reflected_length(e_r, x, z_g)]
    expect = 0.0
    for k in range(4):
        lt, lr = legs_t[k & 1], legs_r[k >> 1]
        tau = (lt + lr) / C
        g = gamma ** ((k & 1) + (k >> 1))
        expect = expect + g * amp / (4 * np.pi * lt * lr) * np.exp(
            -2j * np.pi * (f * tau - 0.5 * wf.slope * tau * tau))
    for n in range(wf.n_chirps):
        assert np.max(np.abs(H[n] - expect)) <= 1e-10 * np.max(np.abs(expect))


def test_bounce_reciprocity_swap_tx_rx():
    cfg = scenes.small_single(n_tris=400, n_samples=16, n_chirps=1, mimo=False)
    sc, wf, arr = cfg.scenes[0], cfg.waveform, cfg.array
    a = bounce.synthesize_bounce(sc, wf, arr)
    b = bounce.synthesize_bounce(sc, wf, RadarArray(tx=arr.rx, rx=arr.tx))
    # channel o = p Q + q of one equals q P + p of the other
    P, Q = arr.tx.shape[0], arr.rx.shape[0]
    perm = [q * P + p for p in range(P) for q in range(Q)]
    assert np.max(np.abs(a - b[perm])) <= 1e-12 * np.max(np.abs(a))


def _plate(y, z, half=0.4):
    """A vertical square facing -y (toward the radar) at distance y, centre height z."""
    v = np.array([[-half, 0, -half], [half, 0, -half], [half, 0, half], [-half, 0, half]],
                 np.float32)
    t = np.array([[0, 1, 2], [0, 2, 3]], np.int32)  # normal -y
    return Mesh(verts=v, tris=t), np.array([0.0, y, z])


def test_reflected_legs_blocked_by_an_awning():
    """A plate at 20 m, 1 m up; the radar at 6 m. The reflected ray meets the ground near
    y = 17.1 m; a horizontal sheet at 0.3 m over y in [16, 18.5] blocks both reflected
    legs' lower parts but not the direct rays: only type 0 stays lit."""
    wf = scenes.paper_waveform(16, 1)
    e = scenes.RADAR_POS.astype(np.float64)
    arr = RadarArray(tx=e[None].copy(), rx=e[None].copy())
    pm, pp = _plate(20.0, 1.0)
    sheet = Mesh(verts=np.array([[-1, 16, 0.3], [1, 16, 0.3], [1, 18.5, 0.3], [-1, 18.5, 0.3]],
                                np.float32), tris=np.array([[0, 1, 2], [0, 2, 3]], np.int32))
    eye = np.eye(3)
    open_sc = Scene(meshes=[pm], instances=[Instance(0, eye, pp, np.zeros(3))])
    m, amb = bounce.visibility_bounce(open_sc, arr, wf)
    assert m[:, 0, :2].all() and not amb.any()
    roofed = Scene(meshes=[pm, sheet], instances=[Instance(0, eye, pp, np.zeros(3)),
                                                  Instance(1, eye, np.zeros(3), np.zeros(3))])
    m, amb = bounce.visibility_bounce(roofed, arr, wf)
    assert m[0, 0, :2].all() and not m[1:, 0, :2].any() and not amb[:, 0, :2].any()
    # the sheet faces up: lit directly and by the image paths it faces (types whose
    # sides all see its top); the plate's type-0 term is unchanged by the sheet
    single, _ = oracle.visibility(roofed, arr, wf)
    assert np.array_equal(single[0], m[0, 0])


def test_road_surface_does_not_block_reflected_legs():
    """A ground grid lying in the plane: its triangles take no image paths (centroids not
    above the plane) and do not block the legs that end on it."""
    wf = scenes.paper_waveform(16, 1)
    e = scenes.RADAR_POS.astype(np.float64)
    arr = RadarArray(tx=e[None].copy(), rx=e[None].copy())
    pm, pp = _plate(20.0, 1.0)
    road = scenes.ground_grid(-3.0, 3.0, 14.0, 22.0, 1.0)
    eye = np.eye(3)
    sc = Scene(meshes=[pm, road], instances=[Instance(0, eye, pp, np.zeros(3)),
                                             Instance(1, eye, np.zeros(3), np.zeros(3))])
    assert list(bounce.in_plane_instances(sc, 0.0)) == [False, True]
    m, amb = bounce.visibility_bounce(sc, arr, wf)
    assert m[:, 0, :2].all() and not amb[:, 0, :2].any()
    assert not m[1:, 0, 2:].any()  # road facets: no image paths

