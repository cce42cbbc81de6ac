"""Pins of the oracle's echo, beat signal and RDM against the paper's closed forms
(eq. (13), eqs. (4)-(5), Table 2), the radar equation (eq. (7)) and exact invariants
(reciprocity, linearity, subdivision). No GPU."""
import json
import os

import numpy as np
import pytest

import oracle
import scenes
from scenes import Mesh, Instance, RadarArray, Scene, Waveform

C = 299_792_458.0
HERE = os.path.dirname(os.path.abspath(__file__))


def _mono_array():
    p = scenes.RADAR_POS[None, :].astype(np.float64)
    return RadarArray(tx=p.copy(), rx=p.copy())


def test_table2_golden():
    with open(os.path.join(HERE, "golden", "table2.json")) as f:
        gold = json.load(f)
    for row in gold["rows"]:
        d = oracle.table2_row(row["samples"])
        assert round(d["chirp_period"] * 1e6, 6) == row["chirp_period_us"]
        assert np.isclose(d["bandwidth"] / 1e9, row["bandwidth_ghz"], rtol=1e-12, atol=0.0)
        assert round(d["range_resolution"], 2) == row["range_resolution_m"]
        assert round(d["max_velocity"], 2) == row["max_velocity_mps"]
        # design range of 60 m (eq. (4) at the sample rate)
        assert 60.0 <= d["max_range"] < 62.0
    # experiment 3 is 'abnormal': 10 m/s exceeds the unambiguous velocity
    for row in gold["rows"]:
        d = oracle.table2_row(row["samples"])
        abnormal = gold["target"]["speed_mps"] > d["max_velocity"]
        assert abnormal == (gold["rdm_display"][str(row["samples"])] == "abnormal")


def test_point_target_equals_eq13():
    """conj(H) of a point target is the IF signal of eq. (13) at t = m / fs."""
    wf = scenes.paper_waveform(256, 16)
    R, v = 37.3, -4.2
    s = 0.7 - 0.2j
    sc = scenes.point_scene([R], [v], amps=[s])
    H = oracle.synthesize(sc, wf, _mono_array())
    x = oracle.beat(H)[0]
    tm = np.arange(wf.n_samples) / wf.fs
    for n in range(wf.n_chirps):
        Rn = R + v * n * wf.chirp_period
        tau = 2 * Rn / C
        amp = np.conj(s) / (4 * np.pi * Rn * Rn)
        eq13 = amp * np.exp(2j * np.pi * (wf.f0 * tau + wf.slope * tm * tau - 0.5 * wf.slope * tau ** 2))
        assert np.max(np.abs(x[n] - eq13)) < 1e-9 * abs(amp)


def test_static_point_on_bin_is_a_delta():
    """A static point whose beat frequency sits on range bin 100 gives one RDM cell
    of power (M N |a|)^2 at Doppler row N/2 and nothing elsewhere (eq. (4))."""
    wf = scenes.paper_waveform(256, 32)
    d = oracle.derived(wf)
    R = 100 * d["range_resolution"]
    sc = scenes.point_scene([R], [0.0])
    H = oracle.synthesize(sc, wf, _mono_array())
    P, Y = oracle.rdm_from_echo(H)
    peak = (wf.n_samples * wf.n_chirps / (4 * np.pi * R * R)) ** 2
    assert np.isclose(P[0, wf.n_chirps // 2, 100], peak, rtol=1e-9, atol=0.0)
    P0 = P[0].copy()
    P0[wf.n_chirps // 2, 100] = 0
    assert P0.max() < 1e-18 * peak
    # Parseval: sum |Y|^2 = M N sum |x|^2
    assert np.isclose(P.sum(), wf.n_samples * wf.n_chirps * np.sum(np.abs(H) ** 2), rtol=1e-12, atol=0.0)


@pytest.mark.parametrize("lp", [-20, -3, 7])
def test_moving_point_doppler_bin(lp):
    """eq. (5): a range rate of l' velocity resolutions peaks in Doppler row N/2 + l'
    (positive = receding), in range bin 2 R B / c."""
    wf = scenes.paper_waveform(256, 128)
    d = oracle.derived(wf)
    R = 100 * d["range_resolution"]
    v = lp * d["velocity_resolution"]
    H = oracle.synthesize(scenes.point_scene([R], [v]), wf, _mono_array())
    P, _ = oracle.rdm_from_echo(H)
    l, k = np.unravel_index(np.argmax(P[0]), P[0].shape)
    assert (l, k) == (wf.n_chirps // 2 + lp, 100)
    assert np.isclose(oracle.velocity_axis(wf)[l], v, atol=1e-9)


def test_experiment3_doppler_alias():
    """Table 2 experiment 3 (512 samples, 110 us): 10 m/s folds to about -7.55 m/s."""
    wf = scenes.paper_waveform(512, 128)
    d = oracle.derived(wf)
    H = oracle.synthesize(scenes.point_scene([40.0], [10.0]), wf, _mono_array())
    P, _ = oracle.rdm_from_echo(H)
    l, k = np.unravel_index(np.argmax(P[0]), P[0].shape)
    v_seen = oracle.velocity_axis(wf)[l]
    assert abs(v_seen - (10.0 - 2 * d["max_velocity"])) <= d["velocity_resolution"]
    assert abs(oracle.range_axis(wf)[k] - 40.0) <= d["range_resolution"]


def _far_wave(slope=1e6):
    return Waveform(f0=77e9, slope=slope, fs=5.12e6, chirp_period=60e-6, n_samples=8,
                    n_chirps=1)


@pytest.mark.parametrize("tilt_deg", [0.0, 1.5])
def test_plate_radar_equation(tilt_deg):
    """eq. (7) with sigma = 4 pi A^2 / lambda^2 (normal incidence) and
    (4 pi / lambda^2) (a b cos t sinc(k a sin t))^2 (tilted): |H| = sqrt(P)."""
    a, b, D = 0.3, 0.2, 1e6
    wf = _far_wave()
    sc = scenes.plate_scene(a, b, 2, 1, D, tilt_rad=np.deg2rad(tilt_deg))
    H = oracle.synthesize(sc, wf, _mono_array())[0, 0]
    f = wf.f0 + np.arange(wf.n_samples) * wf.slope / wf.fs
    lam = C / f
    k = 2 * np.pi / lam
    th = np.deg2rad(tilt_deg)
    sigma = 4 * np.pi / lam ** 2 * (a * b * np.cos(th) * np.sinc(k * a * np.sin(th) / np.pi)) ** 2
    power = sigma * lam ** 2 / ((4 * np.pi) ** 3 * D ** 4)
    assert np.allclose(np.abs(H), np.sqrt(power), rtol=2e-5, atol=0.0)


def test_subdivision_invariance_far_field():
    """Splitting a planar facet leaves the far-field response unchanged."""
    wf = _far_wave()
    coarse = scenes.plate_scene(0.3, 0.2, 1, 1, 1e6, tilt_rad=0.02)
    fine = scenes.plate_scene(0.3, 0.2, 6, 4, 1e6, tilt_rad=0.02)
    arr = _mono_array()
    Hc = oracle.synthesize(coarse, wf, arr)
    Hf = oracle.synthesize(fine, wf, arr)
    assert np.max(np.abs(Hc - Hf)) < 1e-4 * np.max(np.abs(Hc))


def _small_two_box_scene(sep=True):
    m1 = scenes.box_mesh((-1, -0.5, 0), (1, 0.5, 1.2), (4, 2, 3))
    m2 = scenes.box_mesh((-0.6, -0.4, 0), (0.6, 0.4, 0.9), (3, 2, 2))
    i1 = Instance(0, np.eye(3), np.array([-3.0, 20.0, 0.0]), np.array([0.0, -5.0, 0.0]))
    i2 = Instance(1, scenes.yaw_matrix(0.4), np.array([4.0, 26.0, 0.0]), np.array([1.0, 3.0, 0.0]))
    return Scene([m1, m2], [i1, i2]), Scene([m1], [i1]), Scene([m2], [Instance(0, i2.rot, i2.pos0, i2.vel)])


def test_linearity_separated_meshes():
    wf = scenes.paper_waveform(64, 3)
    arr = scenes.sparse_mimo_12x16(wf, 3)
    both, a, b = _small_two_box_scene()
    Hab = oracle.synthesize(both, wf, arr, channels=np.arange(0, 192, 17))
    Ha = oracle.synthesize(a, wf, arr, channels=np.arange(0, 192, 17))
    Hb = oracle.synthesize(b, wf, arr, channels=np.arange(0, 192, 17))
    assert np.max(np.abs(Hab - Ha - Hb)) < 1e-12 * np.max(np.abs(Hab))


def test_reciprocity_swap_tx_rx():
    """Swapping the Tx and Rx arrays leaves every (Tx element, Rx element) response
    unchanged (H'[q P + p] = H[p Q + q])."""
    wf = scenes.paper_waveform(48, 2)
    rng = np.random.default_rng(9)
    tx = scenes.RADAR_POS + rng.normal(size=(2, 3)) * 0.05
    rx = scenes.RADAR_POS + rng.normal(size=(3, 3)) * 0.05
    both, _, _ = _small_two_box_scene()
    H = oracle.synthesize(both, wf, RadarArray(tx, rx))
    Hs = oracle.synthesize(both, wf, RadarArray(rx, tx))
    for p in range(2):
        for q in range(3):
            assert np.max(np.abs(Hs[q * 2 + p] - H[p * 3 + q])) < 1e-13 * np.max(np.abs(H))


def test_zero_area_triangle_is_inert():
    wf = scenes.paper_waveform(32, 2)
    arr = scenes.ula_1tx4rx(wf)
    m = scenes.box_mesh((-1, -0.5, 0), (1, 0.5, 1), (2, 1, 1))
    verts = np.concatenate([m.verts, np.array([[0, -0.6, 0.5], [0.1, -0.6, 0.5]], np.float32)])
    nv = m.verts.shape[0]
    # a degenerate (collinear) triangle in front of the box
    tris = np.concatenate([m.tris, np.array([[nv, nv + 1, nv]], np.int32)])
    inst = Instance(0, np.eye(3), np.array([0.0, 15.0, 0.0]), np.zeros(3))
    H0 = oracle.synthesize(Scene([m], [inst]), wf, arr)
    H1, mask = oracle.synthesize(Scene([Mesh(verts, tris)], [inst]), wf, arr, return_mask=True)
    assert not mask[:, -1].any()
    assert np.max(np.abs(H1 - H0)) == 0.0


def test_intra_chirp_delay_equals_eq12_eq13():
    """Delay at each sample time: a point moving radially away from a monostatic element
    has tau(t) = 2 (R0 + v t) / c (eq. (12)) with t = t_n + m / fs, and the beat sample
    conj(H) is eq. (13) with that tau; the amplitude stays at the chirp start."""
    wf = scenes.paper_waveform(64, 3)
    e = scenes.RADAR_POS.astype(np.float64)
    arr = RadarArray(tx=e[None].copy(), rx=e[None].copy())
    u = np.array([0.3, 0.9, -0.2])
    u /= np.linalg.norm(u)
    R0, v = 23.0, 14.0
    sc = Scene(meshes=[], instances=[],
               points=scenes.Points(pos0=(e + R0 * u)[None], vel=(v * u)[None],
                                    amp=np.array([2.0 + 1.0j])))
    H = oracle.synthesize(sc, wf, arr, intra_chirp=True)[0]
    c = 299792458.0
    m = np.arange(wf.n_samples)
    fm = wf.f0 + m * wf.slope / wf.fs
    for n in range(wf.n_chirps):
        tn = n * wf.chirp_period
        tau = 2.0 * (R0 + v * (tn + m / wf.fs)) / c
        Rn = R0 + v * tn
        expect = (2.0 + 1.0j) / (4 * np.pi * Rn * Rn) * np.exp(
            -2j * np.pi * (fm * tau - 0.5 * wf.slope * tau * tau))
        assert np.max(np.abs(H[n] - expect)) <= 1e-9 * np.max(np.abs(expect))
    # and it differs from stop-and-hop by the Doppler phase accrued within the chirp
    Hs = oracle.synthesize(sc, wf, arr)[0]
    drift = np.angle(H[0, -1] / Hs[0, -1])
    expect_drift = -2 * np.pi * fm[-1] * 2 * v * ((wf.n_samples - 1) / wf.fs) / c
    assert np.angle(np.exp(1j * (drift - expect_drift))) == pytest.approx(0.0, abs=1e-3)


def test_intra_chirp_static_scene_equals_stop_and_hop():
    """Without motion the intra-chirp delay changes nothing."""
    cfg = scenes.small_single(n_tris=300, n_samples=32, n_chirps=2)
    sc = cfg.scenes[0]
    still = Scene(meshes=sc.meshes, instances=[Instance(i.mesh, i.rot, i.pos0, 0.0 * i.vel)
                                               for i in sc.instances])
    a = oracle.synthesize(still, cfg.waveform, cfg.array, channels=[0, 77, 191])
    b = oracle.synthesize(still, cfg.waveform, cfg.array, channels=[0, 77, 191], intra_chirp=True)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))
