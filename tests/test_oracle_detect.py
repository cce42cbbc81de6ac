"""Pins of the oracle's signal chain after the RDM (Section 3.3): CA-CFAR, the angle
FFT of eq. (6) and the point cloud, and the AWGN generator (Section 3.2). Each pin
checks the oracle against something other than itself: brute force on tiny inputs,
closed forms, known-answer vectors and a point scatterer at a known position."""
import json
import os

import numpy as np
import pytest

import oracle
import scenes
from oracle import detect, noise

HERE = os.path.dirname(os.path.abspath(__file__))


def test_cfar_matches_brute_force_on_tiny_maps():
    """Cell by cell on a 7 x 9 map (both axes wrap): mean over the training ring."""
    rng = np.random.default_rng(11)
    P = rng.exponential(size=(7, 9))
    guard, train, scale = (1, 1), (1, 2), 2.5
    det, noise_map, K = detect.ca_cfar(P, guard, train, scale)
    hd, hr = guard[0] + train[0], guard[1] + train[1]
    for n in range(7):
        for m in range(9):
            vals = [P[(n + a) % 7, (m + b) % 9]
                    for a in range(-hd, hd + 1) for b in range(-hr, hr + 1)
                    if not (abs(a) <= guard[0] and abs(b) <= guard[1])]
            assert len(vals) == K == (2 * hd + 1) * (2 * hr + 1) - 3 * 3
            assert noise_map[n, m] == pytest.approx(np.mean(vals), rel=1e-13)
            assert det[n, m] == (P[n, m] > scale * np.mean(vals))


def test_cfar_constant_map_and_single_spike():
    flat = np.full((16, 32), 3.0)
    det, nm, _ = detect.ca_cfar(flat, (1, 2), (2, 3), 1.0)
    assert np.all(nm == 3.0) and not det.any()  # strict '>' at scale 1
    det, _, _ = detect.ca_cfar(flat, (1, 2), (2, 3), 0.999)
    assert det.all()
    spike = flat.copy()
    spike[5, 20] = 300.0
    det, nm, _ = detect.ca_cfar(spike, (1, 2), (2, 3), 10.0)
    assert np.argwhere(det).tolist() == [[5, 20]]
    assert nm[5, 20] == 3.0  # the spike sits in its own guard rectangle


def test_cfar_false_alarm_rate_closed_form():
    """Exponential (square-law, one channel) noise: with K training cells and threshold
    scale * mean, P_fa = (1 + scale / K)^-K."""
    rng = np.random.default_rng(5)
    guard, train = (1, 1), (2, 3)
    K = (2 * 3 + 1) * (2 * 4 + 1) - 9
    scale = K * (1e-2 ** (-1.0 / K) - 1.0)  # design P_fa = 1e-2
    hits = cells = 0
    for _ in range(40):
        P = rng.exponential(size=(64, 64))
        det, _, k = detect.ca_cfar(P, guard, train, scale)
        assert k == K
        hits += int(det.sum())
        cells += det.size
    pfa = hits / cells
    assert abs(pfa - (1.0 + scale / K) ** (-K)) < 0.1 * 1e-2, pfa


def test_angle_fft_eq6_on_the_ula():
    """eq. (6): the path-difference phase step dphi between adjacent elements of a
    lambda/2 line array gives sin(theta) = lambda dphi / (2 pi d) = dphi / pi. The echo
    H carries +dphi per element; Y, formed from the beat signal conj(H), carries -dphi."""
    wf = scenes.paper_waveform(64, 4)
    arr = scenes.ula_1tx4rx(wf)
    ix, iz, nx, nz, d = detect.virtual_grid(arr, wf)
    assert nx == 4 and nz == 1 and list(ix) == [0, 1, 2, 3]
    for kx in (-3, -1, 0, 2, 5):
        na = 16
        u_true = -2.0 * kx / na
        dphi = np.pi * u_true  # echo phase step for direction cosine u_true
        y = np.exp(-1j * dphi * np.arange(4))  # as seen in Y
        A = detect.angle_spectrum(y, ix, iz, na, 1)
        u, w, skx, _, _ = detect.direction_from_peak(A)
        assert skx == kx and u == pytest.approx(u_true, abs=1e-15)
        assert np.degrees(np.arcsin(u)) == pytest.approx(np.degrees(np.arcsin(dphi / np.pi)))


def test_point_cloud_places_a_point_scatterer():
    """A point scatterer at a known position, through the oracle's echo, RDM, CFAR and
    angle FFT: the strongest detection lies within one range cell and one angle cell
    of the truth, and its Doppler row matches the range rate within one cell."""
    wf = scenes.paper_waveform(128, 32)
    arr = scenes.sparse_mimo_12x16(wf, seed=2)
    pos = np.array([[4.0, 20.0, -6.0]])  # direction cosines ~ (0.17, 0.86, -0.48)
    vel = np.array([[0.0, 2.0, 0.0]])
    sc = scenes.Scene(meshes=[], instances=[],
                      points=scenes.Points(pos0=pos, vel=vel, amp=np.array([1.0 + 0j])))
    H = oracle.synthesize(sc, wf, arr)
    P, Y = oracle.rdm_from_echo(H)
    pts = detect.point_cloud(P, Y, wf, arr, guard=(2, 2), train=(3, 6), scale=20.0)
    assert pts
    best = max(pts, key=lambda p: p["power"])
    c_ref = 0.5 * (arr.tx.mean(0) + arr.rx.mean(0))
    r_true = np.linalg.norm(pos[0] - c_ref)
    dv = (pos[0] - c_ref) / r_true
    dres = oracle.derived(wf)
    assert abs(best["range"] - r_true) <= dres["range_resolution"]
    assert abs(best["velocity"] - float(vel[0] @ dv)) <= dres["velocity_resolution"]
    ix, iz, nx, nz, _ = detect.virtual_grid(arr, wf)
    na_x = detect._fft_len(2 * nx)
    na_z = detect._fft_len(2 * nz)
    # within half a bin of the zero-padded grid (plus near-field slack); the sign of
    # both direction cosines is fixed since |u|, |w| exceed those margins
    assert abs(best["u"] - dv[0]) <= 1.0 / na_x + 0.01
    assert abs(best["w"] - dv[2]) <= 1.0 / na_z + 0.02


def test_philox_known_answers():
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.json")) as f:
        kat = json.load(f)
    for v in kat["vectors"]:
        c = [int(x, 16) for x in v["counter"]]
        k = [int(x, 16) for x in v["key"]]
        out = noise.philox4x32(c, k)
        assert [int(x) for x in out] == [int(x, 16) for x in v["out"]]


def test_awgn_statistics_and_snr():
    rng = np.random.default_rng(3)
    H = rng.normal(size=(2, 6, 8, 64)) + 1j * rng.normal(size=(2, 6, 8, 64))
    Hn = noise.add_awgn(H, 10.0, seed=1234)
    for c in range(2):
        nse = Hn[c] - H[c]
        ratio = np.mean(np.abs(H[c]) ** 2) / np.mean(np.abs(nse) ** 2)
        assert 10 * np.log10(ratio) == pytest.approx(10.0, abs=0.3)
        assert abs(np.mean(nse.real)) < 0.05 and abs(np.mean(nse.imag)) < 0.05
        assert abs(np.mean(nse.real * nse.imag)) < 0.05
    # distinct streams per cube, deterministic per seed
    assert not np.allclose(Hn[0] - H[0], Hn[1] - H[1])
    assert np.array_equal(noise.add_awgn(H, 10.0, seed=1234), Hn)
    re, im = noise.standard_normal_pairs(200_000, 0, 99)
    for x in (re, im):
        assert abs(np.mean(x)) < 0.01 and abs(np.var(x) - 1.0) < 0.01
        assert abs(np.mean(x ** 4) - 3.0) < 0.06  # Gaussian kurtosis
