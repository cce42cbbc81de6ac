"""GPU parity of the matrix-core facet sum (the separable Tx x Rx contraction per sample,
Sections 2.2 and 3.2, eqs. (7), (9)-(13)) through the C ABI: against the FP64 oracle
(relative RMS <= 1e-4, the FP32 bar) on arrays of each compiled tile shape, sample
counts spanning several 128-sample tiles with a ragged tail, the intra-chirp delay and
the ground double bounce; against the vector-unit kernel on the same inputs; the
persistent batched form bit-identical to plain launches; and the refusals."""
import sys

import numpy as np
import pytest

import oracle
import scenes
from scenes import RadarArray

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-4
VECTOR, MATRIX = 1, 2


def rel_rms(a, b):
    return float(np.sqrt(np.sum(np.abs(a - b) ** 2) / np.sum(np.abs(b) ** 2)))


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sim_mod():
    import torch  # noqa: F401
    from paper_2208_10939_amd import pipeline
    return pipeline


def _cross_bound(arr, wf):
    """Largest |2 pi slope d_p e_q| (d, e: element offsets from the Tx / Rx phase centre
    over c)."""
    c0 = 299792458.0
    dt = np.linalg.norm(arr.tx - arr.tx.mean(0), axis=1).max()
    dr = np.linalg.norm(arr.rx - arr.rx.mean(0), axis=1).max()
    return 2 * np.pi * abs(wf.slope) * dt * dr / c0 ** 2


def _scaled(arr, k):
    """The array with every element offset from its phase centre scaled by k."""
    ct, cr = arr.tx.mean(0), arr.rx.mean(0)
    return RadarArray(tx=ct + k * (arr.tx - ct), rx=cr + k * (arr.rx - cr))


def _subarray(arr, P, Q):
    return RadarArray(tx=np.array(arr.tx[:P]), rx=np.array(arr.rx[:Q]))


@pytest.mark.parametrize("P,Q", [(1, 4), (3, 16), (6, 8), (12, 16), (5, 11)])
def test_matrix_sum_against_oracle(sim_mod, P, Q):
    """Vehicle scene (1.5k triangles: ~100 tiles of 16 facets with a ragged last one),
    M = 300 (two full 128-sample tiles and a ragged third), oracle masks as input."""
    cfg = scenes.small_single(n_samples=300, n_chirps=2)
    sc, wf = cfg.scenes[0], cfg.waveform
    arr = _subarray(cfg.array, P, Q)
    _log(f"case matrix sum P={P} Q={Q} M=300 N=2")
    sim = sim_mod.Simulator([sc], wf, arr)
    omask, _ = oracle.visibility(sc, arr, wf)
    m_in = sim.mask_from_numpy([omask])
    Hm = sim.synthesize(mask=m_in, mask_mode=1, kernel=MATRIX).cpu().numpy()[0]
    Hv = sim.synthesize(mask=m_in, mask_mode=1, kernel=VECTOR).cpu().numpy()[0]
    Ho = oracle.synthesize(sc, wf, arr, mask=omask)
    em, ev, emv = rel_rms(Hm, Ho), rel_rms(Hv, Ho), rel_rms(Hm, Hv)
    _log(f"  lit/chirp={omask.sum(1)} matrix={em:.3e} vector={ev:.3e} matrix-vector={emv:.3e}")
    assert em <= FP32_TOL and ev <= FP32_TOL


def test_matrix_points_and_intra_chirp(sim_mod):
    """Point scatterers only (every work item a single ragged facet tile), stop-and-hop
    and with the delay at each sample time."""
    wf = scenes.paper_waveform(256, 4)
    arr = scenes.sparse_mimo_12x16(wf, 3)
    sc = scenes.point_scene([14.0, 31.0, 52.0], [15.0, -12.0, 13.0],
                            amps=[1.0, 0.5 - 0.2j, 2j], az_deg=[-25.0, 8.0, 30.0])
    _log("case matrix sum, point scatterers, stop-and-hop and intra-chirp")
    sim = sim_mod.Simulator([sc], wf, arr)
    for intra in (False, True):
        H = sim.synthesize(kernel=MATRIX, intra_chirp=intra).cpu().numpy()[0]
        Ho = oracle.synthesize(sc, wf, arr, intra_chirp=intra)
        err = rel_rms(H, Ho)
        _log(f"  intra={intra} rel_rms={err:.3e}")
        assert err <= 1e-5
    cfg = scenes.small_single(n_samples=256, n_chirps=3)
    sc, wf, arr = cfg.scenes[0], cfg.waveform, cfg.array
    sim = sim_mod.Simulator([sc], wf, arr)
    omask, _ = oracle.visibility(sc, arr, wf)
    H = sim.synthesize(mask=sim.mask_from_numpy([omask]), mask_mode=1, kernel=MATRIX,
                       intra_chirp=True).cpu().numpy()[0]
    Ho = oracle.synthesize(sc, wf, arr, mask=omask, intra_chirp=True)
    err = rel_rms(H, Ho)
    _log(f"  vehicle intra-chirp rel_rms={err:.3e}")
    assert err <= FP32_TOL


def test_matrix_ground_bounce(sim_mod):
    import torch
    from oracle import bounce
    from paper_2208_10939_amd.pipeline import pack_mask
    cfg = scenes.small_single(n_samples=160, n_chirps=2)
    sc, wf, arr = cfg.scenes[0], cfg.waveform, cfg.array
    _log("case matrix sum with the ground double bounce")
    sim = sim_mod.Simulator([sc], wf, arr)
    gamma = -0.9 + 0.2j
    sim.set_ground(True, 0.0, gamma)
    om, _ = bounce.visibility_bounce(sc, arr, wf, 0.0)
    packed = np.concatenate([pack_mask(om[k]).reshape(-1) for k in range(4)])
    m_in = torch.from_numpy(packed.view(np.int32).copy()).cuda()
    H = sim.synthesize(mask=m_in, mask_mode=1, kernel=MATRIX).cpu().numpy()[0]
    Ho = bounce.synthesize_bounce(sc, wf, arr, z_g=0.0, gamma=gamma, masks=om)
    err = rel_rms(H, Ho)
    _log(f"  lit per type {[int(om[k].sum()) for k in range(4)]} rel_rms={err:.3e}")
    assert err <= FP32_TOL


def test_matrix_batched_persistent_equals_plain(sim_mod):
    _log("case matrix sum: batched (4 scenes, persistent + graph) vs plain")
    wf = scenes.paper_waveform(200, 4)
    arr = scenes.sparse_mimo_12x16(wf, 4)
    scs = [scenes.intersection_scene(400 + i, n_vehicles=1 + i, per_vehicle=300 + 200 * i,
                                     with_ground=False) for i in range(4)]
    sim = sim_mod.Simulator(scs, wf, arr)
    plain = sim.synthesize(kernel=MATRIX).cpu().numpy()
    for i in range(4):
        one = sim.synthesize(which=[i], kernel=MATRIX).cpu().numpy()[0]
        assert np.array_equal(one, plain[i])
    pers = sim.synthesize(persistent=True, kernel=MATRIX).cpu().numpy()
    assert np.array_equal(pers, plain)
    buf = sim.echo_buffer(4)
    for rep in range(3):
        buf.zero_()
        sim.synthesize(echo=buf, persistent=True, use_graph=True, kernel=MATRIX)
        assert np.array_equal(buf.cpu().numpy(), plain), f"replay {rep}"
    Ho = oracle.synthesize(scs[1], wf, arr)
    err = rel_rms(plain[1], Ho)
    _log(f"  scene 1 vs oracle rel_rms={err:.3e}")
    assert err <= FP32_TOL


def test_matrix_refusals(sim_mod):
    """FP64 and ineligible arrays are refused when the matrix cores are asked for; the
    automatic choice falls back to the vector units there."""
    from paper_2208_10939_amd.rsim import RSIM_EINVAL, RSIM_ERANGE, RsimError
    wf = scenes.paper_waveform(64, 2)
    arr = scenes.sparse_mimo_12x16(wf, 1)
    sc = scenes.point_scene([20.0], [1.0])
    sim = sim_mod.Simulator([sc], wf, arr)
    with pytest.raises(RsimError) as e:
        sim.synthesize(precision=1, kernel=MATRIX)
    assert e.value.code == RSIM_EINVAL
    with pytest.raises(RsimError) as e:
        sim.synthesize(kernel=4)
    assert e.value.code == RSIM_EINVAL
    # 13 Tx elements: no compiled tile shape
    tx = np.concatenate([arr.tx, arr.tx[:1] + [0.0, 0.0, 0.002]])
    big = RadarArray(tx=tx, rx=np.array(arr.rx))
    sim2 = sim_mod.Simulator([sc], wf, big)
    with pytest.raises(RsimError) as e:
        sim2.synthesize(kernel=MATRIX)
    assert e.value.code == RSIM_ERANGE
    H = sim2.synthesize().cpu().numpy()[0]
    assert rel_rms(H, oracle.synthesize(sc, wf, big)) <= 1e-5
    # a wide aperture (cross term above 1e-5 rad but within the vector kernel's 3e-4)
    wide = _scaled(arr, 6.0)
    assert 1e-5 < _cross_bound(wide, wf) < 3e-4
    sim3 = sim_mod.Simulator([sc], wf, wide)
    with pytest.raises(RsimError) as e:
        sim3.synthesize(kernel=MATRIX)
    assert e.value.code == RSIM_ERANGE
    H = sim3.synthesize().cpu().numpy()[0]
    assert rel_rms(H, oracle.synthesize(sc, wf, wide)) <= 1e-5
