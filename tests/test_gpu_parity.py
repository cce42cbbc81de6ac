"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the same
seeded inputs (element by element), at oracle-sized cases spanning several tiles with
ragged tails. Tolerances: FP64 path <= 1e-10 relative RMS on the echo; FP32 sum with
FP64 phase <= 1e-4 relative RMS (2e-4 on the RDM)."""
import sys

import numpy as np
import pytest

import oracle
import scenes
from scenes import RadarArray

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
FP32_TOL = 1e-4


def rel_rms(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.sqrt(np.sum(np.abs(a - b) ** 2) / np.sum(np.abs(b) ** 2)))


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sim_mod():
    import torch  # noqa: F401  (device memory)
    from paper_2208_10939_amd import pipeline
    return pipeline


def _mono():
    p = scenes.RADAR_POS[None, :].astype(np.float64)
    return RadarArray(tx=p.copy(), rx=p.copy())


@pytest.mark.parametrize("precision", [0, 1])
def test_point_targets(sim_mod, precision):
    _log(f"case point_targets precision={precision}")
    wf = scenes.paper_waveform(128, 16)
    sc = scenes.point_scene([12.3, 37.9, 55.0], [-7.0, 3.3, 12.0], amps=[1.0, 0.5 - 0.2j, 2j],
                            az_deg=[-20.0, 5.0, 33.0])
    arr = scenes.ula_1tx4rx(wf)
    sim = sim_mod.Simulator([sc], wf, arr)
    H = sim.synthesize(precision=precision).cpu().numpy()[0]
    Ho = oracle.synthesize(sc, wf, arr)
    err = rel_rms(H, Ho)
    _log(f"  rel_rms={err:.3e}")
    assert err <= (FP64_TOL if precision else 1e-5)


def test_c1_fp64_end_to_end(sim_mod):
    _log("case c1 fp64")
    cfg = scenes.c1()
    sc, wf, arr = cfg.scenes[0], cfg.waveform, cfg.array
    sim = sim_mod.Simulator([sc], wf, arr)
    mask_t = sim.mask_buffer()
    H = sim.synthesize(precision=1, mask=mask_t)
    rdm, Y = sim.form_rdm(H, precision=1, want_y=True)
    gmask = sim.masks_numpy(mask_t)[0]
    omask, amb = oracle.visibility(sc, arr, wf)
    bad = (gmask != omask) & ~amb
    assert not bad.any(), f"{bad.sum()} unambiguous mask mismatches"
    Ho = oracle.synthesize(sc, wf, arr, mask=omask)
    # if an ambiguous facet differs, compare against the oracle run on the oracle mask via
    # an input-mask GPU run instead
    if (gmask != omask).any():
        H = sim.synthesize(precision=1, mask=sim.mask_from_numpy([omask]), mask_mode=1)
        rdm, Y = sim.form_rdm(H, precision=1, want_y=True)
    err = rel_rms(H.cpu().numpy()[0], Ho)
    Po, Yo = oracle.rdm_from_echo(Ho)
    err_rdm = rel_rms(rdm.cpu().numpy()[0], Po)
    err_y = rel_rms(Y.cpu().numpy()[0], Yo)
    _log(f"  lit/chirp={omask.sum(1)[:3]} echo rel_rms={err:.3e} rdm={err_rdm:.3e} y={err_y:.3e}")
    assert err <= FP64_TOL
    assert err_rdm <= FP64_TOL and err_y <= FP64_TOL


def _check_mask_then_echo(sim_mod, cfg, precision, tol):
    sc, wf, arr = cfg.scenes[0], cfg.waveform, cfg.array
    sim = sim_mod.Simulator([sc], wf, arr)
    mask_t = sim.mask_buffer()
    H_compute = sim.synthesize(precision=precision, mask=mask_t)
    gmask = sim.masks_numpy(mask_t)[0]
    omask, amb = oracle.visibility(sc, arr, wf)
    mism = gmask != omask
    assert not (mism & ~amb).any(), f"{(mism & ~amb).sum()} unambiguous mask mismatches"
    Ho = oracle.synthesize(sc, wf, arr, mask=omask)
    H_in = sim.synthesize(precision=precision, mask=sim.mask_from_numpy([omask]), mask_mode=1)
    err = rel_rms(H_in.cpu().numpy()[0], Ho)
    _log(f"  F={sim.n_facets[0]} lit/chirp={omask.sum(1)} ambiguous={amb.sum()} "
         f"mismatch={mism.sum()} echo rel_rms={err:.3e}")
    assert err <= tol
    if not mism.any():
        assert rel_rms(H_compute.cpu().numpy()[0], Ho) <= tol
    return sim, H_in, Ho


def test_small_single_fp32(sim_mod):
    """M = 96 = 2^5 3: a ragged sample tile for the facet sum and a mixed-radix range
    FFT for the RDM."""
    _log("case small_single fp32 (1.5k tris, 192 ch, M=96 ragged, N=4)")
    sim, H, Ho = _check_mask_then_echo(sim_mod, scenes.small_single(), 0, FP32_TOL)
    rdm = sim.form_rdm(H.contiguous()).cpu().numpy()[0]
    Po, _ = oracle.rdm_from_echo(Ho)
    err = rel_rms(rdm, Po)
    _log(f"  rdm rel_rms={err:.3e}")
    assert err <= 2 * FP32_TOL


def test_small_single_fp64(sim_mod):
    _log("case small_single fp64")
    _check_mask_then_echo(sim_mod, scenes.small_single(n_samples=64, n_chirps=2), 1, FP64_TOL)


def test_small_intersection_fp32_and_rdm(sim_mod):
    _log("case small_intersection fp32 + rdm")
    cfg = scenes.small_intersection()
    sim, H, Ho = _check_mask_then_echo(sim_mod, cfg, 0, FP32_TOL)
    rdm = sim.form_rdm(H).cpu().numpy()[0]
    Po, _ = oracle.rdm_from_echo(Ho)
    err = rel_rms(rdm, Po)
    _log(f"  rdm rel_rms={err:.3e}")
    assert err <= 2 * FP32_TOL


def test_experiment2_waveform_384_samples(sim_mod):
    """The paper's second experiment waveform (384 samples per chirp; Table 2) end to end
    on a small vehicle scene: echo and RDM against the oracle (radix-3 range FFT, and a
    Doppler length of 12 = 2^2 3)."""
    _log("case experiment-2 waveform M=384 N=12, 1.5k-triangle vehicle")
    base = scenes.small_single(n_samples=384, n_chirps=12)
    sim, H, Ho = _check_mask_then_echo(sim_mod, base, 0, FP32_TOL)
    rdm = sim.form_rdm(H).cpu().numpy()[0]
    Po, _ = oracle.rdm_from_echo(Ho)
    err = rel_rms(rdm, Po)
    _log(f"  rdm rel_rms={err:.3e}")
    assert err <= 2 * FP32_TOL


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("M,N", [(256, 64), (384, 48), (162, 6), (96, 9), (64, 81),
                                 (4096, 2), (3888, 2), (2, 4096)])
def test_rdm_fft_against_numpy(sim_mod, precision, M, N):
    """Range/Doppler FFTs and the RDM on a seeded random cube vs numpy.fft (FP64), at
    power-of-two lengths and at mixed radix-2/3 lengths (384 samples is the paper's
    second experiment; 162 = 2 x 3^4); odd chirp counts (9, 81) check that row l holds
    Doppler index l - floor(N/2), as numpy's fftshift puts it; the largest lengths the
    transforms take (4096 samples or chirps; 3888 = 2^4 3^5) and the smallest (2)."""
    import torch
    _log(f"case rdm_fft precision={precision} M={M} N={N}")
    wf = scenes.paper_waveform(M, N)
    arr = scenes.sparse_mimo_12x16(wf, 1)
    sim = sim_mod.Simulator([scenes.point_scene([20.0], [1.0])], wf, arr)
    rng = np.random.default_rng(7)
    H = rng.normal(size=(2, sim.O, wf.n_chirps, wf.n_samples)) + 1j * rng.normal(
        size=(2, sim.O, wf.n_chirps, wf.n_samples))
    dt = torch.complex128 if precision else torch.complex64
    Ht = torch.from_numpy(H).to(dt).cuda()
    rdm, Y = sim.form_rdm(Ht, precision=precision, want_y=True)
    Po, Yo = oracle.rdm_from_echo(H.astype(np.complex64).astype(np.complex128) if not precision else H)
    e1 = rel_rms(Y.cpu().numpy(), Yo)
    e2 = rel_rms(rdm.cpu().numpy(), Po)
    _log(f"  Y rel_rms={e1:.3e} rdm rel_rms={e2:.3e}")
    tol = 1e-13 if precision else 2e-6
    assert e1 <= tol and e2 <= 2 * tol


@pytest.mark.parametrize("M,N", [(128, 32), (96, 12), (48, 27)])
def test_rdm_adjoint_identity(sim_mod, M, N):
    """<A x, g> = <x, A^H g> (real inner product) for the linear map x -> Y."""
    import torch
    _log(f"case rdm_adjoint M={M} N={N}")
    wf = scenes.paper_waveform(M, N)
    arr = scenes.ula_1tx4rx(wf)
    sim = sim_mod.Simulator([scenes.point_scene([20.0], [1.0])], wf, arr)
    rng = np.random.default_rng(3)
    shape = (1, sim.O, wf.n_chirps, wf.n_samples)
    x = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    g = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    xt = torch.from_numpy(x).to(torch.complex64).cuda()
    gt = torch.from_numpy(g).to(torch.complex64).cuda()
    _, Y = sim.form_rdm(xt, want_y=True)
    gx = torch.empty_like(gt)
    sim.ctx.rdm_adjoint(gt, gx)
    lhs = np.sum((np.conj(g) * Y.cpu().numpy().astype(np.complex128)).real)
    rhs = np.sum((np.conj(gx.cpu().numpy().astype(np.complex128)) * x).real)
    _log(f"  lhs={lhs:.6e} rhs={rhs:.6e}")
    assert abs(lhs - rhs) <= 1e-4 * abs(lhs)
    # and against the oracle's numpy adjoint: G_H = FFT_m(FFT_n(conj(unshift(G_Y))))
    ref = np.fft.fft(np.fft.fft(np.conj(np.fft.ifftshift(g, axes=-2)), axis=-2), axis=-1)
    assert rel_rms(gx.cpu().numpy(), ref) <= 2e-6


def test_batched_persistent_equals_plain(sim_mod):
    _log("case batched (4 scenes, persistent + graph) vs plain, vector-unit kernel")
    wf = scenes.paper_waveform(64, 4)
    arr = scenes.sparse_mimo_12x16(wf, 4)
    scs = [scenes.intersection_scene(400 + i, n_vehicles=1 + i, per_vehicle=300 + 200 * i,
                                     with_ground=False) for i in range(4)]
    sim = sim_mod.Simulator(scs, wf, arr)
    plain = sim.synthesize(kernel=1)
    for i in range(4):
        one = sim.synthesize(which=[i], kernel=1)
        assert np.array_equal(one.cpu().numpy()[0], plain.cpu().numpy()[i])
    pers = sim.synthesize(persistent=True, kernel=1)
    assert np.array_equal(pers.cpu().numpy(), plain.cpu().numpy())
    buf = sim.echo_buffer(4)
    for rep in range(3):
        buf.zero_()
        sim.synthesize(echo=buf, persistent=True, use_graph=True, kernel=1)
        assert np.array_equal(buf.cpu().numpy(), plain.cpu().numpy()), f"replay {rep}"
    Ho = oracle.synthesize(scs[2], wf, arr)
    err = rel_rms(plain.cpu().numpy()[2], Ho)
    _log(f"  scene 2 vs oracle rel_rms={err:.3e}")
    assert err <= FP32_TOL


def test_intra_chirp_delay_fp32(sim_mod):
    """Delay at each sample time (range-Doppler coupling within the chirp), FP32 sum on
    the vector units:
    fast point targets and a moving vehicle against the oracle's reading; the result
    differs from stop-and-hop by far more than the tolerance."""
    import torch
    _log("case intra-chirp delay: points at 12-15 m/s and a 1.5k-triangle vehicle")
    wf = scenes.paper_waveform(256, 4)
    arr = scenes.sparse_mimo_12x16(wf, 3)
    sc = scenes.point_scene([14.0, 31.0, 52.0], [15.0, -12.0, 13.0],
                            amps=[1.0, 0.5 - 0.2j, 2j], az_deg=[-25.0, 8.0, 30.0])
    sim = sim_mod.Simulator([sc], wf, arr)
    H = sim.synthesize(intra_chirp=True, kernel=1).cpu().numpy()[0]
    Ho = oracle.synthesize(sc, wf, arr, intra_chirp=True)
    Hs = oracle.synthesize(sc, wf, arr)
    err, moved = rel_rms(H, Ho), rel_rms(Hs, Ho)
    _log(f"  points: rel_rms={err:.3e} (stop-and-hop differs by {moved:.3e})")
    assert err <= 1e-5 and moved >= 1e-2
    cfg = scenes.small_single(n_samples=128, n_chirps=3)
    sc, wf, arr = cfg.scenes[0], cfg.waveform, cfg.array
    sim = sim_mod.Simulator([sc], wf, arr)
    omask, amb = oracle.visibility(sc, arr, wf)
    H = sim.synthesize(mask=sim.mask_from_numpy([omask]), mask_mode=1,
                       intra_chirp=True, kernel=1).cpu().numpy()[0]
    Ho = oracle.synthesize(sc, wf, arr, mask=omask, intra_chirp=True)
    err = rel_rms(H, Ho)
    _log(f"  vehicle: speed {np.linalg.norm(sc.instances[0].vel):.1f} m/s rel_rms={err:.3e}")
    assert err <= FP32_TOL
    # FP64 requests are refused
    with pytest.raises(Exception):
        sim.synthesize(precision=1, intra_chirp=True)
    torch.cuda.synchronize()


def _one_triangle_scene(verts_body, centre):
    """A single triangle (body-frame vertices about the origin) placed at `centre`."""
    from scenes import Instance, Mesh, Scene
    mesh = Mesh(verts=np.asarray(verts_body, np.float32), tris=np.array([[0, 1, 2]], np.int32))
    inst = Instance(mesh=0, rot=np.eye(3), pos0=np.asarray(centre, np.float64), vel=np.zeros(3))
    return Scene(meshes=[mesh], instances=[inst])


def _regime_triangles(wf, arr):
    """Triangles chosen for the branches of the closed-form facet integral Phi (Sec. 3.2):
    broadside (all projected nodes equal: series), an edge across the bisector direction
    (two equal nodes: sinc with a zero argument), a near-degenerate pair (sinc argument
    ~2e-3), a large tilted facet (sinc, arguments of hundreds of radians) and a small facet
    whose widest projected gap crosses the series threshold inside the band. Projected
    node b_k = w . (x_k - c), w = unit(T - c) + unit(R - c) with T, R the phase centres."""
    centre = np.array([3.0, 15.0, 1.0])
    w = sum((p - centre) / np.linalg.norm(p - centre) for p in (arr.tx.mean(0), arr.rx.mean(0)))
    wn = np.linalg.norm(w)
    u = w / wn
    e1 = np.cross(u, [0.0, 0.0, 1.0])
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(u, e1)
    f_mid = wf.f0 + 0.5 * (wf.n_samples - 1) * wf.slope / wf.fs
    s_mid = f_mid / 299792458.0  # turns per metre
    g = 0.5 / (2.0 * np.pi * s_mid) / wn  # offset along u giving a 0.5 rad gap at mid band
    tri = {
        "broadside": [0.04 * e1, -0.03 * e1 + 0.03 * e2, -0.02 * e1 - 0.04 * e2],
        "edge_across_bisector": [-0.05 * e1, 0.05 * e1, 0.04 * u + 0.03 * e2],
        "near_degenerate": [-0.05 * e1, 0.05 * e1 + 1e-6 * u, 0.04 * u + 0.03 * e2],
        "large_tilted": [0.2 * e1 - 0.1 * u, -0.15 * e1 + 0.12 * e2 + 0.08 * u,
                         -0.05 * e1 - 0.2 * e2 + 0.03 * u],
    }

    def crossing(gg):
        return [0.0 * u, 0.01 * e1 + gg * u, 0.008 * e2 + 0.4 * gg * u]

    def mid_gap(v):
        x = np.stack(v).astype(np.float32).astype(np.float64) + centre
        c = x.mean(0)
        ww = sum((p - c) / np.linalg.norm(p - c) for p in (arr.tx.mean(0), arr.rx.mean(0)))
        b = (x - c) @ ww
        return 2.0 * np.pi * s_mid * (b.max() - b.min())

    for _ in range(3):  # the facet's own bisector differs slightly from w at `centre`
        g *= 0.5 / mid_gap(crossing(g))
    tri["series_crossing"] = crossing(g)
    return centre, tri


@pytest.mark.parametrize("precision", [0, 1])
def test_facet_integral_regimes(sim_mod, precision):
    """One triangle per scene, every chirp forced lit (mask input), 192 channels x 256
    samples (two sample tiles): each echo element against the oracle. FP32: elementwise
    relative error <= 2e-5; FP64: <= 1e-10 relative RMS."""
    wf = scenes.paper_waveform(256, 2)
    arr = scenes.sparse_mimo_12x16(wf, seed=2)
    centre, tri = _regime_triangles(wf, arr)
    for name, v in tri.items():
        sc = _one_triangle_scene(np.stack(v), centre)
        _log(f"case facet regime {name} precision={precision}")
        sim = sim_mod.Simulator([sc], wf, arr)
        mask = np.ones((wf.n_chirps, 1), bool)
        H = sim.synthesize(precision=precision, mask=sim.mask_from_numpy([mask]),
                           mask_mode=1).cpu().numpy()[0]
        Ho = oracle.synthesize(sc, wf, arr, mask=mask)
        if precision:
            err = rel_rms(H, Ho)
            _log(f"  rel_rms={err:.3e}")
            assert err <= FP64_TOL
        else:
            err = float(np.max(np.abs(H - Ho) / np.abs(Ho)))
            _log(f"  max elementwise rel={err:.3e} rel_rms={rel_rms(H, Ho):.3e}")
            assert err <= 2e-5


def test_degenerate_scenes(sim_mod):
    """Scenes with nothing to sum: no instance at all, and one with a triangle facing away
    from both phase centres (never lit) beside a mesh of zero-area triangles only. Every
    facet-sum kernel (vector units, matrix cores, NUFFT) gives all-zero echoes and RDMs;
    called with a vehicle scene, plain and persistent, the vehicle's echo is the bits of its
    own call; the backward gives zero gradients."""
    import torch
    from scenes import Instance, Mesh, Scene
    cfg = scenes.small_single(n_samples=64, n_chirps=8, n_tris=800)
    wf = cfg.waveform
    arr = RadarArray(tx=np.array(cfg.array.tx[:3]), rx=np.array(cfg.array.rx[:4]))
    away = Mesh(verts=np.array([[0, 20, 0], [0, 20, 1], [1, 20, 0]], np.float32),
                tris=np.array([[0, 1, 2]], np.int32), name="away")  # normal +y: faces away
    line = Mesh(verts=np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0]], np.float32),
                tris=np.array([[0, 1, 2], [2, 1, 0]], np.int32), name="zero-area")
    eye = np.eye(3)
    dark = Scene([away, line], [Instance(0, eye, np.zeros(3), np.array([0.0, 2.0, 0.0])),
                                Instance(1, eye, np.array([0.0, 15.0, 1.0]), np.zeros(3))])
    _log("case degenerate scenes (empty; unlit + zero-area) with every kernel")
    sim = sim_mod.Simulator([Scene([], []), dark, cfg.scenes[0]], wf, arr)
    assert sim.n_facets[0] == 0 and sim.n_facets[1] == 3
    for kernel in (1, 2, 3):
        for i in (0, 1):
            H = sim.synthesize([i], mask=sim.mask_buffer([i]), kernel=kernel)
            P = sim.form_rdm(H)
            assert torch.count_nonzero(H).item() == 0, (kernel, i)
            assert torch.count_nonzero(P).item() == 0, (kernel, i)
        Hv = sim.synthesize([2], mask=sim.mask_buffer([2]), kernel=kernel).cpu()
        assert torch.count_nonzero(Hv).item() > 0
        for persistent in (False, True):
            Ha = sim.synthesize(mask=sim.mask_buffer(), kernel=kernel, persistent=persistent).cpu()
            assert torch.count_nonzero(Ha[:2]).item() == 0, (kernel, persistent)
            assert torch.equal(Ha[2], Hv[0]), (kernel, persistent)
    O = arr.tx.shape[0] * arr.rx.shape[0]
    rng = np.random.default_rng(5)
    g = (rng.standard_normal((O, wf.n_chirps, wf.n_samples)) +
         1j * rng.standard_normal((O, wf.n_chirps, wf.n_samples))).astype(np.complex64)
    ge = torch.from_numpy(g).cuda()
    for kernel in (1, 3):
        sim.ctx.set_backward_kernel(kernel)
        for i in (0, 1):
            mask = sim.mask_buffer([i])
            sim.synthesize([i], mask=mask, kernel=kernel)
            gv = [torch.zeros((m.verts.shape[0], 3), dtype=torch.float32, device="cuda")
                  for m in ([] if i == 0 else dark.meshes)]
            gvel = torch.full((max(1, 2 * i), 3), 0.0, dtype=torch.float64, device="cuda")
            sim.ctx.backward(sim.scene_ids[i], ge, mask, gv, gvel)
            assert all(torch.count_nonzero(x).item() == 0 for x in gv), (kernel, i)
            assert torch.count_nonzero(gvel).item() == 0, (kernel, i)
    sim.ctx.set_backward_kernel(0)


@pytest.mark.parametrize("case", ["samples", "chirps"])
def test_synthesis_at_maximum_sizes(sim_mod, case):
    """The facet sum at the largest frame sizes the library takes: 4096 samples per chirp
    (a 300-triangle vehicle, oracle visibility as input mask; the vector units, the matrix
    cores and the default kernel) and 4096 chirps (point targets, which need no
    visibility), FP32 sum with FP64 phase against the FP64 oracle."""
    if case == "samples":
        cfg = scenes.small_single(n_samples=4096, n_chirps=2, n_tris=300)
        sc, wf = cfg.scenes[0], cfg.waveform
        arr = RadarArray(tx=np.array(cfg.array.tx[:2]), rx=np.array(cfg.array.rx[:2]))
        mask, _ = oracle.visibility(sc, arr, wf)
        kernels = (1, 2, 0)
    else:
        wf = scenes.paper_waveform(2, 4096)
        sc = scenes.point_scene([12.3, 37.9], [-7.0, 3.3], amps=[1.0, 0.5 - 0.2j],
                                az_deg=[-20.0, 5.0])
        arr = scenes.ula_1tx4rx(wf)
        mask = None
        kernels = (1, 0)
    _log(f"case synthesis at maximum size: {case} (M={wf.n_samples}, N={wf.n_chirps})")
    sim = sim_mod.Simulator([sc], wf, arr)
    Ho = oracle.synthesize(sc, wf, arr, mask=mask)
    m_t = sim.mask_from_numpy([mask]) if mask is not None else sim.mask_buffer()
    for k in kernels:
        mode = 1 if mask is not None else 0
        H = sim.synthesize(mask=m_t, mask_mode=mode, kernel=k).cpu().numpy()[0]
        err = rel_rms(H, Ho)
        _log(f"  kernel {k}: rel_rms={err:.3e}")
        assert err <= 1e-4, k

