"""Parity at the full workload sizes, in the launch configuration bench.py times
(FP32 sum with FP64 phase, default tiles), on outputs the FP64 oracle computes one by
one: sampled chirps x channels x samples, sampled mask rows and properties that hold at
any size. Tolerance 1e-4 relative RMS on the echo."""
import os
import sys

import numpy as np
import pytest

import oracle
import scenes

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_rms(a, b):
    return float(np.sqrt(np.sum(np.abs(np.asarray(a) - np.asarray(b)) ** 2) /
                         np.sum(np.abs(np.asarray(b)) ** 2)))


def _sampled_parity(sim, sc, wf, arr, chirps, channels, samples, scene_index=0, echo=None,
                    gmask_rows=None):
    """Oracle visibility for the sampled chirps, mask-row check, then the echo on the
    sampled outputs. If an ambiguous facet was decided differently, the GPU is rerun with
    those rows taken from the oracle (mask input mode) before comparing."""
    om, amb = oracle.visibility(sc, arr, wf, chirps=chirps)
    mism = gmask_rows != om
    assert not (mism & ~amb).any(), f"{(mism & ~amb).sum()} unambiguous mask mismatches"
    H = echo
    if mism.any():
        _log(f"  {mism.sum()} ambiguous facets decided differently: rerun with oracle rows")
        full = sim.masks_numpy(sim.last_mask, [scene_index])[0]
        full[np.asarray(chirps)] = om
        H = sim.synthesize([scene_index], mask=sim.mask_from_numpy([full]), mask_mode=1)
        H = H.cpu().numpy()[0]
    mask_all = np.zeros((wf.n_chirps, om.shape[1]), bool)
    mask_all[np.asarray(chirps)] = om
    Ho = oracle.synthesize(sc, wf, arr, mask=mask_all, chirps=chirps, channels=channels,
                           samples=samples)
    Hg = H[np.ix_(channels, chirps, samples)]
    return rel_rms(Hg, Ho), om, amb


def test_single_vehicle_50k_full_size():
    """Both facet-sum kernels (the bench times the autotuner's pick, the other one is
    reported beside it) against the same oracle samples."""
    import torch
    from paper_2208_10939_amd.pipeline import Simulator
    _log("case 50k-triangle vehicle, 192 ch x 256 x 128 (bench launch configuration)")
    cfg = scenes.c2()
    sc, wf, arr = cfg.scenes[0], cfg.waveform, cfg.array
    sim = Simulator([sc], wf, arr)
    mask = sim.mask_buffer()
    sim.last_mask = mask
    Ht = sim.synthesize(mask=mask, kernel=1)
    Hm = sim.synthesize(mask=mask, kernel=2).cpu().numpy()[0]
    rdm = sim.form_rdm(Ht)
    torch.cuda.synchronize()
    H = Ht.cpu().numpy()[0]
    chirps = [0, 127]
    gm = sim.masks_numpy(mask)[0][chirps]
    channels = np.array([0, 37, 95, 128, 160, 191])
    err, om, amb = _sampled_parity(sim, sc, wf, arr, chirps, channels, np.arange(256), echo=H,
                                   gmask_rows=gm)
    _log(f"  lit={om.sum(1)} ambiguous={amb.sum()} vector-unit echo rel_rms={err:.3e}")
    assert err <= TOL
    if not (gm != om).any():  # same lit sets: the matrix-core echo against the same samples
        mask_all = np.zeros((wf.n_chirps, om.shape[1]), bool)
        mask_all[np.asarray(chirps)] = om
        Ho = oracle.synthesize(sc, wf, arr, mask=mask_all, chirps=chirps, channels=channels,
                               samples=np.arange(256))
        errm = rel_rms(Hm[np.ix_(channels, chirps, np.arange(256))], Ho)
        _log(f"  matrix-core echo rel_rms={errm:.3e}")
        assert errm <= TOL
    # Parseval over every chirp and channel of the RDM (no window, unnormalised FFTs)
    P = rdm.double().sum().item()
    E = (Ht.abs().double() ** 2).sum().item() * wf.n_samples * wf.n_chirps
    _log(f"  Parseval sum RDM / (M N sum |H|^2) = {P / E:.8f}")
    assert abs(P / E - 1.0) < 1e-5


C3_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                         "c3_oracle_samples.npz")


def _unpack_rows(packed, n_facets):
    bits = np.unpackbits(np.asarray(packed), axis=1, bitorder="little")
    return bits[:, :n_facets].astype(bool)


@pytest.mark.slow
def test_intersection_1m_default_path_and_every_kernel():
    """The 1M-triangle intersection (ground grid + 20 vehicles, 192 ch x 512 x 256) in
    bench's launch configuration: the library's autotuner runs first and the default
    (AUTO) facet sum is checked, then each facet-sum kernel explicitly on the same mask.
    Against the FP64 oracle's stored values (tests/golden/make_c3_samples.py, oracle only):
    the lit masks of chirps 0 and 255 over all 1M facets (mismatches only where the oracle
    flags the decision ambiguous), and the echo of six channels spread over the array x
    all 512 samples at those chirps, summed over every lit facet (bar 1e-4)."""
    import torch
    from paper_2208_10939_amd.pipeline import Simulator
    g = np.load(C3_GOLDEN, allow_pickle=False)
    chirps = [int(n) for n in g["chirps"]]
    channels = np.asarray(g["channels"])
    _log(f"case intersection 1M triangles, default path after autotune: chirps {chirps}, "
         f"channels {list(channels)}, 512 samples")
    cfg = scenes.c3()
    sc, wf, arr = cfg.scenes[0], cfg.waveform, cfg.array
    assert scenes.scene_digest(sc) == str(g["scene_sha16"]), "scene generator drift"
    F = int(g["n_facets"])
    om = _unpack_rows(g["mask"], F)
    amb = _unpack_rows(g["ambiguous"], F)
    sim = Simulator([sc], wf, arr)
    import tempfile
    fd, path = tempfile.mkstemp(suffix=".jsonl")
    os.close(fd)
    sim.ctx.autotune([sim.scene_ids[0]], path)
    with open(path) as f:
        import json
        tuned = json.loads(f.read().strip().splitlines()[-1])
    os.remove(path)
    _log(f"  autotuned kernel: {tuned['kernel']}")
    mask = sim.mask_buffer()
    H = sim.synthesize(mask=mask)
    torch.cuda.synchronize()
    full = sim.masks_numpy(mask)[0]
    gm = full[chirps]
    mism = gm != om
    _log(f"  lit={gm.sum(1)} oracle lit={om.sum(1)} ambiguous={amb.sum(1)} "
         f"mismatched={mism.sum(1)}")
    assert not (mism & ~amb).any(), f"{int((mism & ~amb).sum())} unambiguous mask mismatches"
    if mism.any():  # rerun with the oracle's rows for the sampled chirps
        full[chirps] = om
        mask = sim.mask_from_numpy([full])
        H = sim.synthesize(mask=mask, mask_mode=1)
    Hs = H[0][torch.as_tensor(channels).cuda()][:, chirps].cpu().numpy()
    err = rel_rms(Hs, g["echo"])
    _log(f"  default ({tuned['kernel']}) echo rel_rms={err:.3e}")
    assert err <= TOL
    for kernel, name in ((1, "vector"), (2, "matrix"), (3, "nufft")):
        Hk = sim.synthesize(mask=mask, mask_mode=1, kernel=kernel)
        Hs = Hk[0][torch.as_tensor(channels).cuda()][:, chirps].cpu().numpy()
        errk = rel_rms(Hs, g["echo"])
        _log(f"  {name} echo rel_rms={errk:.3e}")
        assert errk <= TOL
        del Hk


@pytest.mark.slow
def test_batched_64_scenes_equals_plain_and_oracle():
    import torch
    from paper_2208_10939_amd.pipeline import Simulator
    _log("case 64 scenes (10k-400k triangles): persistent graph launch vs plain (vector, "
         "NUFFT, matrix), oracle samples")
    cfg = scenes.c4()
    wf, arr = cfg.waveform, cfg.array
    sim = Simulator(cfg.scenes, wf, arr)
    n = len(cfg.scenes)
    mask = sim.mask_buffer()
    for kernel in (1, 3, 2):  # vector units, NUFFT, then matrix cores (kept in `batched`)
        batched = sim.synthesize(mask=mask, persistent=True, use_graph=True, kernel=kernel)
        torch.cuda.synchronize()
        same = True
        for i in range(n):
            one = sim.synthesize([i], kernel=kernel)
            same &= bool(torch.equal(one[0], batched[i]))
        assert same, f"kernel {kernel}: persistent and plain differ"
    masks = sim.masks_numpy(mask)
    for i in (int(np.argmin([s.n_tris for s in cfg.scenes])), 7):
        sc = cfg.scenes[i]
        om, amb = oracle.visibility(sc, arr, wf, chirps=[64])
        gm = masks[i][[64]]
        assert not ((gm != om) & ~amb).any()
        if (gm != om).any():
            continue  # ambiguous decisions: echo compared elsewhere
        mask_all = np.zeros((wf.n_chirps, om.shape[1]), bool)
        mask_all[64] = om[0]
        Ho = oracle.synthesize(sc, wf, arr, mask=mask_all, chirps=[64], channels=[3, 111],
                               samples=np.arange(0, 256, 4))
        Hg = batched[i].cpu().numpy()[np.ix_([3, 111], [64], np.arange(0, 256, 4))]
        err = rel_rms(Hg, Ho)
        _log(f"  scene {i}: {sc.n_tris} triangles, lit={om.sum()} rel_rms={err:.3e}")
        assert err <= TOL


C5_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c5_fd.npz")


@pytest.mark.slow
@pytest.mark.parametrize("kernel", [0, 3, 2])
def test_gradient_200k_two_vehicles(kernel):
    """The gradient workload (two vehicles of 100k triangles, loss sum (RDM - T)^2 against
    the seeded perturbed scene's RDM) at the reduced frame M = 32, 4 x 4 channels, N = 8,
    the masks held fixed at the oracle's: the library's adjoint (default choice, then the
    NUFFT and matrix-core adjoints explicitly) against the FP64 oracle's central finite
    differences stored by tests/golden/make_c5_fd.py: 50 seeded body-frame vertices x 3
    (25 uniform over both meshes, 25 on lit facets) and every velocity component of both
    vehicles. Bar: relative L2 <= 1e-3 over each set, and relative error <= 1e-3 for every
    component with |g| > 1e-3 max |g|."""
    import torch
    from paper_2208_10939_amd.pipeline import Simulator
    from scenes import RadarArray
    g = np.load(C5_GOLDEN, allow_pickle=False)
    M, P, Q, N = (int(v) for v in g["frame"])
    _log(f"case gradient, 200k triangles, M={M} {P}x{Q} N={N}, backward kernel {kernel}")
    base = scenes.c5(n_samples=M, n_chirps=N)
    sc, wf = base.scenes[0], base.waveform
    arr = RadarArray(tx=base.array.tx[:P].copy(), rx=base.array.rx[:Q].copy())
    assert scenes.scene_digest(sc) == str(g["scene_sha16"]), "scene generator drift"
    mask = _unpack_rows(g["mask"], int(g["n_facets"]))
    sim = Simulator([sc], wf, arr)
    m_t = sim.mask_from_numpy([mask])
    echo = sim.synthesize(mask=m_t, mask_mode=1)
    rdm, y = sim.form_rdm(echo, want_y=True)
    T = torch.from_numpy(np.asarray(g["target_rdm"], np.float32)).cuda()[None]
    ge = torch.empty_like(echo)
    sim.ctx.rdm_backward((2.0 * (rdm - T)).contiguous(), y, ge)
    gv = [torch.zeros((m.verts.shape[0], 3), dtype=torch.float32, device="cuda") for m in sc.meshes]
    gvel = torch.zeros((len(sc.instances), 3), dtype=torch.float64, device="cuda")
    sim.ctx.set_backward_kernel(kernel)
    sim.ctx.backward(sim.scene_ids[0], ge, m_t, gv, gvel)
    gv = [x.cpu().numpy().astype(np.float64) for x in gv]
    ad_v = np.array([gv[k][v] for k, v in zip(g["vert_mesh"], g["vert_index"])])
    ad_w = gvel.cpu().numpy()
    for name, ad, fd in (("vertices", ad_v, np.asarray(g["fd_vert"])),
                         ("velocities", ad_w, np.asarray(g["fd_vel"]))):
        rel_l2 = np.linalg.norm(ad - fd) / np.linalg.norm(fd)
        big = np.abs(fd) > 1e-3 * np.abs(fd).max()
        worst = float(np.max(np.abs(ad - fd)[big] / np.abs(fd)[big]))
        _log(f"  {name}: n={fd.size} (above 1e-3 max: {int(big.sum())}) rel_l2={rel_l2:.3e} "
             f"worst relative component error {worst:.3e}")
        assert rel_l2 <= 1e-3 and worst <= 1e-3
