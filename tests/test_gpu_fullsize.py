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
    _log("case 64 scenes (10k-400k triangles): persistent graph launch vs plain, oracle samples")
    cfg = scenes.c4()
    wf, arr = cfg.waveform, cfg.array
    sim = Simulator(cfg.scenes, wf, arr)
    n = len(cfg.scenes)
    mask = sim.mask_buffer()
    for kernel in (1, 2):  # vector units, then matrix cores (kept in `batched`)
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


@pytest.mark.slow
def test_gradient_200k_two_vehicles():
    """Full 200k-triangle two-vehicle scene at a reduced frame (the oracle must form
    every chirp): M=32, 4x4 channels, N=4. FD of the oracle loss uses the linearity of
    the facet sum: a vertex move changes only its incident facets' terms."""
    import torch
    from paper_2208_10939_amd.pipeline import Simulator
    from scenes import Instance, Mesh, RadarArray, Scene
    _log("case gradient, 200k triangles, M=32 4x4 N=4")
    base = scenes.c5(n_samples=32, n_chirps=4)
    sc, wf = base.scenes[0], base.waveform
    arr = RadarArray(tx=base.array.tx[:4].copy(), rx=base.array.rx[:4].copy())
    target = base.notes["target_scene"]
    mask, amb = oracle.visibility(sc, arr, wf)
    T, _ = oracle.rdm_from_echo(oracle.synthesize(target, wf, arr))
    H0 = oracle.synthesize(sc, wf, arr, mask=mask)

    def loss_from(H):
        P, _ = oracle.rdm_from_echo(H)
        return oracle.rdm_loss(P, T)

    sim = Simulator([sc], wf, arr)
    m_t = sim.mask_from_numpy([mask])
    echo = sim.synthesize(mask=m_t, mask_mode=1)
    rdm, y = sim.form_rdm(echo, want_y=True)
    g = 2.0 * (rdm - torch.from_numpy(T.astype(np.float32)).cuda()[None])
    ge = torch.empty_like(echo)
    sim.ctx.rdm_backward(g.contiguous(), y, ge)
    gv = [torch.zeros((m.verts.shape[0], 3), dtype=torch.float32, device="cuda") for m in sc.meshes]
    gvel = torch.zeros((2, 3), dtype=torch.float64, device="cuda")
    sim.ctx.backward(sim.scene_ids[0], ge, m_t, gv, gvel)
    gv = [x.cpu().numpy().astype(np.float64) for x in gv]
    gvel = gvel.cpu().numpy()

    tri0, inst_of, local_of = oracle.world_triangles(sc, 0.0)
    P_, Q_ = arr.tx.shape[0], arr.rx.shape[0]
    pq = [(o // Q_, o % Q_) for o in range(P_ * Q_)]
    freqs = wf.f0 + wf.slope / wf.fs * np.arange(wf.n_samples)
    import importlib
    E = importlib.import_module("oracle.echo")

    def delta_H(mesh_k, v, ax, dv):
        """H(verts + dv e_ax) - H(verts), via the incident lit facets only."""
        out = np.zeros_like(H0)
        for ii, inst in enumerate(sc.instances):
            if inst.mesh != mesh_k:
                continue
            m = sc.meshes[mesh_k]
            inc = np.nonzero((m.tris == v).any(axis=1))[0]
            base_idx = np.nonzero(inst_of == ii)[0][0]
            for n in range(wf.n_chirps):
                t = n * wf.chirp_period
                lit = inc[mask[n, base_idx + inc]]
                if lit.size == 0:
                    continue
                vb = m.verts.astype(np.float64)
                vb2 = vb.copy()
                vb2[v, ax] += dv
                for vv, sign in ((vb2, 1.0), (vb, -1.0)):
                    w = vv @ inst.rot.T + (inst.pos0 + inst.vel * t)
                    out[:, n, :] += sign * E.facet_terms(w[m.tris[lit]], wf, arr, freqs, pq)
        return out

    rng = np.random.default_rng(13)
    lit_f = np.nonzero(mask[0])[0]
    fd, ad = [], []
    for f in rng.choice(lit_f, 12, replace=False):
        k = sc.instances[inst_of[f]].mesh
        v = int(sc.meshes[k].tris[local_of[f], rng.integers(0, 3)])
        for ax in range(3):
            lp = loss_from(H0 + delta_H(k, v, ax, 1e-5))
            lm = loss_from(H0 + delta_H(k, v, ax, -1e-5))
            fd.append((lp - lm) / 2e-5)
            ad.append(gv[k][v, ax])
    fd, ad = np.array(fd), np.array(ad)
    rel_l2 = np.linalg.norm(ad - fd) / np.linalg.norm(fd)
    _log(f"  vertices: rel_l2={rel_l2:.3e} (n={fd.size}, ambiguous facets={amb.sum()})")
    assert rel_l2 <= 1e-3
    # velocity: one component per vehicle (along the lane), full re-synthesis of the scene
    fdv, adv = [], []
    for ik in range(2):
        hs = []
        for dv in (1e-2, -1e-2):
            insts = [Instance(i.mesh, i.rot, i.pos0, i.vel + (np.array([0.0, dv, 0.0]) if j == ik else 0.0))
                     for j, i in enumerate(sc.instances)]
            hs.append(loss_from(oracle.synthesize(Scene(sc.meshes, insts), wf, arr, mask=mask)))
        fdv.append((hs[0] - hs[1]) / 2e-2)
        adv.append(gvel[ik, 1])
    fdv, adv = np.array(fdv), np.array(adv)
    relv = np.linalg.norm(adv - fdv) / np.linalg.norm(fdv)
    _log(f"  velocities: adj={adv} fd={fdv} rel_l2={relv:.3e}")
    assert relv <= 1e-3
