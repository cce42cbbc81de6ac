"""GPU parity of the facet-to-facet double bounce (Section 2.2: a ray reflected by one facet
joined with a ray from the other end on a second facet; the connection rules and the
footprint term of oracle/dbounce.py) through the C ABI, against the FP64 oracle:

* the connection table the library computes (the facet B of every launching end, chirp
  and facet A) equals the oracle's except where the oracle marks a decision ambiguous;
* given the oracle's connections and no lit facet (RSIM_MASK_INPUT), the echo is the
  double bounce alone: against the oracle's at the FP32 bar (1e-4 relative RMS), and the
  record census counts exactly those connections;
* the whole echo (single + double bounce, complex gamma) against the oracle's sum;
* the dihedral closed form (sigma = 8 pi a^2 b^2 / lambda^2) through the GPU path;
* the adjoint (NUFFT, connections held) against FP64 central differences of the oracle's
  loss over the single + double-bounce echo (oracle/dbounce.pairs_for_table);
* the refusals.
"""
import sys

import numpy as np
import pytest

import oracle
import scenes
from oracle import dbounce
from scenes import RadarArray, Waveform

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-4


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_rms(a, b):
    return float(np.sqrt(np.sum(np.abs(a - b) ** 2) / np.sum(np.abs(b) ** 2)))


def _sim(sc, wf, arr, gamma=-1.0):
    from paper_2208_10939_amd.pipeline import Simulator
    sim = Simulator([sc], wf, arr)
    sim.set_double_bounce(True, gamma)
    return sim


def _cases():
    small = scenes.small_single(n_samples=64, n_chirps=2, n_tris=1500)
    fine = scenes.small_single(n_samples=64, n_chirps=2, n_tris=6000)
    inter = scenes.small_intersection(n_samples=64, n_chirps=2)
    wf_d = Waveform(f0=77e9, slope=12.5e12, fs=5.12e6, chirp_period=60e-6, n_samples=64,
                    n_chirps=2)
    dih = scenes.dihedral_scene(0.3, 0.2, 30.0, 4, 4)
    return [("vehicle 1.5k", small.scenes[0], small.waveform, small.array, 4, 6),
            ("vehicle 6k", fine.scenes[0], fine.waveform, fine.array, 4, 4),
            ("intersection", inter.scenes[0], inter.waveform, inter.array, 3, 4),
            ("dihedral 30 m", dih, wf_d, small.array, 2, 4)]


@pytest.mark.parametrize("case", range(4))
def test_double_bounce_against_oracle(case):
    name, sc, wf, arr, P, Q = _cases()[case]
    arr = RadarArray(tx=np.array(arr.tx[:P]), rx=np.array(arr.rx[:Q]))
    _log(f"case double bounce: {name}, {sc.n_tris} triangles, {P}x{Q}, M={wf.n_samples}")
    sim = _sim(sc, wf, arr)
    F, N = sim.n_facets[0], wf.n_chirps
    pairs = dbounce.double_bounce_pairs(sc, arr, wf)
    want = dbounce.connection_table(pairs, F)
    n_pairs = int((want >= 0).sum())
    assert n_pairs > 0
    # 1. the library's connections
    mask = sim.mask_buffer()
    sim.synthesize(mask=mask)
    got = sim.connections_numpy(mask)[0]
    amb = np.zeros_like(want, bool)
    for ni, per in enumerate(pairs):
        for k in (0, 1):
            amb[k, ni, per[k]["amb_facets"]] = True
    diff = got != want
    _log(f"  connections: oracle {n_pairs}, library {int((got >= 0).sum())}, differing "
         f"{int(diff.sum())} (all on ambiguous decisions: {bool(not (diff & ~amb).any())}, "
         f"ambiguous {int(amb.sum())})")
    assert not (diff & ~amb).any()
    # 2. the double bounce alone on the oracle's connections
    m_in = sim.mask_with_connections([np.zeros((N, F), bool)], [want])
    H = sim.synthesize(mask=m_in, mask_mode=1, census=True).cpu().numpy()[0]
    n_rec = sum(sim.ctx.last_census().values())
    Ho = dbounce.synthesize_double(sc, wf, arr, pairs=pairs)
    err = rel_rms(H, Ho)
    _log(f"  records {n_rec}; double bounce alone rel_rms={err:.3e}")
    assert n_rec == n_pairs
    assert err <= FP32_TOL


def test_double_bounce_with_single_bounce():
    """The whole echo: the oracle's lit set and connections, against the oracle's single +
    double bounce; gamma complex."""
    cfg = scenes.small_single(n_samples=64, n_chirps=2, n_tris=6000)
    sc, wf = cfg.scenes[0], cfg.waveform
    arr = RadarArray(tx=np.array(cfg.array.tx[:4]), rx=np.array(cfg.array.rx[:4]))
    g = -0.8 + 0.3j
    _log("case double bounce + single bounce, 6k-triangle vehicle, gamma -0.8+0.3j")
    sim = _sim(sc, wf, arr, g)
    om, _ = oracle.visibility(sc, arr, wf)
    pairs = dbounce.double_bounce_pairs(sc, arr, wf)
    m_in = sim.mask_with_connections([om], [dbounce.connection_table(pairs, sim.n_facets[0])])
    H = sim.synthesize(mask=m_in, mask_mode=1).cpu().numpy()[0]
    Hd = dbounce.synthesize_double(sc, wf, arr, gamma=g, pairs=pairs)
    Ho = oracle.synthesize(sc, wf, arr, mask=om) + Hd
    err = rel_rms(H, Ho)
    _log(f"  rel_rms={err:.3e} (the double bounce is {rel_rms(Ho - Hd, Ho):.2f} of the echo)")
    assert err <= FP32_TOL


def test_dihedral_closed_form_on_gpu():
    """Far field (1e6 m), monostatic: the GPU's double bounce of a 0.3 x 0.2 m dihedral
    has the magnitude of the oracle's flat plate of area sqrt(2) a b."""
    p = scenes.RADAR_POS[None, :].astype(np.float64)
    arr = RadarArray(tx=p.copy(), rx=p.copy())
    wf = Waveform(f0=77e9, slope=12.5e12, fs=5.12e6, chirp_period=60e-6, n_samples=32,
                  n_chirps=1)
    D = 1e6
    sc = scenes.dihedral_scene(0.3, 0.2, D, 3, 2)
    _log("case dihedral closed form, far field")
    sim = _sim(sc, wf, arr)
    pairs = dbounce.double_bounce_pairs(sc, arr, wf)
    m_in = sim.mask_with_connections([np.zeros((1, sim.n_facets[0]), bool)],
                                     [dbounce.connection_table(pairs, sim.n_facets[0])])
    H = sim.synthesize(mask=m_in, mask_mode=1).cpu().numpy()[0, 0, 0]
    # the library finds the same connections (no decision is ambiguous here)
    mask = sim.mask_buffer()
    sim.synthesize(mask=mask)
    assert np.array_equal(sim.connections_numpy(mask)[0],
                          dbounce.connection_table(pairs, sim.n_facets[0]))
    Hp = oracle.synthesize(scenes.plate_scene(0.3, np.sqrt(2.0) * 0.2, 1, 1, D), wf, arr)[0, 0]
    r = np.abs(H) / np.abs(Hp)
    _log(f"  |H| / |H_plate| in [{r.min():.6f}, {r.max():.6f}]")
    assert np.allclose(r, 1.0, rtol=1e-4)


def _with_vertex(sc, mesh_k, vert, axis, dv):
    from scenes import Mesh, Scene
    meshes = []
    for k, m in enumerate(sc.meshes):
        v = m.verts.astype(np.float64)
        if k == mesh_k:
            v = v.copy()
            v[vert, axis] += dv
        meshes.append(Mesh(verts=v, tris=m.tris, name=m.name))
    return Scene(meshes, sc.instances)


def _with_velocity(sc, inst_k, axis, dv):
    from scenes import Instance, Scene
    insts = []
    for k, i in enumerate(sc.instances):
        vel = np.array(i.vel, np.float64).copy()
        if k == inst_k:
            vel[axis] += dv
        insts.append(Instance(i.mesh, i.rot, i.pos0, vel))
    return Scene(sc.meshes, insts)


@pytest.mark.parametrize("case", [0, 1])
def test_double_bounce_adjoint_matches_finite_differences(case):
    """rsim_backward with the double bounce on (NUFFT adjoint): each connection's sums go
    through the footprint construction to the vertices of both facets. Against central
    differences of the oracle's loss sum (RDM - T)^2 over the single-bounce echo (lit mask
    held) plus the double bounce of the held connection table (footprints recomputed from
    the perturbed scene), on vertices of connected facets and the velocity. The adjoint
    without the double bounce misses the bar, so the check sees its terms. Cases: the
    1.5k-triangle vehicle (4x6 channels; the double bounce 1.4% of the echo's norm) and the
    small intersection (ground grid and three motorcycles, 3x4 channels; ground-vehicle
    dihedrals, the double bounce 3.9 times the single bounce's norm)."""
    import torch
    if case == 0:
        cfg = scenes.small_single(n_samples=64, n_chirps=2, n_tris=1500)
        P, Q, name = 4, 6, "1.5k-triangle vehicle"
    else:
        cfg = scenes.small_intersection(n_samples=64, n_chirps=2)
        P, Q, name = 3, 4, "small intersection"
    sc, wf = cfg.scenes[0], cfg.waveform
    arr = RadarArray(tx=np.array(cfg.array.tx[:P]), rx=np.array(cfg.array.rx[:Q]))
    g = -0.8 + 0.3j
    _log(f"case double-bounce adjoint vs FD, {name}, {P}x{Q} channels, M=64, N=2")
    sim = _sim(sc, wf, arr, g)
    F = sim.n_facets[0]
    om, _ = oracle.visibility(sc, arr, wf)
    table = dbounce.connection_table(dbounce.double_bounce_pairs(sc, arr, wf), F)

    def echo(scene):
        return (oracle.synthesize(scene, wf, arr, mask=om) +
                dbounce.synthesize_double(scene, wf, arr, gamma=g,
                                          pairs=dbounce.pairs_for_table(scene, arr, wf, table)))

    P0, _ = oracle.rdm_from_echo(echo(sc))
    T = 0.5 * P0

    def loss(scene):
        P, _ = oracle.rdm_from_echo(echo(scene))
        return oracle.rdm_loss(P, T)

    m_in = sim.mask_with_connections([om], [table])
    H = sim.synthesize(mask=m_in, mask_mode=1)
    rdm, y = sim.form_rdm(H, want_y=True)
    ge = torch.empty_like(H)
    sim.ctx.rdm_backward((2.0 * (rdm - torch.from_numpy(T.astype(np.float32)).cuda()[None]))
                         .contiguous(), y, ge)

    def adjoint():
        gv = [torch.zeros((m.verts.shape[0], 3), dtype=torch.float32, device="cuda")
              for m in sc.meshes]
        gvel = torch.zeros((len(sc.instances), 3), dtype=torch.float64, device="cuda")
        sim.ctx.backward(sim.scene_ids[0], ge, m_in, gv, gvel)
        return [x.cpu().numpy().astype(np.float64) for x in gv], gvel.cpu().numpy()

    gverts, gvel = adjoint()
    sim.ctx.set_double_bounce(False)
    sv, svel = adjoint()
    sim.ctx.set_double_bounce(True, g)
    # vertices of the A and B facets of seeded connections
    rng = np.random.default_rng(31)
    tri, inst_of, local_of = oracle.world_triangles(sc, 0.0)
    kk, aa = np.nonzero(table[:, 0, :] >= 0)
    picks = []
    for i in rng.choice(aa.size, size=3, replace=False):
        for f in (aa[i], table[kk[i], 0, aa[i]]):
            mesh_k = sc.instances[inst_of[f]].mesh
            picks.append((mesh_k, int(sc.meshes[mesh_k].tris[local_of[f], rng.integers(0, 3)])))
    h, hv = 1e-5, 1e-2
    fd, ad, sh = [], [], []
    for (mk, v) in picks:
        for ax in range(3):
            fd.append((loss(_with_vertex(sc, mk, v, ax, h)) -
                       loss(_with_vertex(sc, mk, v, ax, -h))) / (2 * h))
            ad.append(gverts[mk][v, ax])
            sh.append(sv[mk][v, ax])
    moving = [k for k, i in enumerate(sc.instances) if np.any(np.asarray(i.vel) != 0.0)]
    for ax in range(2):
        ik = moving[0]
        fd.append((loss(_with_velocity(sc, ik, ax, hv)) - loss(_with_velocity(sc, ik, ax, -hv))) /
                  (2 * hv))
        ad.append(gvel[ik, ax])
        sh.append(svel[ik, ax])
    fd, ad, sh = np.array(fd), np.array(ad), np.array(sh)
    rel_l2 = np.linalg.norm(ad - fd) / np.linalg.norm(fd)
    big = np.abs(fd) > 1e-3 * np.abs(fd).max()
    rel_c = np.abs(ad - fd)[big] / np.abs(fd)[big]
    rel_sh = np.linalg.norm(sh - fd) / np.linalg.norm(fd)
    _log(f"  connections {int((table >= 0).sum())}; rel_l2={rel_l2:.3e} "
         f"max_rel_component={rel_c.max():.3e} (n={fd.size}); without the double bounce "
         f"rel_l2={rel_sh:.3e}")
    assert rel_l2 <= 1e-3
    assert rel_c.max() <= 1e-2
    assert rel_sh > 2e-3


def test_autograd_double_bounce_matches_direct_calls():
    """RadarRDM with Simulator.set_double_bounce(True): the forward finds the connections
    (kept with its mask) and the backward differentiates them with the table held (the
    same numbers as the explicit calls, up to the order of the FP64 atomic sums)."""
    import torch
    from paper_2208_10939_amd.autograd import RadarRDM
    cfg = scenes.small_single(n_samples=64, n_chirps=4, n_tris=1500)
    sc, wf = cfg.scenes[0], cfg.waveform
    arr = RadarArray(tx=np.array(cfg.array.tx[:4]), rx=np.array(cfg.array.rx[:6]))
    _log("case RadarRDM autograd with the facet-to-facet double bounce")
    sim = _sim(sc, wf, arr, -0.8 + 0.3j)
    verts = [torch.from_numpy(m.verts.copy()).requires_grad_(True) for m in sc.meshes]
    vel = torch.from_numpy(np.stack([i.vel for i in sc.instances])).requires_grad_(True)
    T = torch.from_numpy((0.5 * oracle.rdm_from_echo(oracle.synthesize(sc, wf, arr))[0])
                         .astype(np.float32)).cuda()
    ((RadarRDM.apply(sim, 0, vel, *verts) - T) ** 2).sum().backward()
    mask_t = sim.mask_buffer()
    echo = sim.synthesize(mask=mask_t)
    assert int((sim.connections_numpy(mask_t)[0] >= 0).sum()) > 0
    P, y = sim.form_rdm(echo, want_y=True)
    ge = torch.empty_like(echo)
    sim.ctx.rdm_backward((2.0 * (P - T[None])).contiguous(), y, ge)
    gv = [torch.zeros((m.verts.shape[0], 3), dtype=torch.float32, device="cuda")
          for m in sc.meshes]
    gvel = torch.zeros((len(sc.instances), 3), dtype=torch.float64, device="cuda")
    sim.ctx.backward(sim.scene_ids[0], ge, mask_t, gv, gvel)
    assert torch.allclose(verts[0].grad.cuda(), gv[0], rtol=1e-5,
                          atol=1e-6 * gv[0].abs().max().item())
    assert torch.allclose(vel.grad.cuda(), gvel, rtol=1e-5, atol=1e-8 * gvel.abs().max().item())


def test_double_bounce_chunked_equals_whole():
    """Chirps in chunks of at most 3 (rsim_set_nufft_chunk) against one chunk, with the
    double bounce: the forward echo bit for bit; the adjoint's gradients to the last bits
    of the connections' FP64 atomic sums (their order differs)."""
    import torch
    cfg = scenes.small_single(n_samples=64, n_chirps=8, n_tris=1500)
    sc, wf = cfg.scenes[0], cfg.waveform
    arr = RadarArray(tx=np.array(cfg.array.tx[:4]), rx=np.array(cfg.array.rx[:6]))
    _log("case double bounce, nufft chunks of 3 chirps vs one chunk (N=8), forward and adjoint")
    sim = _sim(sc, wf, arr, -0.8 + 0.3j)
    mask = sim.mask_buffer()
    O = arr.tx.shape[0] * arr.rx.shape[0]
    rng = np.random.default_rng(9)
    g = (rng.standard_normal((O, wf.n_chirps, wf.n_samples)) +
         1j * rng.standard_normal((O, wf.n_chirps, wf.n_samples))).astype(np.complex64)
    ge = torch.from_numpy(g).cuda()
    res = {}
    for chunk in (0, 3):
        sim.ctx.set_nufft_chunk(chunk)
        H = sim.synthesize(mask=mask).cpu().numpy()
        gv = [torch.zeros((m.verts.shape[0], 3), dtype=torch.float32, device="cuda")
              for m in sc.meshes]
        gvel = torch.zeros((len(sc.instances), 3), dtype=torch.float64, device="cuda")
        sim.ctx.backward(sim.scene_ids[0], ge, mask, gv, gvel)
        res[chunk] = (H, np.concatenate([x.cpu().numpy().ravel() for x in gv]).astype(np.float64),
                      gvel.cpu().numpy().ravel())
    sim.ctx.set_nufft_chunk(0)
    assert int((sim.connections_numpy(mask)[0] >= 0).sum()) > 0
    dh = rel_rms(res[3][0], res[0][0])
    dv = np.linalg.norm(res[3][1] - res[0][1]) / np.linalg.norm(res[0][1])
    dw = np.linalg.norm(res[3][2] - res[0][2]) / np.linalg.norm(res[0][2])
    _log(f"  echo rel_rms={dh:.3e}, vertex gradients {dv:.3e}, velocity gradients {dw:.3e}")
    assert dh == 0.0
    assert dv <= 1e-6 and dw <= 1e-10


def test_double_bounce_refusals():
    from paper_2208_10939_amd.rsim import RsimError
    cfg = scenes.small_single(n_samples=32, n_chirps=2, n_tris=300)
    sc, wf = cfg.scenes[0], cfg.waveform
    arr = RadarArray(tx=np.array(cfg.array.tx[:2]), rx=np.array(cfg.array.rx[:2]))
    sim = _sim(sc, wf, arr)
    for kw in ({"kernel": 1}, {"kernel": 2}, {"precision": 1}, {"intra_chirp": True}):
        with pytest.raises(RsimError) as e:
            sim.synthesize(**kw)
        assert e.value.code == -1, kw  # EINVAL
    with pytest.raises(RsimError) as e:
        sim.ctx.autotune(sim.scene_ids)
    assert e.value.code == -4  # ESTATE
    # the backward: the NUFFT adjoint only
    import torch
    mask = sim.mask_buffer()
    H = sim.synthesize(mask=mask)
    gv = [torch.zeros((m.verts.shape[0], 3), dtype=torch.float32, device="cuda")
          for m in sc.meshes]
    gvel = torch.zeros((len(sc.instances), 3), dtype=torch.float64, device="cuda")
    for k in (1, 2):
        sim.ctx.set_backward_kernel(k)
        with pytest.raises(RsimError) as e:
            sim.ctx.backward(sim.scene_ids[0], H, mask, gv, gvel)
        assert e.value.code == -1, k  # EINVAL
    sim.ctx.set_backward_kernel(0)
    sim.ctx.set_double_bounce(False)
    sim.synthesize(kernel=1)  # the direct kernels again


def test_connections_full_size_sampled():
    """The 50k-triangle vehicle at its full array and waveform (192 channels, 256 x 128),
    chirps 0 and 127: the library's connection of 400 seeded facets per chirp against the
    oracle's, launched from those facets over the whole scene (differences only on
    decisions the oracle marks ambiguous)."""
    cfg = scenes.c2()
    sc, wf, arr = cfg.scenes[0], cfg.waveform, cfg.array
    _log("case double bounce connections, 50k-triangle vehicle, full frame, sampled")
    sim = _sim(sc, wf, arr)
    F = sim.n_facets[0]
    mask = sim.mask_buffer()
    sim.synthesize(mask=mask)
    got = sim.connections_numpy(mask)[0]
    rng = np.random.default_rng(77)
    sample = np.sort(rng.choice(F, 400, replace=False))
    total = 0
    for n in (0, wf.n_chirps - 1):
        per = dbounce.double_bounce_pairs(sc, arr, wf, chirps=[n], facets=sample)[0]
        for k in (0, 1):
            want = np.full(F, -1, np.int32)
            want[per[k]["A"]] = per[k]["B"]
            amb = np.zeros(F, bool)
            amb[per[k]["amb_facets"]] = True
            diff = (got[k, n, sample] != want[sample]) & ~amb[sample]
            total += int((want[sample] >= 0).sum())
            assert not diff.any(), (n, k, sample[diff][:5])
    _log(f"  {total} connections among the samples match; the whole frame has "
         f"{int((got >= 0).sum())}")
    assert total > 0
