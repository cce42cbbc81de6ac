"""GPU adjoint vs FP64 central finite differences of the oracle's RDM loss.

Loss L = sum (RDM - T)^2 with T the oracle RDM of a perturbed copy of the scene. The
lit-facet mask is the oracle's and is held fixed on both sides (the GPU receives it as
an input mask). Finite differences perturb body-frame vertices (in float64, oracle
only) and instance velocities."""
import sys

import numpy as np
import pytest

import oracle
import scenes
from scenes import Instance, Mesh, RadarArray, Scene

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _setup():
    wf = scenes.paper_waveform(32, 8)
    full = scenes.sparse_mimo_12x16(wf, 5)
    arr = RadarArray(tx=full.tx[:3].copy(), rx=full.rx[:5].copy())
    car = scenes.vehicle_mesh("car", 700)
    moto = scenes.vehicle_mesh("motorcycle", 400)
    insts = [Instance(0, scenes.yaw_matrix(1.5), np.array([3.0, 18.0, 0.0]), np.array([0.3, -6.0, 0.0])),
             Instance(1, scenes.yaw_matrix(-1.4), np.array([-4.0, 24.0, 0.0]), np.array([-0.5, 4.0, 0.0]))]
    sc = Scene([car, moto], insts)
    target = scenes.perturbed(sc, 77, pos_sigma=0.02, vel_sigma=0.3, vert_sigma=2e-3)
    return wf, arr, sc, target


def _with(sc, mesh_k=None, vert=None, axis=None, dv=0.0, inst_k=None, vaxis=None, dvel=0.0):
    meshes = []
    for k, m in enumerate(sc.meshes):
        v = m.verts.astype(np.float64)
        if k == mesh_k:
            v = v.copy()
            v[vert, axis] += dv
        meshes.append(Mesh(verts=v, tris=m.tris, name=m.name))
    insts = []
    for k, i in enumerate(sc.instances):
        vel = i.vel.copy()
        if k == inst_k:
            vel[vaxis] += dvel
        insts.append(Instance(i.mesh, i.rot, i.pos0, vel))
    return Scene(meshes, insts)


@pytest.mark.parametrize("kernel", [1, 2, 3])
def test_adjoint_ground_bounce_matches_finite_differences(kernel):
    """With the ground plane (gamma -0.7 + 0.2j): the backward differentiates all four path
    types (their masks from the oracle, held fixed) against central differences of the
    oracle's loss over the image-method echo (oracle/bounce.py)."""
    import torch
    from oracle import bounce
    from paper_2208_10939_amd.pipeline import Simulator, pack_mask
    g = -0.7 + 0.2j
    _log(f"case adjoint with the ground bounce vs FD, kernel={kernel}")
    wf, arr, sc, target = _setup()
    masks, amb = bounce.visibility_bounce(sc, arr, wf, 0.0)
    T, _ = oracle.rdm_from_echo(bounce.synthesize_bounce(target, wf, arr, 0.0, g))

    def loss(scene):
        P, _ = oracle.rdm_from_echo(bounce.synthesize_bounce(scene, wf, arr, 0.0, g, masks=masks))
        return oracle.rdm_loss(P, T)

    sim = Simulator([sc], wf, arr)
    sim.set_ground(True, 0.0, g)
    packed = np.concatenate([pack_mask(masks[k]).reshape(-1) for k in range(4)])
    m_t = torch.from_numpy(packed.view(np.int32).copy()).cuda()
    echo = sim.synthesize(mask=m_t, mask_mode=1)
    rdm, y = sim.form_rdm(echo, want_y=True)
    Tt = torch.from_numpy(T.astype(np.float32)).cuda()[None]
    grad_echo = torch.empty_like(echo)
    sim.ctx.rdm_backward((2.0 * (rdm - Tt)).contiguous(), y, grad_echo)
    gverts = [torch.zeros((m.verts.shape[0], 3), dtype=torch.float32, device="cuda")
              for m in sc.meshes]
    gvel = torch.zeros((len(sc.instances), 3), dtype=torch.float64, device="cuda")
    sim.ctx.set_backward_kernel(kernel)
    sim.ctx.backward(sim.scene_ids[0], grad_echo, m_t, gverts, gvel)
    gverts = [g_.cpu().numpy().astype(np.float64) for g_ in gverts]
    gvel = gvel.cpu().numpy()
    rng = np.random.default_rng(12)
    tri, inst_of, local_of = oracle.world_triangles(sc, 0.0)
    lit_f = np.nonzero(masks[:, 0].any(axis=0))[0]
    picks = []
    for f in rng.choice(lit_f, size=6, replace=False):
        k = inst_of[f]
        picks.append((sc.instances[k].mesh,
                      int(sc.meshes[sc.instances[k].mesh].tris[local_of[f], rng.integers(0, 3)])))
    h = 1e-5
    fd, ad = [], []
    for (mk, v) in picks:
        for ax in range(3):
            fd.append((loss(_with(sc, mk, v, ax, +h)) - loss(_with(sc, mk, v, ax, -h))) / (2 * h))
            ad.append(gverts[mk][v, ax])
    hv = 1e-2
    for ik in range(len(sc.instances)):
        for ax in range(2):
            fd.append((loss(_with(sc, inst_k=ik, vaxis=ax, dvel=+hv)) -
                       loss(_with(sc, inst_k=ik, vaxis=ax, dvel=-hv))) / (2 * hv))
            ad.append(gvel[ik, ax])
    fd, ad = np.array(fd), np.array(ad)
    rel_l2 = np.linalg.norm(ad - fd) / np.linalg.norm(fd)
    big = np.abs(fd) > 1e-3 * np.abs(fd).max()
    rel_c = np.abs(ad - fd)[big] / np.abs(fd)[big]
    _log(f"  lit per type {[int(masks[k].sum()) for k in range(4)]} rel_l2={rel_l2:.3e} "
         f"max_rel_component={rel_c.max():.3e} (n={fd.size}, ambiguous={int(amb.sum())})")
    assert rel_l2 <= 1e-3
    assert rel_c.max() <= 1e-2


@pytest.mark.parametrize("M,N", [(32, 8), (144, 4)])
def test_adjoint_intra_chirp_matches_finite_differences(M, N):
    """The delay within the chirp (eq. (12) at the sample times; rsim_set_backward_intra_chirp):
    the vector-unit adjoint of that echo against central differences of the oracle's loss
    over its intra-chirp echo (vertices, and velocities, which now also move each facet
    within the chirp). M = 144 spans three 64-sample blocks of the adjoint (the last
    ragged), each with its own chord. The stop-and-hop adjoint of the same echo gradient
    misses the bar, so the check sees the chirp delay's terms."""
    import torch
    from paper_2208_10939_amd.pipeline import Simulator
    _log(f"case intra-chirp adjoint vs FD (2 vehicles, 3x5 channels, M={M}, N={N})")
    wf0, arr, sc, target = _setup()
    wf = scenes.paper_waveform(M, N)
    mask, amb = oracle.visibility(sc, arr, wf)
    T, _ = oracle.rdm_from_echo(oracle.synthesize(target, wf, arr, intra_chirp=True))

    def loss(scene):
        P, _ = oracle.rdm_from_echo(oracle.synthesize(scene, wf, arr, mask=mask, intra_chirp=True))
        return oracle.rdm_loss(P, T)

    sim = Simulator([sc], wf, arr)
    m_t = sim.mask_from_numpy([mask])
    echo = sim.synthesize(mask=m_t, mask_mode=1, intra_chirp=True)
    rdm, y = sim.form_rdm(echo, want_y=True)
    Tt = torch.from_numpy(T.astype(np.float32)).cuda()[None]
    grad_echo = torch.empty_like(echo)
    sim.ctx.rdm_backward((2.0 * (rdm - Tt)).contiguous(), y, grad_echo)

    def adjoint(intra):
        gv = [torch.zeros((m.verts.shape[0], 3), dtype=torch.float32, device="cuda")
              for m in sc.meshes]
        gvl = torch.zeros((len(sc.instances), 3), dtype=torch.float64, device="cuda")
        sim.ctx.set_backward_intra_chirp(intra)
        sim.ctx.set_backward_kernel(0)
        sim.ctx.backward(sim.scene_ids[0], grad_echo, m_t, gv, gvl)
        return [g.cpu().numpy().astype(np.float64) for g in gv], gvl.cpu().numpy()

    gverts, gvel = adjoint(True)
    sv, svel = adjoint(False)
    rng = np.random.default_rng(13)
    tri, inst_of, local_of = oracle.world_triangles(sc, 0.0)
    lit_f = np.nonzero(mask[0])[0]
    picks = []
    for f in rng.choice(lit_f, size=6, replace=False):
        k = inst_of[f]
        picks.append((sc.instances[k].mesh,
                      int(sc.meshes[sc.instances[k].mesh].tris[local_of[f], rng.integers(0, 3)])))
    h, hv = 1e-5, 1e-2
    fd, ad, sh = [], [], []
    for (mk, v) in picks:
        for ax in range(3):
            fd.append((loss(_with(sc, mk, v, ax, +h)) - loss(_with(sc, mk, v, ax, -h))) / (2 * h))
            ad.append(gverts[mk][v, ax])
            sh.append(sv[mk][v, ax])
    for ik in range(len(sc.instances)):
        for ax in range(2):
            fd.append((loss(_with(sc, inst_k=ik, vaxis=ax, dvel=+hv)) -
                       loss(_with(sc, inst_k=ik, vaxis=ax, dvel=-hv))) / (2 * hv))
            ad.append(gvel[ik, ax])
            sh.append(svel[ik, ax])
    fd, ad, sh = np.array(fd), np.array(ad), np.array(sh)
    rel_l2 = np.linalg.norm(ad - fd) / np.linalg.norm(fd)
    big = np.abs(fd) > 1e-3 * np.abs(fd).max()
    rel_c = np.abs(ad - fd)[big] / np.abs(fd)[big]
    rel_sh = np.linalg.norm(sh - fd) / np.linalg.norm(fd)
    _log(f"  rel_l2={rel_l2:.3e} max_rel_component={rel_c.max():.3e} (n={fd.size}, "
         f"ambiguous={int(amb.sum())}); the stop-and-hop adjoint: rel_l2={rel_sh:.3e}")
    assert rel_l2 <= 1e-3
    assert rel_c.max() <= 1e-2
    assert rel_sh > 2e-3


def test_autograd_intra_chirp_matches_direct_calls():
    """RadarRDM with Simulator.set_intra_chirp(True): the forward takes the chirp delay and
    the backward differentiates it (the same numbers as the explicit calls)."""
    import torch
    from paper_2208_10939_amd.autograd import RadarRDM
    from paper_2208_10939_amd.pipeline import Simulator
    _log("case RadarRDM autograd with the delay within the chirp")
    wf, arr, sc, target = _setup()
    sim = Simulator([sc], wf, arr)
    sim.set_intra_chirp(True)
    verts = [torch.from_numpy(m.verts.copy()).requires_grad_(True) for m in sc.meshes]
    vel = torch.from_numpy(np.stack([i.vel for i in sc.instances])).requires_grad_(True)
    T = torch.from_numpy(oracle.rdm_from_echo(oracle.synthesize(target, wf, arr))[0]
                         .astype(np.float32)).cuda()
    ((RadarRDM.apply(sim, 0, vel, *verts) - T) ** 2).sum().backward()
    mask_t = sim.mask_buffer()
    echo = sim.synthesize(mask=mask_t, intra_chirp=True)
    P, y = sim.form_rdm(echo, want_y=True)
    ge = torch.empty_like(echo)
    sim.ctx.rdm_backward((2.0 * (P - T[None])).contiguous(), y, ge)
    gv = [torch.zeros((m.verts.shape[0], 3), dtype=torch.float32, device="cuda") for m in sc.meshes]
    gvel = torch.zeros((2, 3), dtype=torch.float64, device="cuda")
    sim.ctx.set_backward_intra_chirp(True)
    sim.ctx.backward(sim.scene_ids[0], ge, mask_t, gv, gvel)
    assert torch.allclose(verts[0].grad.cuda(), gv[0], rtol=1e-5, atol=1e-6 * gv[0].abs().max().item())
    assert torch.allclose(vel.grad.cuda(), gvel, rtol=1e-5, atol=1e-8 * gvel.abs().max().item())


@pytest.mark.parametrize("kernel", [1, 2, 3])
def test_adjoint_matches_finite_differences(kernel):
    """kernel 1: the vector-unit adjoint; 2: the matrix-core adjoint; 3: the NUFFT adjoint
    (type-2 gather of Gaussian moments; Taylor-coefficient derivatives by FP64 central
    differences)."""
    import torch
    from paper_2208_10939_amd.pipeline import Simulator
    _log(f"case adjoint vs FD (2 vehicles, 3x5 channels, M=32, N=8), kernel={kernel}")
    wf, arr, sc, target = _setup()
    mask, amb = oracle.visibility(sc, arr, wf)
    T, _ = oracle.rdm_from_echo(oracle.synthesize(target, wf, arr))

    def loss(scene):
        P, _ = oracle.rdm_from_echo(oracle.synthesize(scene, wf, arr, mask=mask))
        return oracle.rdm_loss(P, T)

    sim = Simulator([sc], wf, arr)
    m_t = sim.mask_from_numpy([mask])
    echo = sim.synthesize(mask=m_t, mask_mode=1)
    rdm, y = sim.form_rdm(echo, want_y=True)
    Tt = torch.from_numpy(T.astype(np.float32)).cuda()[None]
    grad_rdm = 2.0 * (rdm - Tt)
    grad_echo = torch.empty_like(echo)
    sim.ctx.rdm_backward(grad_rdm.contiguous(), y, grad_echo)
    gverts = [torch.zeros((m.verts.shape[0], 3), dtype=torch.float32, device="cuda")
              for m in sc.meshes]
    gvel = torch.zeros((len(sc.instances), 3), dtype=torch.float64, device="cuda")
    sim.ctx.set_backward_kernel(kernel)
    sim.ctx.backward(sim.scene_ids[0], grad_echo, m_t, gverts, gvel)
    gverts = [g.cpu().numpy().astype(np.float64) for g in gverts]
    gvel = gvel.cpu().numpy()

    # sampled vertices of facets lit at chirp 0
    rng = np.random.default_rng(11)
    tri, inst_of, local_of = oracle.world_triangles(sc, 0.0)
    lit_f = np.nonzero(mask[0])[0]
    picks = []
    for f in rng.choice(lit_f, size=8, replace=False):
        k = inst_of[f]
        picks.append((sc.instances[k].mesh, int(sc.meshes[sc.instances[k].mesh].tris[local_of[f], rng.integers(0, 3)])))
    h = 1e-5
    fd, ad = [], []
    for (mk, v) in picks:
        for ax in range(3):
            lp = loss(_with(sc, mk, v, ax, +h))
            lm = loss(_with(sc, mk, v, ax, -h))
            fd.append((lp - lm) / (2 * h))
            ad.append(gverts[mk][v, ax])
    hv = 1e-2
    for ik in range(len(sc.instances)):
        for ax in range(2):
            lp = loss(_with(sc, inst_k=ik, vaxis=ax, dvel=+hv))
            lm = loss(_with(sc, inst_k=ik, vaxis=ax, dvel=-hv))
            fd.append((lp - lm) / (2 * hv))
            ad.append(gvel[ik, ax])
    fd = np.array(fd)
    ad = np.array(ad)
    rel_l2 = np.linalg.norm(ad - fd) / np.linalg.norm(fd)
    big = np.abs(fd) > 1e-3 * np.abs(fd).max()
    rel_c = np.abs(ad - fd)[big] / np.abs(fd)[big]
    _log(f"  L={loss(sc):.4e} rel_l2={rel_l2:.3e} max_rel_component={rel_c.max():.3e} "
         f"(n={fd.size}, ambiguous={amb.sum()})")
    for a, b in zip(ad, fd):
        _log(f"    adj {a:+.6e} fd {b:+.6e}")
    assert rel_l2 <= 1e-3
    assert rel_c.max() <= 1e-2


@pytest.mark.parametrize("kernel", [0, 3])
def test_adjoint_full_array_matches_finite_differences(kernel):
    """Same check with the 12 x 16 sparse array (192 channels: whole-wave workgroups,
    the DPP reduction path) at a small frame; kernel 0: the default choice, 3: the NUFFT
    adjoint (three channel groups adding into one facet)."""
    import torch
    from paper_2208_10939_amd.pipeline import Simulator
    _log(f"case adjoint vs FD (192 channels, M=16, N=4), kernel={kernel}")
    wf = scenes.paper_waveform(16, 4)
    arr = scenes.sparse_mimo_12x16(wf, 6)
    car = scenes.vehicle_mesh("car", 500)
    sc = Scene([car], [Instance(0, scenes.yaw_matrix(1.6), np.array([2.0, 15.0, 0.0]),
                                np.array([0.2, -5.0, 0.0]))])
    target = scenes.perturbed(sc, 78, pos_sigma=0.02, vel_sigma=0.3, vert_sigma=2e-3)
    mask, amb = oracle.visibility(sc, arr, wf)
    T, _ = oracle.rdm_from_echo(oracle.synthesize(target, wf, arr))

    def loss(scene):
        P, _ = oracle.rdm_from_echo(oracle.synthesize(scene, wf, arr, mask=mask))
        return oracle.rdm_loss(P, T)

    sim = Simulator([sc], wf, arr)
    m_t = sim.mask_from_numpy([mask])
    echo = sim.synthesize(mask=m_t, mask_mode=1)
    rdm, y = sim.form_rdm(echo, want_y=True)
    grad_rdm = 2.0 * (rdm - torch.from_numpy(T.astype(np.float32)).cuda()[None])
    ge = torch.empty_like(echo)
    sim.ctx.rdm_backward(grad_rdm.contiguous(), y, ge)
    gv = [torch.zeros((car.verts.shape[0], 3), dtype=torch.float32, device="cuda")]
    gvel = torch.zeros((1, 3), dtype=torch.float64, device="cuda")
    sim.ctx.set_backward_kernel(kernel)
    sim.ctx.backward(sim.scene_ids[0], ge, m_t, gv, gvel)
    gv = gv[0].cpu().numpy().astype(np.float64)
    gvel = gvel.cpu().numpy()
    rng = np.random.default_rng(12)
    lit_f = np.nonzero(mask[0])[0]
    verts = [int(car.tris[f, rng.integers(0, 3)]) for f in rng.choice(lit_f, 4, replace=False)]
    fd, ad = [], []
    for v in verts:
        for ax in range(3):
            d = (loss(_with(sc, 0, v, ax, 1e-5)) - loss(_with(sc, 0, v, ax, -1e-5))) / 2e-5
            fd.append(d)
            ad.append(gv[v, ax])
    for ax in range(2):
        d = (loss(_with(sc, inst_k=0, vaxis=ax, dvel=1e-2)) -
             loss(_with(sc, inst_k=0, vaxis=ax, dvel=-1e-2))) / 2e-2
        fd.append(d)
        ad.append(gvel[0, ax])
    fd, ad = np.array(fd), np.array(ad)
    rel_l2 = np.linalg.norm(ad - fd) / np.linalg.norm(fd)
    _log(f"  rel_l2={rel_l2:.3e} (n={fd.size})")
    assert rel_l2 <= 1e-3


def test_autograd_function_matches_direct_calls():
    import torch
    from paper_2208_10939_amd.autograd import RadarRDM
    from paper_2208_10939_amd.pipeline import Simulator
    _log("case RadarRDM autograd")
    wf, arr, sc, target = _setup()
    sim = Simulator([sc], wf, arr)
    verts = [torch.from_numpy(m.verts.copy()).requires_grad_(True) for m in sc.meshes]
    vel = torch.from_numpy(np.stack([i.vel for i in sc.instances])).requires_grad_(True)
    rdm = RadarRDM.apply(sim, 0, vel, *verts)
    T, _ = oracle.rdm_from_echo(oracle.synthesize(target, wf, arr))
    L = ((rdm - torch.from_numpy(T.astype(np.float32)).cuda()) ** 2).sum()
    L.backward()
    assert verts[0].grad is not None and vel.grad is not None
    assert torch.isfinite(verts[0].grad).all() and torch.isfinite(vel.grad).all()
    assert verts[0].grad.abs().max() > 0
    # same numbers through the explicit calls with the forward's own mask
    mask_t = sim.mask_buffer()
    echo = sim.synthesize(mask=mask_t)
    P, y = sim.form_rdm(echo, want_y=True)
    ge = torch.empty_like(echo)
    sim.ctx.rdm_backward((2.0 * (P - torch.from_numpy(T.astype(np.float32)).cuda()[None])).contiguous(), y, ge)
    gv = [torch.zeros((m.verts.shape[0], 3), dtype=torch.float32, device="cuda") for m in sc.meshes]
    gvel = torch.zeros((2, 3), dtype=torch.float64, device="cuda")
    sim.ctx.backward(sim.scene_ids[0], ge, mask_t, gv, gvel)
    assert torch.allclose(verts[0].grad.cuda(), gv[0], rtol=1e-5, atol=1e-6 * gv[0].abs().max().item())
    assert torch.allclose(vel.grad.cuda(), gvel, rtol=1e-5, atol=1e-8 * gvel.abs().max().item())


def test_autograd_two_forwards_one_backward():
    """Two RadarRDM applies on one simulator with different vertices and velocities, one
    backward through the sum of their losses: each apply's gradient is taken at its own
    geometry (the backward re-loads it), so the result equals the two separate
    backwards added."""
    import torch
    from paper_2208_10939_amd.autograd import RadarRDM
    from paper_2208_10939_amd.pipeline import Simulator
    _log("case RadarRDM: two forwards, one backward")
    wf, arr, sc, target = _setup()
    sim = Simulator([sc], wf, arr)
    T = torch.from_numpy(oracle.rdm_from_echo(oracle.synthesize(target, wf, arr))[0]
                         .astype(np.float32)).cuda()
    rng = np.random.default_rng(5)
    geo = []
    for k in range(2):
        vs = [m.verts.copy() + (k * rng.normal(scale=2e-3, size=m.verts.shape)).astype(np.float32)
              for m in sc.meshes]
        vel = np.stack([i.vel for i in sc.instances]) + k * np.array([0.3, -0.2, 0.0])
        geo.append((vs, vel))

    def leaves(k):
        vs, vel = geo[k]
        return ([torch.from_numpy(v.copy()).requires_grad_(True) for v in vs],
                torch.from_numpy(vel.copy()).requires_grad_(True))

    sep = []
    for k in range(2):
        verts, vel = leaves(k)
        L = ((RadarRDM.apply(sim, 0, vel, *verts) - T) ** 2).sum()
        L.backward()
        sep.append(([v.grad.clone() for v in verts], vel.grad.clone()))
    (v0, vel0), (v1, vel1) = leaves(0), leaves(1)
    L = (((RadarRDM.apply(sim, 0, vel0, *v0) - T) ** 2).sum() +
         ((RadarRDM.apply(sim, 0, vel1, *v1) - T) ** 2).sum())
    L.backward()
    for j in range(len(sc.meshes)):
        want = [sep[0][0][j], sep[1][0][j]]
        got = [v0[j].grad, v1[j].grad]
        for a, b in zip(got, want):
            assert torch.allclose(a, b, rtol=1e-5, atol=1e-6 * b.abs().max().item())
    assert torch.allclose(vel0.grad, sep[0][1], rtol=1e-5, atol=1e-8 * sep[0][1].abs().max().item())
    assert torch.allclose(vel1.grad, sep[1][1], rtol=1e-5, atol=1e-8 * sep[1][1].abs().max().item())
    # the two geometries give different gradients (the check above is not vacuous)
    assert not torch.allclose(sep[0][1], sep[1][1], rtol=1e-3, atol=0.0)


@pytest.mark.parametrize("P,Q,M", [(12, 16, 96), (3, 5, 64), (1, 4, 160), (6, 8, 40)])
def test_matrix_adjoint_equals_vector_adjoint(P, Q, M):
    """The matrix-core adjoint against the vector-unit one on the same gradient input:
    vertex and velocity gradients within 1e-4 relative L2 (FP32 sums in different orders,
    and the Tx-Rx cross term the matrix cores drop, <= 1e-5). Sample counts leave a ragged
    64-sample tile; a 1500-triangle vehicle gives hundreds of 4-facet tiles per chirp."""
    import torch
    from paper_2208_10939_amd.pipeline import Simulator
    _log(f"case matrix-core vs vector-unit adjoint, P={P} Q={Q} M={M}")
    cfg = scenes.small_single(n_samples=M, n_chirps=3)
    sc, wf = cfg.scenes[0], cfg.waveform
    arr = RadarArray(tx=np.array(cfg.array.tx[:P]), rx=np.array(cfg.array.rx[:Q]))
    sim = Simulator([sc], wf, arr)
    mask = sim.mask_buffer()
    echo = sim.synthesize(mask=mask)
    rng = np.random.default_rng(P * 100 + Q)
    g = rng.normal(size=echo.shape) + 1j * rng.normal(size=echo.shape)
    ge = torch.from_numpy(g.astype(np.complex64)).cuda()
    out = {}
    for kernel in (1, 2):
        gv = [torch.zeros((m.verts.shape[0], 3), dtype=torch.float32, device="cuda")
              for m in sc.meshes]
        gvel = torch.zeros((len(sc.instances), 3), dtype=torch.float64, device="cuda")
        sim.ctx.set_backward_kernel(kernel)
        sim.ctx.backward(sim.scene_ids[0], ge, mask, gv, gvel)
        out[kernel] = (np.concatenate([x.cpu().numpy().ravel() for x in gv]).astype(np.float64),
                       gvel.cpu().numpy().ravel())
    dv = np.linalg.norm(out[2][0] - out[1][0]) / np.linalg.norm(out[1][0])
    dvel = np.linalg.norm(out[2][1] - out[1][1]) / np.linalg.norm(out[1][1])
    _log(f"  lit/chirp={sim.masks_numpy(mask)[0].sum(1)} vertices rel_l2={dv:.3e} "
         f"velocity rel_l2={dvel:.3e}")
    assert dv <= 1e-4 and dvel <= 1e-4
    # the same call twice gives the same gradients (no atomics: deterministic)
    gv2 = [torch.zeros((m.verts.shape[0], 3), dtype=torch.float32, device="cuda")
           for m in sc.meshes]
    gvel2 = torch.zeros((len(sc.instances), 3), dtype=torch.float64, device="cuda")
    sim.ctx.backward(sim.scene_ids[0], ge, mask, gv2, gvel2)
    again = np.concatenate([x.cpu().numpy().ravel() for x in gv2]).astype(np.float64)
    assert np.array_equal(again, out[2][0])
