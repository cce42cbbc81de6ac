"""torch.autograd.Function around the echo synthesis and RDM with the library's
hand-written adjoint. Visibility is decided in the forward call and held fixed in
the backward; the backward recomputes every chirp inside the library."""
from __future__ import annotations

import torch

from .pipeline import Simulator


class RadarRDM(torch.autograd.Function):
    """rdm = RadarRDM.apply(sim, scene_index, vel, *verts)

    sim         Simulator holding the scene (sim.intra_chirp: the delay within the chirp in
                the forward and the backward; Simulator.set_intra_chirp)
    scene_index index into sim.scene_ids
    vel         [n_instances, 3] float64 tensor: instance velocities (world frame)
    verts       one [n_verts, 3] float32 tensor per mesh of the scene, body frame
    returns     [O, N, M] float32 power RDM (Doppler rows shifted)
    """

    @staticmethod
    def _load_geometry(sim: Simulator, scene_index: int, verts_np, vel_np):
        """Upload this call's vertices and velocities into the library's scene."""
        sid = sim.scene_ids[scene_index]
        for mid, v in zip(sim.ctx.scene_meshes[sid], verts_np):
            sim.ctx.update_mesh(mid, v)
        pos0 = sim.inst_pos0[scene_index]
        for i in range(len(pos0)):
            sim.ctx.set_instance_motion(sid, i, pos0[i], vel_np[i])

    @staticmethod
    def forward(ctx, sim: Simulator, scene_index: int, vel, *verts):
        sid = sim.scene_ids[scene_index]
        meshes = sim.ctx.scene_meshes[sid]
        verts_np = [v.detach().cpu().numpy().copy() for v in verts]
        vel_np = vel.detach().cpu().numpy().copy()
        RadarRDM._load_geometry(sim, scene_index, verts_np, vel_np)
        pos0 = sim.inst_pos0[scene_index]
        mask = sim.mask_buffer([scene_index])
        echo = sim.synthesize([scene_index], mask=mask, intra_chirp=sim.intra_chirp)
        rdm, y = sim.form_rdm(echo, want_y=True)
        ctx.sim = sim
        ctx.scene_index = scene_index
        ctx.meshes = meshes
        ctx.n_verts = [v.shape[0] for v in verts]
        ctx.vert_devices = [v.device for v in verts]
        ctx.vel_device = vel.device
        ctx.n_inst = len(pos0)
        ctx.intra_chirp = sim.intra_chirp
        # the backward recomputes the chirps from the library's scene, which a later
        # forward on the same simulator may have replaced: keep this call's geometry
        ctx.verts_np = verts_np
        ctx.vel_np = vel_np
        ctx.save_for_backward(mask, y)
        return rdm[0]

    @staticmethod
    def backward(ctx, grad_rdm):
        mask, y = ctx.saved_tensors
        sim = ctx.sim
        dev = y.device
        g = grad_rdm.to(torch.float32).contiguous().reshape(y.shape)
        grad_echo = torch.empty_like(y)
        sim.ctx.rdm_backward(g, y, grad_echo)
        n_mesh_ids = max(ctx.meshes) + 1
        per_id = [None] * n_mesh_ids
        grads = []
        for mid, nv in zip(ctx.meshes, ctx.n_verts):
            t = torch.zeros((nv, 3), dtype=torch.float32, device=dev)
            per_id[mid] = t
            grads.append(t)
        grad_vel = torch.zeros((ctx.n_inst, 3), dtype=torch.float64, device=dev)
        RadarRDM._load_geometry(sim, ctx.scene_index, ctx.verts_np, ctx.vel_np)
        sim.ctx.set_backward_intra_chirp(ctx.intra_chirp)
        sim.ctx.backward(sim.scene_ids[ctx.scene_index], grad_echo, mask, per_id, grad_vel)
        grads = [g.to(d) for g, d in zip(grads, ctx.vert_devices)]
        return (None, None, grad_vel.to(ctx.vel_device), *grads)
