"""Scene state per chirp and facet geometry (test infrastructure; FP64).

Section 3.2: the target position is evaluated at every chirp time of the frame,
and eq. (12) moves the target at constant velocity. Reading: rigid instances
translate at constant velocity with no rotation change; each chirp sees the
geometry frozen at its start time t_n (stop-and-hop).
"""
from __future__ import annotations

import numpy as np


def world_triangles(scene, t: float):
    """World coordinates of every triangle at time t.

    Returns (tri [F,3,3] float64, inst_of [F] int, local_of [F] int) with the
    triangles of the instances concatenated in instance order. Body vertices are
    float32 and are promoted exactly to float64 before the rigid transform
    x = R x_body + p0 + v t."""
    tris, inst_of, local_of = [], [], []
    for ii, inst in enumerate(scene.instances):
        mesh = scene.meshes[inst.mesh]
        vb = mesh.verts.astype(np.float64)
        vw = vb @ np.asarray(inst.rot, np.float64).T + (inst.pos0 + inst.vel * t)
        tris.append(vw[mesh.tris.astype(np.int64)])
        inst_of.append(np.full(mesh.n_tris, ii, np.int64))
        local_of.append(np.arange(mesh.n_tris, dtype=np.int64))
    if not tris:
        return (np.zeros((0, 3, 3)), np.zeros(0, np.int64), np.zeros(0, np.int64))
    return np.concatenate(tris), np.concatenate(inst_of), np.concatenate(local_of)


def facet_frames(tri: np.ndarray):
    """Centroid c, unit normal n (CCW order), and area A of triangles [F,3,3].
    Zero-area triangles get a zero normal."""
    c = tri.mean(axis=1)
    nvec = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
    two_a = np.linalg.norm(nvec, axis=1)
    n = np.zeros_like(nvec)
    ok = two_a > 0
    n[ok] = nvec[ok] / two_a[ok, None]
    return c, n, 0.5 * two_a


def point_positions(scene, t: float) -> np.ndarray:
    """Point scatterer positions at time t (eq. (12): constant velocity)."""
    if scene.points is None or scene.points.n == 0:
        return np.zeros((0, 3))
    return scene.points.pos0 + scene.points.vel * t
