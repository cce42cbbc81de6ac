"""Ground double bounce by the image method (test infrastructure; FP64).

Section 2.2: bidirectional analytic ray tracing joins a forward ray from the
transmitter and a backward ray from the receiver on a facet, also after reflections.
Reading for the reflections built here: the road is a flat specular plane z = z_g with
a reflection coefficient gamma (default -1: perfectly conducting, scalar field), and a
ray may bounce on it once on the transmit side and/or once on the receive side. By the
image method a bounce on the transmit side is propagation from the mirrored
transmitter (x, y, 2 z_g - z), so each of the four path types is the single-bounce
facet term of eqs. (7), (9)-(13) with mirrored elements, times gamma per bounce:

  type 0: T -> f -> R          (the single-bounce path)
  type 1: T -> ground -> f -> R           = T' -> f -> R,    factor gamma
  type 2: T -> f -> ground -> R           = T -> f -> R',    factor gamma
  type 3: T -> ground -> f -> ground -> R = T' -> f -> R',   factor gamma^2

Visibility per facet and side (transmit or receive, phase centre E):
  * direct: the facet faces E and the segment centroid -> E is clear (as for type 0);
  * image: the centroid lies strictly above the plane, the facet faces E', and both
    legs of the reflected ray, centroid -> S and S -> E with S where the segment
    centroid -> E' meets the plane, are clear. Triangles of instances that lie entirely
    in the plane (the road surface itself) do not block these legs.
Type k is lit when its transmit-side and receive-side conditions both hold. Point
scatterers are always lit on all four paths.
"""
from __future__ import annotations

import numpy as np

from .echo import synthesize
from .geometry import facet_frames, world_triangles
from .visibility import COS_MARGIN, segment_occluded

PLANE_TOL = 1e-6  # m: an instance lies in the plane when every vertex is this close


def mirror(x: np.ndarray, z_g: float) -> np.ndarray:
    """Image of points [..., 3] in the plane z = z_g."""
    y = np.array(x, dtype=np.float64, copy=True)
    y[..., 2] = 2.0 * z_g - y[..., 2]
    return y


def mirrored_array(array, z_g: float, tx: bool, rx: bool):
    """The array with its Tx and/or Rx elements replaced by their images."""
    cls = type(array)
    return cls(tx=mirror(array.tx, z_g) if tx else np.array(array.tx, np.float64),
               rx=mirror(array.rx, z_g) if rx else np.array(array.rx, np.float64))


def in_plane_instances(scene, z_g: float) -> np.ndarray:
    """[n_instances] bool: every world vertex within PLANE_TOL of the plane at t = 0 and
    no vertical velocity (so it stays there)."""
    out = []
    for inst in scene.instances:
        v = scene.meshes[inst.mesh].verts.astype(np.float64) @ np.asarray(inst.rot).T + inst.pos0
        out.append(bool(v.size) and bool(np.all(np.abs(v[:, 2] - z_g) <= PLANE_TOL))
                   and inst.vel[2] == 0.0)
    return np.array(out, bool)


def _side(tri, c, nrm, area, fsel, E, z_g, plane_tri):
    """Direct and image conditions for phase centre E: (direct, image, amb_d, amb_i)."""
    F = fsel.size
    d = E - c
    cd = np.einsum("ij,ij->i", nrm, d)
    front = (cd > 0) & (area > 0)
    amb_d = (area > 0) & (np.abs(cd) < COS_MARGIN * np.linalg.norm(d, axis=1))
    idx = np.nonzero(front)[0]
    occ, amb = segment_occluded(np.repeat(E[None], idx.size, 0), c[idx], tri, fsel[idx])
    direct = np.zeros(F, bool)
    direct[idx] = ~occ
    amb_d[idx] |= amb
    # image side
    Ei = mirror(E, z_g)
    di = Ei - c
    ci = np.einsum("ij,ij->i", nrm, di)
    above = c[:, 2] > z_g
    front_i = (ci > 0) & (area > 0) & above
    amb_i = (area > 0) & above & (np.abs(ci) < COS_MARGIN * np.linalg.norm(di, axis=1))
    idx = np.nonzero(front_i)[0]
    s = (c[idx, 2] - z_g) / (c[idx, 2] - Ei[2])
    S = c[idx] + s[:, None] * (Ei - c[idx])
    S[:, 2] = z_g
    keep = ~plane_tri  # the road surface does not block legs that end on it
    sub = tri[keep]
    remap = np.full(tri.shape[0], -1, np.int64)
    remap[np.nonzero(keep)[0]] = np.arange(int(keep.sum()))
    excl = remap[fsel[idx]]
    occ1, amb1 = segment_occluded(S, c[idx], sub, excl)
    occ2, amb2 = segment_occluded(np.repeat(E[None], idx.size, 0), S, sub,
                                  np.full(idx.size, -1, np.int64))
    image = np.zeros(F, bool)
    image[idx] = ~occ1 & ~occ2
    robust = (occ1 & ~amb1) | (occ2 & ~amb2)
    amb_i[idx] |= (amb1 | amb2) & ~robust
    return direct, image, amb_d, amb_i


def visibility_bounce(scene, array, wf, z_g: float = 0.0, chirps=None):
    """Lit masks of the four path types: (mask [4, n_chirps_sel, F], ambiguous [same])."""
    tx_c = np.asarray(array.tx, np.float64).mean(axis=0)
    rx_c = np.asarray(array.rx, np.float64).mean(axis=0)
    chirps = np.arange(wf.n_chirps) if chirps is None else np.asarray(chirps)
    flat = in_plane_instances(scene, z_g)
    masks, ambs = [], []
    for n in chirps:
        tri, inst_of, _ = world_triangles(scene, float(n) * wf.chirp_period)
        fsel = np.arange(tri.shape[0])
        c, nrm, area = facet_frames(tri)
        plane_tri = flat[inst_of] if inst_of.size else np.zeros(0, bool)
        dt, it, adt, ait = _side(tri, c, nrm, area, fsel, tx_c, z_g, plane_tri)
        dr, ir, adr, air = _side(tri, c, nrm, area, fsel, rx_c, z_g, plane_tri)
        t_ok, t_amb = (dt, it), (adt, ait)
        r_ok, r_amb = (dr, ir), (adr, air)
        m4, a4 = [], []
        for k in range(4):
            ti, ri = k & 1, k >> 1
            m4.append(t_ok[ti] & r_ok[ri])
            # an ambiguous side matters only if the other side is lit or itself ambiguous
            a4.append((t_amb[ti] & (r_ok[ri] | r_amb[ri])) | (r_amb[ri] & (t_ok[ti] | t_amb[ti])))
        masks.append(m4)
        ambs.append(a4)
    return np.array(masks).transpose(1, 0, 2), np.array(ambs).transpose(1, 0, 2)


def synthesize_bounce(scene, wf, array, z_g: float = 0.0, gamma: complex = -1.0, masks=None,
                      channels=None, samples=None):
    """Echo H[o, n, m] summed over the four path types (masks [4, N, F] from
    visibility_bounce unless given)."""
    if masks is None:
        masks, _ = visibility_bounce(scene, array, wf, z_g)
    H = 0.0
    for k in range(4):
        arr_k = mirrored_array(array, z_g, tx=bool(k & 1), rx=bool(k >> 1))
        g = gamma ** (bin(k).count("1"))
        H = H + g * synthesize(scene, wf, arr_k, mask=masks[k], channels=channels,
                               samples=samples)
    return H
