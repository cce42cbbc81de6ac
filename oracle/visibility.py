"""Single-bounce visibility by brute force (test infrastructure; FP64).

Section 2.2: BART joins a forward ray from the transmitter and a backward ray from
the receiver where they meet on the same facet. Reading for the single-bounce
path: facet f is lit at chirp n when
  * it faces both phase centres (strict n . (T - c) > 0 and n . (R - c) > 0), and
  * neither segment T -> c nor R -> c is blocked by any other triangle of the scene
    (any facing; closed barycentric test; segment parameter in [T_EPS, 1 - T_EPS]).
T and R are the means of the Tx and Rx element positions; rays go to the centroid
only (no partial lighting). Zero-area triangles are never lit and never block.

Each decision also carries an `ambiguous` flag: the facing cosine or some ray-
triangle test lies within a small margin of its threshold, so a correct
implementation in lower precision may decide either way.
"""
from __future__ import annotations

import numpy as np

from .geometry import facet_frames, world_triangles

T_EPS = 1e-6  # segment-parameter window [T_EPS, 1 - T_EPS]
MARGIN = 1e-4  # ambiguity margin on barycentric / segment-parameter slacks
COS_MARGIN = 1e-9  # ambiguity margin on the facing cosine


def _aabb_overlap(lo_r, hi_r, lo_t, hi_t):
    return np.all((lo_r[:, None, :] <= hi_t[None, :, :]) &
                  (lo_t[None, :, :] <= hi_r[:, None, :]), axis=-1)


def segment_occluded(src: np.ndarray, dst: np.ndarray, tris: np.ndarray,
                     exclude: np.ndarray, chunk: int = 256):
    """For segments src[r] -> dst[r] ([R,3]) against triangles [F,3,3], ignoring
    triangle exclude[r] for segment r: returns (occluded [R], ambiguous [R]).

    Moller-Trumbore in FP64. A conservative bounding-box overlap test picks the
    candidate pairs first (a segment that meets a triangle always overlaps its box)."""
    src = np.asarray(src, np.float64)
    dst = np.asarray(dst, np.float64)
    R = src.shape[0]
    occ = np.zeros(R, bool)
    amb = np.zeros(R, bool)
    if R == 0 or tris.shape[0] == 0:
        return occ, amb
    tlo, thi = tris.min(axis=1), tris.max(axis=1)
    v0 = tris[:, 0]
    e1 = tris[:, 1] - v0
    e2 = tris[:, 2] - v0
    nrm = np.cross(e1, e2)
    nrm_len = np.linalg.norm(nrm, axis=1)
    for s0 in range(0, R, chunk):
        sl = slice(s0, min(R, s0 + chunk))
        S, Dst = src[sl], dst[sl]
        lo_r = np.minimum(S, Dst)
        hi_r = np.maximum(S, Dst)
        cand = _aabb_overlap(lo_r, hi_r, tlo, thi)
        cand[np.arange(cand.shape[0]), exclude[sl]] = False
        ri, ti = np.nonzero(cand)
        if ri.size == 0:
            continue
        D = Dst[ri] - S[ri]
        p = np.cross(D, e2[ti])
        det = np.einsum("ij,ij->i", e1[ti], p)
        ok = (det != 0.0) & (nrm_len[ti] > 0.0)
        det_s = np.where(ok, det, 1.0)
        s = S[ri] - v0[ti]
        u = np.einsum("ij,ij->i", s, p) / det_s
        q = np.cross(s, e1[ti])
        v = np.einsum("ij,ij->i", D, q) / det_s
        t = np.einsum("ij,ij->i", e2[ti], q) / det_s
        slack = np.min(np.stack([u, v, 1.0 - u - v, t - T_EPS, (1.0 - T_EPS) - t]), axis=0)
        cosang = np.abs(det) / np.maximum(np.linalg.norm(D, axis=1) * nrm_len[ti], 1e-300)
        margin = MARGIN / np.maximum(cosang, 1e-3)
        hit = ok & (slack >= 0.0)
        near = ok & (np.abs(slack) < margin)
        robust_hit = hit & ~near
        local = np.zeros(sl.stop - sl.start, bool)
        np.logical_or.at(local, ri, robust_hit)
        local_near = np.zeros(sl.stop - sl.start, bool)
        np.logical_or.at(local_near, ri, near)
        local_any = np.zeros(sl.stop - sl.start, bool)
        np.logical_or.at(local_any, ri, hit)
        occ[sl] = local_any
        amb[sl] = local_near & ~local
    return occ, amb


def visibility(scene, array, wf, chirps=None, facets=None):
    """Lit-facet mask (Section 2.2 reading above) for the given chirps and facets.

    Returns (mask [n_chirps_sel, n_facets_sel] bool, ambiguous [same] bool) with
    facets indexed in the scene's global order (instances concatenated)."""
    tx_c = np.asarray(array.tx, np.float64).mean(axis=0)
    rx_c = np.asarray(array.rx, np.float64).mean(axis=0)
    chirps = np.arange(wf.n_chirps) if chirps is None else np.asarray(chirps)
    masks, ambs = [], []
    for n in chirps:
        tri, _, _ = world_triangles(scene, float(n) * wf.chirp_period)
        F = tri.shape[0]
        fsel = np.arange(F) if facets is None else np.asarray(facets, np.int64)
        c, nrm, area = facet_frames(tri[fsel])
        dt = tx_c - c
        dr = rx_c - c
        ct = np.einsum("ij,ij->i", nrm, dt)
        cr = np.einsum("ij,ij->i", nrm, dr)
        front = (ct > 0) & (cr > 0) & (area > 0)
        amb_front = (area > 0) & (
            (np.abs(ct) < COS_MARGIN * np.linalg.norm(dt, axis=1)) |
            (np.abs(cr) < COS_MARGIN * np.linalg.norm(dr, axis=1)))
        idx = np.nonzero(front)[0]
        occ_t, amb_t = segment_occluded(np.repeat(tx_c[None], idx.size, 0), c[idx], tri,
                                        fsel[idx])
        occ_r, amb_r = segment_occluded(np.repeat(rx_c[None], idx.size, 0), c[idx], tri,
                                        fsel[idx])
        lit = np.zeros(fsel.size, bool)
        lit[idx] = ~occ_t & ~occ_r
        amb = amb_front.copy()
        # a robustly blocked ray decides the facet whatever the other ray does
        robust_blocked = (occ_t & ~amb_t) | (occ_r & ~amb_r)
        amb[idx] |= (amb_t | amb_r) & ~robust_blocked
        masks.append(lit)
        ambs.append(amb)
    return np.array(masks), np.array(ambs)
