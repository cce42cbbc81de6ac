"""Single-bounce visibility by exhaustive ray-triangle testing (test infrastructure; FP64).

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

Every (segment, triangle) pair that could meet is tested with Moller-Trumbore in
FP64. Pairs are skipped only by a test that provably cannot drop a meeting pair:
  * if every triangle lies strictly below the segments' common start point S (the
    radar sits on a pole above the traffic), the central projection from S maps
    each segment to one point and each triangle to a triangle, so a triangle can
    meet the segment only if its projected bounding box (inflated for the
    ambiguity margin) contains that point;
  * otherwise, the segment's and the triangle's axis-aligned boxes must overlap.
"""
from __future__ import annotations

import numpy as np

from .geometry import facet_frames, world_triangles

T_EPS = 1e-6  # segment-parameter window [T_EPS, 1 - T_EPS]
MARGIN = 1e-4  # ambiguity margin on barycentric / segment-parameter slacks
COS_MARGIN = 1e-9  # ambiguity margin on the facing cosine


def _aabb_pairs(src, dst, tris, chunk=256):
    tlo, thi = tris.min(axis=1), tris.max(axis=1)
    for s0 in range(0, src.shape[0], chunk):
        sl = slice(s0, min(src.shape[0], s0 + chunk))
        lo_r = np.minimum(src[sl], dst[sl])
        hi_r = np.maximum(src[sl], dst[sl])
        ok = np.all((lo_r[:, None, :] <= thi[None, :, :]) &
                    (tlo[None, :, :] <= hi_r[:, None, :]), axis=-1)
        ri, ti = np.nonzero(ok)
        yield ri + s0, ti


def _projected_pairs(S, dst, tris, grid=512, chunk_pairs=4_000_000):
    """Candidate pairs via the central projection from S (all triangles below S)."""
    h = S[2] - tris[:, :, 2]  # > 0 for every vertex
    pv = (tris[:, :, :2] - S[:2]) / h[..., None]  # projected vertices [F,3,2]
    lo, hi = pv.min(axis=1), pv.max(axis=1)
    pad = 0.1 * (hi - lo).max(axis=1, keepdims=True) + 1e-12
    lo, hi = lo - pad, hi + pad
    hd = S[2] - dst[:, 2]
    pr = (dst[:, :2] - S[:2]) / hd[:, None]  # projected segment points [R,2]
    g_lo = pr.min(axis=0) - 1e-9
    g_hi = pr.max(axis=0) + 1e-9
    cell = (g_hi - g_lo) / grid
    cell = np.where(cell > 0, cell, 1.0)
    # cells covered by each triangle box, clipped to the grid of segment points
    c0 = np.floor((lo - g_lo) / cell).astype(np.int64)
    c1 = np.floor((hi - g_lo) / cell).astype(np.int64)
    keep = np.all(c1 >= 0, axis=1) & np.all(c0 < grid, axis=1)
    c0 = np.clip(c0, 0, grid - 1)
    c1 = np.clip(c1, 0, grid - 1)
    tid = np.nonzero(keep)[0]
    nx = (c1[tid, 0] - c0[tid, 0] + 1)
    ny = (c1[tid, 1] - c0[tid, 1] + 1)
    cnt = nx * ny
    rep_t = np.repeat(tid, cnt)
    k = np.arange(rep_t.size) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    rnx = np.repeat(nx, cnt)
    cx = np.repeat(c0[tid, 0], cnt) + k % rnx
    cy = np.repeat(c0[tid, 1], cnt) + k // rnx
    cid = cx * grid + cy
    order = np.argsort(cid, kind="stable")
    cid_s, tri_s = cid[order], rep_t[order]
    starts = np.searchsorted(cid_s, np.arange(grid * grid), side="left")
    ends = np.searchsorted(cid_s, np.arange(grid * grid), side="right")
    rc = np.floor((pr - g_lo) / cell).astype(np.int64)
    rc = np.clip(rc, 0, grid - 1)
    rcell = rc[:, 0] * grid + rc[:, 1]
    n_c = ends[rcell] - starts[rcell]
    r_all = np.arange(dst.shape[0])
    pos = 0
    while pos < r_all.size:
        # take rays until the pair budget is reached
        cum = np.cumsum(n_c[pos:])
        stop = pos + max(1, int(np.searchsorted(cum, chunk_pairs, side="right")))
        rr = r_all[pos:stop]
        nn = n_c[rr]
        ri = np.repeat(rr, nn)
        kk = np.arange(ri.size) - np.repeat(np.cumsum(nn) - nn, nn)
        ti = tri_s[np.repeat(starts[rcell[rr]], nn) + kk]
        yield ri, ti
        pos = stop


def segment_occluded(src: np.ndarray, dst: np.ndarray, tris: np.ndarray,
                     exclude: np.ndarray):
    """For segments src[r] -> dst[r] ([R,3]) against triangles [F,3,3], ignoring
    triangle exclude[r] for segment r: returns (occluded [R], ambiguous [R])."""
    src = np.asarray(src, np.float64)
    dst = np.asarray(dst, np.float64)
    R = src.shape[0]
    occ = np.zeros(R, bool)
    amb_near = np.zeros(R, bool)
    robust = np.zeros(R, bool)
    if R == 0 or tris.shape[0] == 0:
        return occ, amb_near
    v0 = tris[:, 0]
    e1 = tris[:, 1] - v0
    e2 = tris[:, 2] - v0
    nrm_len = np.linalg.norm(np.cross(e1, e2), axis=1)
    S = src[0]
    same_src = bool(np.all(src == S))
    if same_src and np.all(tris[:, :, 2] < S[2]) and np.all(dst[:, 2] < S[2]):
        pairs = _projected_pairs(S, dst, tris)
    else:
        pairs = _aabb_pairs(src, dst, tris)
    for ri, ti in pairs:
        sel = ti != exclude[ri]
        ri, ti = ri[sel], ti[sel]
        if ri.size == 0:
            continue
        D = dst[ri] - src[ri]
        p = np.cross(D, e2[ti])
        det = np.einsum("ij,ij->i", e1[ti], p)
        ok = (det != 0.0) & (nrm_len[ti] > 0.0)
        det_s = np.where(ok, det, 1.0)
        s = src[ri] - v0[ti]
        u = np.einsum("ij,ij->i", s, p) / det_s
        q = np.cross(s, e1[ti])
        v = np.einsum("ij,ij->i", D, q) / det_s
        t = np.einsum("ij,ij->i", e2[ti], q) / det_s
        slack = np.min(np.stack([u, v, 1.0 - u - v, t - T_EPS, (1.0 - T_EPS) - t]), axis=0)
        cosang = np.abs(det) / np.maximum(np.linalg.norm(D, axis=1) * nrm_len[ti], 1e-300)
        margin = MARGIN / np.maximum(cosang, 1e-3)
        hit = ok & (slack >= 0.0)
        near = ok & (np.abs(slack) < margin)
        np.logical_or.at(occ, ri, hit)
        np.logical_or.at(robust, ri, hit & ~near)
        np.logical_or.at(amb_near, ri, near)
    return occ, amb_near & ~robust


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
