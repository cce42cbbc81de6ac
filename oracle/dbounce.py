"""Facet-to-facet double bounce (test infrastructure; FP64).

Section 2.2 (BART): a forward ray from the transmitter is followed as the facets reflect
it, a backward ray is traced from the receiver, and a scattering path is formed where
the two meet on one facet. Reading built here for two bounces; every step is a plain
geometric rule.

Rays are launched from both ends, for chirp n with the geometry at t_n: k = 0 follows a
ray from the transmitter phase centre T (E = T, O = R), k = 1 one from the receiver phase
centre R (E = R, O = T). A is the facet the launched ray reflects off and B the facet where
it meets the backward ray from O.

  1. A is a reflector lit from E: nonzero area, faces E (strict n_A . (E - c_A) > 0) and
     the segment c_A -> E is clear (the single-bounce rules, A excluded).
  2. The forward ray leaves c_A in the specular direction r = d - 2 (d . n_A) n_A with
     d = (c_A - E) / |c_A - E| (law of reflection); its first hit (ray parameter above
     T_MIN metres, A excluded, closed barycentric test) is facet B at the point h.
  3. The backward ray meets it on B: B has nonzero area, faces the image E' of E in A's
     plane (n_B . (E' - h) > 0) and faces O (n_B . (O - h) > 0), and the segment h -> O
     is clear (B excluded).
  4. The tube reflected by A lands on B's plane as the footprint triangle F, the central
     projection from E' of A's vertices onto that plane (x = E' + s (v - E') with every
     s > S_MIN: the plane is met ahead of the image source, at or near A and beyond),
     its vertices ordered so that its normal is n_B. The connection is kept when F is not much larger than the scene's largest
     facet: every vertex of F within FOOTPRINT_LIMIT r_lim of F's centroid, r_lim the
     largest vertex-to-centroid distance of any triangle of the scene's meshes (a larger
     footprint means a grazing tube, outside what a facet-sized tube describes).
  5. The connection's echo is gamma times the single-bounce facet term of F (eqs. (7),
     (9)-(13)) with the elements on E's side replaced by their images in A's plane: by
     the image method the wave reflected by A is that of the mirrored elements, and the
     distance from an image element to a point equals the length of the path folded at
     A's plane.
  6. Each physical path T -> X -> Y -> R is found from both ends (k = 0 with A = X, B =
     Y; k = 1 with A = Y, B = X), evaluated once with the tube from T and once with the
     tube from R. The echo takes the mean of the two: gamma / 2 times every connection's
     term, so that each path counts once and the sum is reciprocal (swapping the Tx and
     Rx elements swaps k = 0 and k = 1).

The footprint is not clipped to B (the tube is taken to land on B's plane whole). Point
scatterers take no double bounce. Only stop-and-hop geometry.
"""
from __future__ import annotations

import numpy as np

from .echo import facet_terms
from .geometry import facet_frames, world_triangles
from .visibility import COS_MARGIN, segment_occluded

T_MIN = 1e-6       # m: smallest ray parameter of a reflected ray's hit
HIT_MARGIN = 1e-6  # barycentric slack (and relative distance gap) below which a hit is ambiguous
S_MIN = 0.5        # footprint projection parameters must exceed this
FOOTPRINT_LIMIT = 1.5  # footprint radius limit in units of the scene's largest facet radius


def mirror_points(x: np.ndarray, p: np.ndarray, n: np.ndarray) -> np.ndarray:
    """Images of points x [..., 3] in the plane through p with unit normal n."""
    x = np.asarray(x, np.float64)
    return x - 2.0 * np.einsum("...k,k->...", x - p, n)[..., None] * n


def scene_r_lim(scene) -> float:
    """Largest vertex-to-centroid distance of any triangle of the scene's meshes."""
    r = 0.0
    for inst in scene.instances:
        m = scene.meshes[inst.mesh]
        tri = m.verts.astype(np.float64)[m.tris.astype(np.int64)]
        if tri.shape[0]:
            c = tri.mean(axis=1)
            r = max(r, float(np.linalg.norm(tri - c[:, None, :], axis=2).max()))
    return r


def closest_hits(orig: np.ndarray, dirs: np.ndarray, tris: np.ndarray, exclude: np.ndarray,
                 chunk: int = 64):
    """First triangle hit by each ray orig[r] + t dirs[r] (dirs unit, t > T_MIN), triangle
    exclude[r] ignored, by Moller-Trumbore against every triangle (closed test). Returns
    (index [R] or -1, t [R], ambiguous [R]): ambiguous when the hit lies within HIT_MARGIN
    of a triangle edge or another triangle is hit within HIT_MARGIN (1 + t) of it."""
    R = orig.shape[0]
    idx = np.full(R, -1, np.int64)
    tbest = np.full(R, np.inf)
    amb = np.zeros(R, bool)
    if R == 0 or tris.shape[0] == 0:
        return idx, tbest, amb
    v0 = tris[:, 0]
    e1 = tris[:, 1] - v0
    e2 = tris[:, 2] - v0
    area_ok = np.linalg.norm(np.cross(e1, e2), axis=1) > 0.0
    for r0 in range(0, R, chunk):
        sl = slice(r0, min(R, r0 + chunk))
        D = dirs[sl][:, None, :]                      # [r, 1, 3]
        p = np.cross(D, e2[None])                     # [r, F, 3]
        det = np.einsum("fk,rfk->rf", e1, p)
        ok = (det != 0.0) & area_ok[None]
        det_s = np.where(ok, det, 1.0)
        s = orig[sl][:, None, :] - v0[None]
        u = np.einsum("rfk,rfk->rf", s, p) / det_s
        q = np.cross(s, e1[None])
        v = np.einsum("rk,rfk->rf", dirs[sl], q) / det_s
        t = np.einsum("fk,rfk->rf", e2, q) / det_s
        slack = np.minimum(np.minimum(u, v), 1.0 - u - v)
        hit = ok & (slack >= 0.0) & (t > T_MIN)
        rows = np.arange(sl.stop - sl.start)
        hit[rows, exclude[sl]] = False
        tt = np.where(hit, t, np.inf)
        j = np.argmin(tt, axis=1)
        tj = tt[rows, j]
        found = np.isfinite(tj)
        idx[sl] = np.where(found, j, -1)
        tbest[sl] = tj
        # near-edge hits, near-ties with another triangle, and near-misses that would
        # have come first
        edge = found & (slack[rows, j] < HIT_MARGIN)
        tt2 = tt.copy()
        tt2[rows, j] = np.inf
        with np.errstate(invalid="ignore"):  # inf - inf where nothing is hit
            tie = found & (tt2.min(axis=1) - tj < HIT_MARGIN * (1.0 + tj))
        near = ok & (slack > -HIT_MARGIN) & (slack < 0.0) & (t > T_MIN)
        near[rows, exclude[sl]] = False
        tn = np.where(near, t, np.inf).min(axis=1)
        miss_first = tn < np.where(found, tj, np.inf) + HIT_MARGIN * (1.0 + np.minimum(tn, 1e9))
        amb[sl] = edge | tie | miss_first
    return idx, tbest, amb


def _plane_normal(tri):
    nv = np.cross(tri[..., 1, :] - tri[..., 0, :], tri[..., 2, :] - tri[..., 0, :])
    return nv


def footprints(A_tri: np.ndarray, E_img: np.ndarray, B_c: np.ndarray, B_n: np.ndarray):
    """Central projections from E_img [P,3] of the triangles A_tri [P,3,3] onto the planes
    through B_c [P,3] with unit normals B_n [P,3], ordered so that their normal is B_n.
    Returns (F [P,3,3], ok [P], s_min [P])."""
    d = A_tri - E_img[:, None, :]                           # [P, 3, 3]
    num = np.einsum("pk,pk->p", B_c - E_img, B_n)            # [P]
    den = np.einsum("pvk,pk->pv", d, B_n)                    # [P, 3]
    with np.errstate(divide="ignore", invalid="ignore"):
        s = num[:, None] / den
    ok = np.all(np.isfinite(s) & (s > S_MIN), axis=1)
    s = np.where(np.isfinite(s), s, 0.0)
    F = E_img[:, None, :] + s[..., None] * d
    flip = np.einsum("pk,pk->p", _plane_normal(F), B_n) < 0.0
    F[flip] = F[flip][:, [0, 2, 1], :]
    return F, ok, s.min(axis=1)


def double_bounce_pairs(scene, array, wf, chirps=None, facets=None):
    """The connections (A, B) launched from both ends, per chirp: a list (one entry per
    chirp) of dicts k -> {"A": [P], "B": [P], "F": [P,3,3], "plane_p": [P,3],
    "plane_n": [P,3], "amb": [P]} over the kept pairs, plus "amb_rejected": the number of
    rejected candidates A whose rejection hung on an ambiguous decision, and "amb_facets":
    every candidate A (kept or rejected) with an ambiguous decision. facets: launch only
    from these facets A (a sample; every facet can still be hit)."""
    tx_c = np.asarray(array.tx, np.float64).mean(axis=0)
    rx_c = np.asarray(array.rx, np.float64).mean(axis=0)
    chirps = np.arange(wf.n_chirps) if chirps is None else np.asarray(chirps)
    r_lim = scene_r_lim(scene)
    out = []
    for n in chirps:
        tri, _, _ = world_triangles(scene, float(n) * wf.chirp_period)
        c, nrm, area = facet_frames(tri)
        per = {}
        for k, (E, O) in enumerate(((tx_c, rx_c), (rx_c, tx_c))):
            # A stage's ambiguity counts for the rows still in play (kept so far, or
            # rejected only by an ambiguous decision); a row rejected by a clear decision
            # stays clear.
            def stage(ok, amb_s):
                nonlocal keep, amb
                live = keep | amb
                amb = amb | (amb_s & live)
                keep = keep & ok
            # 1. reflectors lit from E (candidates: nonzero area, facing E or nearly)
            dE = E - c
            fe = np.einsum("ij,ij->i", nrm, dE)
            near = np.abs(fe) < COS_MARGIN * np.linalg.norm(dE, axis=1)
            ok_a = (area > 0) & ((fe > 0) | near)
            if facets is not None:
                sub = np.zeros_like(ok_a)
                sub[np.asarray(facets)] = True
                ok_a &= sub
            cand = np.nonzero(ok_a)[0]
            keep = np.ones(cand.size, bool)
            amb = np.zeros(cand.size, bool)
            stage(fe[cand] > 0, near[cand])
            occ, amb_o = segment_occluded(np.repeat(E[None], cand.size, 0), c[cand], tri, cand)
            stage(~occ, amb_o)
            # 2. specular ray from the centroid and its first hit
            d = c[cand] - E
            d /= np.linalg.norm(d, axis=1, keepdims=True)
            nA = nrm[cand]
            r = d - 2.0 * np.einsum("ij,ij->i", d, nA)[:, None] * nA
            B, t, amb_h = closest_hits(c[cand], r, tri, cand)
            stage(B >= 0, amb_h)
            hit = B >= 0
            Bs = np.where(hit, B, 0)
            h = c[cand] + np.where(hit, t, 0.0)[:, None] * r
            # 3. B faces the image of E and O; h -> O clear (rows with a hit)
            E_img = np.array([mirror_points(E, c[a], nrm[a]) for a in cand]).reshape(-1, 3)
            nB = nrm[Bs]
            f1 = np.einsum("ij,ij->i", nB, E_img - h)
            f2 = np.einsum("ij,ij->i", nB, O - h)
            near_f = (np.abs(f1) < COS_MARGIN * np.linalg.norm(E_img - h, axis=1)) | \
                (np.abs(f2) < COS_MARGIN * np.linalg.norm(O - h, axis=1))
            stage((area[Bs] > 0) & (f1 > 0) & (f2 > 0), near_f & hit)
            occ2, amb_o2 = segment_occluded(h, np.repeat(O[None], cand.size, 0), tri, Bs)
            stage(~occ2, amb_o2 & hit)
            # 4. footprint ahead of the image source, not much larger than the largest facet
            Ft, ok_s, s_min = footprints(tri[cand], E_img, c[Bs], nB)
            cF = Ft.mean(axis=1)
            rF = np.linalg.norm(Ft - cF[:, None, :], axis=2).max(axis=1)
            lim = FOOTPRINT_LIMIT * r_lim
            stage(ok_s & (rF <= lim),
                  hit & ((np.abs(rF - lim) <= 1e-9 * max(lim, 1e-300)) |
                         (np.abs(s_min - S_MIN) <= 1e-9)))
            sel = np.nonzero(keep)[0]
            per[k] = {"A": cand[sel], "B": B[sel], "F": Ft[sel], "plane_p": c[cand[sel]],
                      "plane_n": nrm[cand[sel]], "amb": amb[sel],
                      "amb_rejected": int(np.count_nonzero(amb & ~keep)),
                      "amb_facets": cand[amb]}
        out.append(per)
    return out


def connection_table(pairs, n_facets: int) -> np.ndarray:
    """[2, n_chirps, F] int32: the facet B each launched ray connects to, or -1."""
    t = np.full((2, len(pairs), n_facets), -1, np.int32)
    for ni, per in enumerate(pairs):
        for k in (0, 1):
            t[k, ni, per[k]["A"]] = per[k]["B"]
    return t


def pairs_for_table(scene, array, wf, table: np.ndarray, chirps=None):
    """The connections of a given table ([2, n_chirps, F] from connection_table: launching
    end k, chirp, facet A -> facet B or -1) with their geometry taken from the scene as it
    is (steps 4 and 5 without the decisions of steps 1-4): for each kept (A, B) the image
    E' of the launching phase centre in A's plane and the footprint of A's vertices
    projected from E' onto B's plane, ordered to B's normal. The same dicts as
    double_bounce_pairs (without the ambiguity fields), for synthesize_double; with the
    scene perturbed and the table held, the echo is a smooth function of the vertices."""
    tx_c = np.asarray(array.tx, np.float64).mean(axis=0)
    rx_c = np.asarray(array.rx, np.float64).mean(axis=0)
    chirps = np.arange(wf.n_chirps) if chirps is None else np.asarray(chirps)
    out = []
    for ni, n in enumerate(chirps):
        tri, _, _ = world_triangles(scene, float(n) * wf.chirp_period)
        c, nrm, _ = facet_frames(tri)
        per = {}
        for k, E in enumerate((tx_c, rx_c)):
            A = np.nonzero(table[k, ni] >= 0)[0]
            B = table[k, ni, A].astype(np.int64)
            E_img = np.array([mirror_points(E, c[a], nrm[a]) for a in A]).reshape(-1, 3)
            Ft, _, _ = footprints(tri[A], E_img, c[B], nrm[B])
            per[k] = {"A": A, "B": B, "F": Ft, "plane_p": c[A], "plane_n": nrm[A]}
        out.append(per)
    return out


def synthesize_double(scene, wf, array, gamma: complex = -1.0, pairs=None, chirps=None,
                      channels=None, samples=None):
    """Double-bounce echo H[o, n, m]: gamma / 2 times the footprint terms of the
    connections launched from both ends (pairs from double_bounce_pairs unless given, for
    the same chirps)."""
    P, Q = array.tx.shape[0], array.rx.shape[0]
    chirps = np.arange(wf.n_chirps) if chirps is None else np.asarray(chirps)
    channels = np.arange(P * Q) if channels is None else np.asarray(channels)
    samples = np.arange(wf.n_samples) if samples is None else np.asarray(samples)
    pq = [(int(o) // Q, int(o) % Q) for o in channels]
    freqs = wf.f0 + (wf.slope / wf.fs) * samples.astype(np.float64)
    if pairs is None:
        pairs = double_bounce_pairs(scene, array, wf, chirps=chirps)
    cls = type(array)
    tx = np.asarray(array.tx, np.float64)
    rx = np.asarray(array.rx, np.float64)
    H = np.zeros((channels.size, chirps.size, samples.size), np.complex128)
    for ni in range(chirps.size):
        for k in (0, 1):
            pk = pairs[ni][k]
            for j in range(pk["A"].size):
                p0, nA = pk["plane_p"][j], pk["plane_n"][j]
                arr = (cls(tx=mirror_points(tx, p0, nA), rx=rx) if k == 0 else
                       cls(tx=tx, rx=mirror_points(rx, p0, nA)))
                H[:, ni, :] += (0.5 * gamma) * facet_terms(pk["F"][j][None], wf, arr, freqs, pq)
    return H
