"""Pins of the oracle's visibility against analytic cases (no GPU): a convex box is
lit exactly on the faces whose outward half-space contains both phase centres; a
floating box shadows exactly the ground cells whose rays cross it (slab test)."""
import numpy as np

import oracle
import scenes
from scenes import Instance, RadarArray, Scene


def _arr():
    p = scenes.RADAR_POS
    return RadarArray(tx=(p + np.array([[-0.02, 0, 0.0]])), rx=(p + np.array([[0.01, 0, 0], [0.03, 0, 0.0]])))


def test_convex_box_faces():
    wf = scenes.paper_waveform(16, 2)
    lo, hi = np.array([-1.0, -0.7, 0.2]), np.array([1.4, 0.9, 1.9])
    m = scenes.box_mesh(lo, hi, (5, 3, 4))
    pos0 = np.array([3.0, 14.0, 0.0])
    vel = np.array([0.0, -8.0, 0.0])
    sc = Scene([m], [Instance(0, np.eye(3), pos0, vel)])
    arr = _arr()
    mask, amb = oracle.visibility(sc, arr, wf)
    assert not amb.any()
    T, R = arr.tx.mean(0), arr.rx.mean(0)
    cen = m.verts.astype(np.float64)[m.tris].mean(axis=1)
    for n in range(wf.n_chirps):
        off = pos0 + vel * n * wf.chirp_period
        blo, bhi = lo + off, hi + off
        expect = np.zeros(m.n_tris, bool)
        for f in range(m.n_tris):
            cw = cen[f] + off
            # which face plane the centroid lies on
            for d in range(3):
                for side, plane in ((0, blo[d]), (1, bhi[d])):
                    if abs(cw[d] - plane) < 1e-6:
                        out = (lambda p: p[d] < plane) if side == 0 else (lambda p: p[d] > plane)
                        expect[f] = out(T) and out(R)
        assert np.array_equal(mask[n], expect)


def _segment_hits_box(p0, p1, lo, hi):
    """Slab test: does the closed segment p0 -> p1 meet the box [lo, hi]?"""
    d = p1 - p0
    t0, t1 = 0.0, 1.0
    for k in range(3):
        if abs(d[k]) < 1e-15:
            if p0[k] < lo[k] or p0[k] > hi[k]:
                return False
            continue
        a, b = (lo[k] - p0[k]) / d[k], (hi[k] - p0[k]) / d[k]
        t0, t1 = max(t0, min(a, b)), min(t1, max(a, b))
        if t0 > t1:
            return False
    return True


def test_box_shadow_on_ground():
    wf = scenes.paper_waveform(16, 1)
    ground = scenes.ground_grid(-4.0, 4.0, 6.0, 20.0, 0.5)
    lo, hi = np.array([-1.0, -1.0, 1.0]), np.array([1.0, 1.0, 2.5])
    box = scenes.box_mesh(lo, hi, (2, 2, 2))
    bpos = np.array([0.5, 10.0, 0.0])
    sc = Scene([ground, box], [Instance(0, np.eye(3), np.zeros(3), np.zeros(3)),
                               Instance(1, np.eye(3), bpos, np.zeros(3))])
    arr = _arr()
    mask, amb = oracle.visibility(sc, arr, wf)
    T, R = arr.tx.mean(0), arr.rx.mean(0)
    g = ground.verts.astype(np.float64)[ground.tris].mean(axis=1)
    blo, bhi = lo + bpos, hi + bpos
    expect = np.array([not (_segment_hits_box(c, T, blo, bhi) or _segment_hits_box(c, R, blo, bhi))
                       for c in g])
    got = mask[0, :ground.n_tris]
    a = amb[0, :ground.n_tris]
    assert (~expect).sum() > 10  # there is a shadow
    assert np.array_equal(got[~a], expect[~a])
    assert a.sum() <= 2


def test_hidden_box_is_dark():
    wf = scenes.paper_waveform(16, 1)
    big = scenes.box_mesh((-3, -1, 0), (3, 1, 4), (6, 2, 4))
    small = scenes.box_mesh((-0.5, -0.5, 0), (0.5, 0.5, 0.8), (2, 2, 2))
    sc = Scene([big, small], [Instance(0, np.eye(3), np.array([0.0, 12.0, 0.0]), np.zeros(3)),
                              Instance(1, np.eye(3), np.array([0.0, 14.0, 0.0]), np.zeros(3))])
    mask, amb = oracle.visibility(sc, _arr(), wf)
    assert not mask[0, big.n_tris:].any()
    assert mask[0, :big.n_tris].any()


def test_projection_prefilter_matches_box_prefilter():
    """The two candidate searches are exact prefilters: they give identical decisions."""
    import importlib
    V = importlib.import_module("oracle.visibility")
    sc = scenes.intersection_scene(21, n_vehicles=3, per_vehicle=500, with_ground=True,
                                   ground_cell=2.0)
    tri, _, _ = oracle.world_triangles(sc, 0.0)
    c, n, _ = oracle.facet_frames(tri)
    S = scenes.RADAR_POS + np.array([0.01, 0.0, 0.0])
    idx = np.nonzero(np.einsum("ij,ij->i", n, S - c) > 0)[0]
    src = np.repeat(S[None], idx.size, 0)
    occ_p, amb_p = V.segment_occluded(src, c[idx], tri, idx)
    # force the box path by moving one triangle above the source
    tri2 = tri.copy()
    far = tri2.shape[0] - 1
    tri2[far] += np.array([500.0, 500.0, 100.0])
    occ_b, amb_b = V.segment_occluded(src, c[idx], tri2, idx)
    occ_p2, amb_p2 = V.segment_occluded(src, c[idx], np.delete(tri, far, 0), np.where(idx > far, idx - 1, idx))
    assert occ_p.sum() > 10
    assert np.array_equal(occ_b, occ_p2) and np.array_equal(amb_b, amb_p2)
    assert np.array_equal(occ_b, occ_p) and np.array_equal(amb_b, amb_p)
