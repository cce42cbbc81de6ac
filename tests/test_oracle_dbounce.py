"""Pins of the facet-to-facet double bounce oracle (oracle/dbounce.py; Section 2.2, rays
joined on a facet after a reflection; eqs. (7), (9)-(13) for the facet term).

* Closed form: a right-angle dihedral of a x b plates seen along its bisector returns
  sigma = 8 pi a^2 b^2 / lambda^2, the echo of a flat plate of area sqrt(2) a b facing the
  radar (far field, any facet grid).
* gamma enters once per path.
* Reciprocity: swapping the Tx and Rx elements leaves the double-bounce echo unchanged.
* Geometry: every footprint lies in B's plane, faces like B, and its centroid's folded
  path through A's plane has the length of the straight path from the image source.
* The first-hit search against hand-made triangles.
* Planted mistakes (sign of the reflection, images in a tilted plane, both ends counted
  in full) each fail the closed form.
* pairs_for_table (geometry of a held connection table) reproduces the connection search's
  footprints, planes and echo on the scene the table came from, and follows a moved vertex.
"""
import numpy as np
import pytest

import oracle
import scenes
from oracle import dbounce
from scenes import RadarArray, Waveform


def _far_wave(n_samples=8):
    return Waveform(f0=77e9, slope=1e6, fs=5.12e6, chirp_period=60e-6, n_samples=n_samples,
                    n_chirps=1)


def _mono_array():
    p = scenes.RADAR_POS[None, :].astype(np.float64)
    return RadarArray(tx=p.copy(), rx=p.copy())


def _dihedral_ratio(n_a, n_b, D=1e6, gamma=-1.0):
    a, b = 0.3, 0.2
    wf, arr = _far_wave(), _mono_array()
    H2 = dbounce.synthesize_double(scenes.dihedral_scene(a, b, D, n_a, n_b), wf, arr,
                                   gamma=gamma)[0, 0]
    Hp = oracle.synthesize(scenes.plate_scene(a, np.sqrt(2.0) * b, 1, 1, D), wf, arr)[0, 0]
    return np.abs(H2) / np.abs(Hp)


@pytest.mark.parametrize("n_a,n_b", [(1, 1), (3, 2)])
def test_dihedral_closed_form(n_a, n_b):
    """|H_dihedral| = |H_plate(sqrt(2) a b)| over the band (sigma = 8 pi a^2 b^2 / lambda^2)."""
    r = _dihedral_ratio(n_a, n_b)
    assert np.allclose(r, 1.0, rtol=1e-5, atol=0.0)


def test_gamma_enters_once():
    wf, arr = _far_wave(), _mono_array()
    sc = scenes.dihedral_scene(0.3, 0.2, 50.0, 2, 2)
    pr = dbounce.double_bounce_pairs(sc, arr, wf)
    H1 = dbounce.synthesize_double(sc, wf, arr, gamma=1.0, pairs=pr)
    Hg = dbounce.synthesize_double(sc, wf, arr, gamma=0.5j, pairs=pr)
    assert np.max(np.abs(Hg - 0.5j * H1)) <= 1e-14 * np.max(np.abs(H1))
    assert np.max(np.abs(H1)) > 0.0


def _vehicle_case():
    cfg = scenes.small_single(n_samples=32, n_chirps=2, n_tris=1500)
    arr = RadarArray(tx=np.array(cfg.array.tx[:2]), rx=np.array(cfg.array.rx[:3]))
    return cfg.scenes[0], cfg.waveform, arr


def test_reciprocity_swap_tx_rx():
    sc, wf, arr = _vehicle_case()
    sw = RadarArray(tx=arr.rx.copy(), rx=arr.tx.copy())
    H = dbounce.synthesize_double(sc, wf, arr)
    Hs = dbounce.synthesize_double(sc, wf, sw)
    P, Q = arr.tx.shape[0], arr.rx.shape[0]
    # channel (p, q) of one is (q, p) of the other
    Hs = Hs.reshape(Q, P, *Hs.shape[1:]).transpose(1, 0, 2, 3).reshape(H.shape)
    n = sum(int(p[k]["A"].size) for p in dbounce.double_bounce_pairs(sc, arr, wf) for k in (0, 1))
    assert n > 0
    assert np.max(np.abs(H - Hs)) <= 1e-12 * np.max(np.abs(H))


def test_footprint_geometry():
    sc, wf, arr = _vehicle_case()
    pairs = dbounce.double_bounce_pairs(sc, arr, wf)
    tx_c, rx_c = arr.tx.mean(axis=0), arr.rx.mean(axis=0)
    checked = 0
    for ni, per in enumerate(pairs):
        tri, _, _ = oracle.world_triangles(sc, ni * wf.chirp_period)
        c, nrm, _ = oracle.facet_frames(tri)
        for k, E in ((0, tx_c), (1, rx_c)):
            pk = per[k]
            for j in range(pk["A"].size):
                A, B, F = pk["A"][j], pk["B"][j], pk["F"][j]
                # in B's plane, facing like B
                assert np.max(np.abs((F - c[B]) @ nrm[B])) <= 1e-9
                nF = np.cross(F[1] - F[0], F[2] - F[0])
                assert nF @ nrm[B] > 0.0
                # folded path of the centroid: |E' - cF| = |E - p| + |p - cF|
                Ei = E - 2.0 * ((E - c[A]) @ nrm[A]) * nrm[A]
                cF = F.mean(axis=0)
                s = ((c[A] - Ei) @ nrm[A]) / ((cF - Ei) @ nrm[A])
                p = Ei + s * (cF - Ei)
                assert abs(np.linalg.norm(cF - Ei) -
                           (np.linalg.norm(E - p) + np.linalg.norm(cF - p))) <= 1e-9
                checked += 1
    assert checked > 10


def test_closest_hits_by_hand():
    t0 = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    tris = np.stack([t0, t0 + [0, 0, 0.5], t0 + [0, 0, -2.0], t0 + [5.0, 0, 0.25]])
    o = np.array([[0.2, 0.2, 1.0], [0.2, 0.2, 1.0], [0.2, 0.2, 0.25], [3.0, 3.0, 1.0]])
    d = np.array([[0.0, 0.0, -1.0]] * 4)
    idx, t, amb = dbounce.closest_hits(o, d, tris, np.array([-1, 1, -1, -1]))
    assert idx.tolist() == [1, 0, 0, -1]
    assert np.allclose(t[:3], [0.5, 1.0, 0.25])
    assert not amb.any()


def test_planted_mistakes_fail_the_closed_form(monkeypatch):
    good = _dihedral_ratio(2, 2)
    assert np.allclose(good, 1.0, rtol=1e-5)
    # 1. reflection with the wrong sign: no ray reaches the other plate
    real_hits = dbounce.closest_hits
    monkeypatch.setattr(dbounce, "closest_hits",
                        lambda o, d, t, e: real_hits(o, -d, t, e))
    assert not np.allclose(_dihedral_ratio(2, 2), 1.0, rtol=1e-2)
    monkeypatch.undo()
    # 2. images in a plane tilted from A's by 0.05 rad: the footprint term is no longer
    #    evaluated in its specular direction
    real_mirror = dbounce.mirror_points

    def tilted(x, p, n):
        m = np.asarray(n, np.float64) + np.array([0.05, 0.0, 0.0])
        return real_mirror(x, p, m / np.linalg.norm(m))
    monkeypatch.setattr(dbounce, "mirror_points", tilted)
    assert not np.allclose(_dihedral_ratio(2, 2), 1.0, rtol=1e-2)
    monkeypatch.undo()
    # 3. both ends counted in full (no mean): twice the amplitude
    wf, arr = _far_wave(), _mono_array()
    sc = scenes.dihedral_scene(0.3, 0.2, 1e6, 2, 2)
    H2 = 2.0 * dbounce.synthesize_double(sc, wf, arr)[0, 0]
    Hp = oracle.synthesize(scenes.plate_scene(0.3, np.sqrt(2.0) * 0.2, 1, 1, 1e6), wf, arr)[0, 0]
    assert not np.allclose(np.abs(H2) / np.abs(Hp), 1.0, rtol=1e-2)


def test_pairs_for_table_reproduces_the_search():
    sc, wf, arr = _vehicle_case()
    pairs = dbounce.double_bounce_pairs(sc, arr, wf)
    F = sum(m.tris.shape[0] for m in [sc.meshes[i.mesh] for i in sc.instances])
    table = dbounce.connection_table(pairs, F)
    held = dbounce.pairs_for_table(sc, arr, wf, table)
    n_conn = 0
    for ni in range(wf.n_chirps):
        for k in (0, 1):
            a, b = pairs[ni][k], held[ni][k]
            order = np.argsort(a["A"])
            assert np.array_equal(a["A"][order], b["A"])
            assert np.array_equal(a["B"][order], b["B"])
            assert np.array_equal(a["F"][order], b["F"])
            assert np.array_equal(a["plane_n"][order], b["plane_n"])
            n_conn += b["A"].size
    assert n_conn > 10
    H = dbounce.synthesize_double(sc, wf, arr, pairs=pairs)
    Hh = dbounce.synthesize_double(sc, wf, arr, pairs=held)
    assert np.max(np.abs(H - Hh)) <= 1e-12 * np.max(np.abs(H))
    # a vertex of a connected facet B moved off B's plane (along its normal, in the body
    # frame) moves the footprint with it
    ni, k = 0, 0
    B0 = held[ni][k]["B"][0]
    tri, inst_of, local_of = oracle.world_triangles(sc, 0.0)
    inst = sc.instances[inst_of[B0]]
    mesh = sc.meshes[inst.mesh]
    v = int(mesh.tris[local_of[B0], 0])
    _, nrm, _ = oracle.facet_frames(tri[B0][None])
    verts = mesh.verts.astype(np.float64).copy()
    verts[v] += 1e-3 * (np.asarray(inst.rot, np.float64).T @ nrm[0])
    from scenes import Mesh, Scene
    meshes = [Mesh(verts=verts, tris=m.tris, name=m.name) if m is mesh else m for m in sc.meshes]
    moved = dbounce.pairs_for_table(Scene(meshes, sc.instances), arr, wf, table)
    dF = np.abs(moved[ni][k]["F"][0] - held[ni][k]["F"][0]).max()
    assert 0.0 < dF < 1e-2
