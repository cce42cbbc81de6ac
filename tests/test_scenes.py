"""Synthetic input generators: sizes, determinism and outward winding (no GPU)."""
import numpy as np

import scenes


def _signed_volume(m):
    v = m.verts.astype(np.float64)[m.tris]
    return np.sum(np.einsum("ij,ij->i", v[:, 0], np.cross(v[:, 1], v[:, 2]))) / 6.0


def test_c1_box_has_1000_triangles_and_is_closed_outward():
    cfg = scenes.c1()
    m = cfg.scenes[0].meshes[0]
    assert m.n_tris == 1000
    assert np.isclose(_signed_volume(m), 4.5 * 1.8 * 1.5, rtol=1e-6)
    # every edge shared by exactly two triangles (watertight after welding)
    e = np.sort(np.concatenate([m.tris[:, [0, 1]], m.tris[:, [1, 2]], m.tris[:, [2, 0]]]), axis=1)
    _, counts = np.unique(e, axis=0, return_counts=True)
    assert np.all(counts == 2)


def test_hull_sizes_and_determinism():
    for cls, target in (("car", 50_000), ("bus", 44_250), ("motorcycle", 5_000)):
        m = scenes.vehicle_mesh(cls, target)
        assert abs(m.n_tris - target) <= 0.01 * target
        assert _signed_volume(m) > 0
    a, b = scenes.c2(), scenes.c2()
    assert np.array_equal(a.scenes[0].meshes[0].verts, b.scenes[0].meshes[0].verts)
    assert np.array_equal(a.array.tx, b.array.tx)
    assert a.array.n_channels == 192


def test_waveforms_match_paper_setup():
    wf = scenes.paper_waveform(256, 128)
    assert np.isclose(wf.chirp_period, 60e-6)
    assert np.isclose(wf.n_samples * wf.slope / wf.fs, 0.625e9)
    lit = scenes.literal_77_81_waveform()
    assert np.isclose(lit.n_samples * lit.slope / lit.fs, 4e9)
