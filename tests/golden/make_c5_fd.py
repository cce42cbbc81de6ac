"""Write tests/golden/c5_fd.npz: FP64 central finite differences of the RDM loss of the
gradient workload (two vehicles of 100k triangles each, car and truck at 20-40 m; target
RDM from the seeded perturbed scene) at the reduced frame of 32 samples, 4 Tx x 4 Rx and
8 chirps, so that the oracle forms every chirp.

Loss L = sum (P - T)^2 over the power RDM P = |Y|^2 of the echo H with the lit masks held
fixed (Section 3.3; eqs. (7)-(13) as the oracle reads them). A parameter step changes the
echo by dH (only the facets it moves contribute, by linearity of the facet sum); then
dY = FFT(dH), dP = 2 Re(conj(Y) dY) + |dY|^2 and dL = sum dP (2 (P - T) + dP), with no
cancellation against L itself. Central differences:
  * 50 body-frame vertices x 3 coordinates, step 1e-6 m: 25 drawn uniformly from all
    vertices of both meshes and 25 from the vertices of facets lit at some chirp;
  * every velocity component of both vehicles, step 1e-4 m/s.

Calls only oracle/ and scenes/; the work is split over forked processes by chirp.

  python tests/golden/make_c5_fd.py [--workers 8]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import scenes  # noqa: E402
from oracle.echo import facet_terms  # noqa: E402
from oracle.geometry import world_triangles  # noqa: E402
from scenes import RadarArray  # noqa: E402

M, N, PQ = 32, 8, 4
H_VERT, H_VEL = 1e-6, 1e-4
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_fd.npz")

_W = {}


def workload():
    base = scenes.c5(n_samples=M, n_chirps=N)
    sc, wf = base.scenes[0], base.waveform
    arr = RadarArray(tx=base.array.tx[:PQ].copy(), rx=base.array.rx[:PQ].copy())
    return sc, wf, arr, base.notes["target_scene"]


def _vis(task):
    which, n = task
    sc = _W["scene"] if which == 0 else _W["target"]
    m, a = oracle.visibility(sc, _W["arr"], _W["wf"], chirps=[n])
    return m[0], a[0]


def _echo(task):
    which, n, lit = task
    sc = _W["scene"] if which == 0 else _W["target"]
    row = np.zeros(sc.n_tris, bool)
    row[lit] = True
    return oracle.synthesize(sc, _W["wf"], _W["arr"], mask={int(n): row}, chirps=[n])[:, 0, :]


def _freqs(wf):
    return wf.f0 + wf.slope / wf.fs * np.arange(wf.n_samples)


def _pq(arr):
    Q = arr.rx.shape[0]
    return [(o // Q, o % Q) for o in range(arr.tx.shape[0] * Q)]


def _vel_delta(task):
    """dH for instance ii's velocity component ax moved by dv: the lit facets of that
    instance at every chirp, moved minus unmoved."""
    ii, ax, dv = task
    sc, wf, arr, mask = _W["scene"], _W["wf"], _W["arr"], _W["mask"]
    out = np.zeros((len(_pq(arr)), wf.n_chirps, wf.n_samples), np.complex128)
    for n in range(wf.n_chirps):
        t = n * wf.chirp_period
        tri, inst_of, _ = world_triangles(sc, t)
        sel = np.nonzero(mask[n] & (inst_of == ii))[0]
        if sel.size == 0 or t == 0.0:
            continue
        shift = np.zeros(3)
        shift[ax] = dv * t
        moved = tri[sel] + shift
        out[:, n, :] = (facet_terms(moved, wf, arr, _freqs(wf), _pq(arr)) -
                        facet_terms(tri[sel], wf, arr, _freqs(wf), _pq(arr)))
    return out


def vertex_delta(sc, wf, arr, mask, k, v, ax, dv):
    """dH for body vertex v of mesh k moved by dv along axis ax (every instance of the
    mesh): its incident lit facets at every chirp, moved minus unmoved."""
    out = np.zeros((len(_pq(arr)), wf.n_chirps, wf.n_samples), np.complex128)
    m = sc.meshes[k]
    inc = np.nonzero((m.tris == v).any(axis=1))[0]
    base_of = {}
    off = 0
    for ii, inst in enumerate(sc.instances):
        base_of[ii] = off
        off += sc.meshes[inst.mesh].n_tris
    vb = m.verts.astype(np.float64)
    vb2 = vb.copy()
    vb2[v, ax] += dv
    for ii, inst in enumerate(sc.instances):
        if inst.mesh != k:
            continue
        for n in range(wf.n_chirps):
            lit = inc[mask[n, base_of[ii] + inc]]
            if lit.size == 0:
                continue
            t = n * wf.chirp_period
            for vv, sign in ((vb2, 1.0), (vb, -1.0)):
                w = vv @ inst.rot.T + (inst.pos0 + inst.vel * t)
                out[:, n, :] += sign * facet_terms(w[m.tris[lit]], wf, arr, _freqs(wf), _pq(arr))
    return out


def dloss(dH, Y0, P0, T):
    dY = oracle.doppler_fft(oracle.range_fft(oracle.beat(dH)))
    dP = 2.0 * np.real(np.conj(Y0) * dY) + np.abs(dY) ** 2
    return float(np.sum(dP * (2.0 * (P0 - T) + dP)))


def main():
    import multiprocessing as mp
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    sc, wf, arr, target = workload()
    _W.update(scene=sc, target=target, wf=wf, arr=arr)
    t0 = time.time()
    with mp.get_context("fork").Pool(args.workers) as pool:
        vis = pool.map(_vis, [(w, n) for w in (0, 1) for n in range(N)])
    mask = np.array([v[0] for v in vis[:N]])
    amb = np.array([v[1] for v in vis[:N]])
    tmask = np.array([v[0] for v in vis[N:]])
    print(f"visibility: lit/chirp {mask.sum(1)} ({time.time() - t0:.0f} s)", flush=True)
    _W["mask"] = mask
    t0 = time.time()
    tasks = [(0, n, np.nonzero(mask[n])[0]) for n in range(N)]
    tasks += [(1, n, np.nonzero(tmask[n])[0]) for n in range(N)]
    with mp.get_context("fork").Pool(args.workers) as pool:
        rows = pool.map(_echo, tasks)
    H0 = np.stack(rows[:N], axis=1)
    HT = np.stack(rows[N:], axis=1)
    P0, Y0 = oracle.rdm_from_echo(H0)
    T, _ = oracle.rdm_from_echo(HT)
    print(f"echo and target ({time.time() - t0:.0f} s)", flush=True)
    # vertices: 25 uniform, 25 on facets lit at some chirp
    rng = np.random.default_rng(55)
    nv = [m.verts.shape[0] for m in sc.meshes]
    picks = []
    for _ in range(25):
        k = int(rng.integers(0, len(nv)))
        picks.append((k, int(rng.integers(0, nv[k]))))
    tri_inst = np.concatenate([np.full(sc.meshes[i.mesh].n_tris, j)
                               for j, i in enumerate(sc.instances)])
    tri_local = np.concatenate([np.arange(sc.meshes[i.mesh].n_tris) for i in sc.instances])
    lit_any = np.nonzero(mask.any(axis=0))[0]
    for f in rng.choice(lit_any, 25, replace=False):
        k = sc.instances[int(tri_inst[f])].mesh
        picks.append((k, int(sc.meshes[k].tris[tri_local[f], int(rng.integers(0, 3))])))
    t0 = time.time()
    fd_vert = np.zeros((len(picks), 3))
    for i, (k, v) in enumerate(picks):
        for ax in range(3):
            lp = dloss(vertex_delta(sc, wf, arr, mask, k, v, ax, H_VERT), Y0, P0, T)
            lm = dloss(vertex_delta(sc, wf, arr, mask, k, v, ax, -H_VERT), Y0, P0, T)
            fd_vert[i, ax] = (lp - lm) / (2.0 * H_VERT)
    print(f"vertex differences ({time.time() - t0:.0f} s)", flush=True)
    t0 = time.time()
    vt = [(ii, ax, s * H_VEL) for ii in range(len(sc.instances)) for ax in range(3)
          for s in (1.0, -1.0)]
    with mp.get_context("fork").Pool(args.workers) as pool:
        dHs = pool.map(_vel_delta, vt)
    fd_vel = np.zeros((len(sc.instances), 3))
    for j in range(0, len(vt), 2):
        ii, ax, _ = vt[j]
        fd_vel[ii, ax] = (dloss(dHs[j], Y0, P0, T) - dloss(dHs[j + 1], Y0, P0, T)) / (2.0 * H_VEL)
    print(f"velocity differences ({time.time() - t0:.0f} s)", flush=True)
    np.savez_compressed(
        OUT, mask=np.packbits(mask, axis=1, bitorder="little"),
        ambiguous=np.packbits(amb, axis=1, bitorder="little"), n_facets=np.int64(sc.n_tris),
        target_rdm=T, vert_mesh=np.array([p[0] for p in picks]),
        vert_index=np.array([p[1] for p in picks]), fd_vert=fd_vert, fd_vel=fd_vel,
        loss=np.float64(oracle.rdm_loss(P0, T)), scene_sha16=scenes.scene_digest(sc),
        target_sha16=scenes.scene_digest(target),
        frame=np.array([M, PQ, PQ, N]), steps=np.array([H_VERT, H_VEL]),
        note=np.array("FP64 oracle central differences of sum (RDM - T)^2, masks fixed; "
                      "vertices in the body frame of their mesh"))
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
