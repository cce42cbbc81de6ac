"""Write tests/golden/c3_oracle_samples.npz: the FP64 oracle on the 1M-triangle
intersection workload (ground grid + 20 vehicles, 192 channels, 512 samples x 256 chirps)
at chirps {0, 255}: the lit mask and its ambiguity flags over every facet, and the echo
H[o, n, m] for six channels spread over the array and all 512 samples, summed over every
lit facet (Sections 2.2 and 3.2, eqs. (7)-(13), as the oracle reads them).

Calls only oracle/ and scenes/. The work is split over forked processes: visibility by
blocks of facets, the echo by blocks of lit facets (the sum is linear in the facets).

  python tests/golden/make_c3_samples.py [--workers 8]
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

CHIRPS = (0, 255)
CHANNELS = (0, 37, 95, 128, 160, 191)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_oracle_samples.npz")

_CFG = None


def _vis(task):
    n, facets = task
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        m, a = oracle.visibility(_CFG.scenes[0], _CFG.array, _CFG.waveform, chirps=[n],
                                 facets=facets)
    return m[0], a[0]


def _sum(task):
    n, lit = task
    from threadpoolctl import threadpool_limits
    sc = _CFG.scenes[0]
    row = np.zeros(sc.n_tris, bool)
    row[lit] = True
    with threadpool_limits(1):
        H = oracle.synthesize(sc, _CFG.waveform, _CFG.array, mask={int(n): row}, chirps=[n],
                              channels=np.array(CHANNELS))
    return H[:, 0, :]


def main():
    import multiprocessing as mp
    global _CFG
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    _CFG = scenes.c3()
    sc, wf = _CFG.scenes[0], _CFG.waveform
    F = sc.n_tris
    blocks = np.array_split(np.arange(F), 4 * args.workers)
    masks, ambs, H = [], [], []
    with mp.get_context("fork").Pool(args.workers) as pool:
        for n in CHIRPS:
            t0 = time.time()
            res = pool.map(_vis, [(n, b) for b in blocks])
            m = np.concatenate([r[0] for r in res])
            a = np.concatenate([r[1] for r in res])
            lit = np.nonzero(m)[0]
            print(f"chirp {n}: lit {lit.size} ambiguous {int(a.sum())} "
                  f"({time.time() - t0:.0f} s)", flush=True)
            t0 = time.time()
            parts = pool.map(_sum, [(n, b) for b in np.array_split(lit, 4 * args.workers)])
            Hn = np.zeros((len(CHANNELS), wf.n_samples), np.complex128)
            for p in parts:  # fixed order
                Hn += p
            print(f"chirp {n}: echo ({time.time() - t0:.0f} s)", flush=True)
            masks.append(m)
            ambs.append(a)
            H.append(Hn)
    np.savez_compressed(
        OUT, chirps=np.array(CHIRPS), channels=np.array(CHANNELS),
        mask=np.packbits(np.array(masks), axis=1, bitorder="little"),
        ambiguous=np.packbits(np.array(ambs), axis=1, bitorder="little"),
        n_facets=np.int64(F), echo=np.stack(H, axis=1), scene_sha16=scenes.scene_digest(sc),
        note=np.array("FP64 oracle (oracle.visibility, oracle.synthesize) on scenes.c3(); "
                      "echo[o_sel, n_sel, m] for the listed chirps and channels, all samples"))
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
