"""Convenience layer over the binding: load a scene, waveform and array into a context
and run echo synthesis and range-Doppler processing into torch device tensors.
All arithmetic happens in librsim; this module only allocates and marshals."""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np
import torch

from .rsim import (Context, POINT_DTYPE, RSIM_FP32_PHASE64, RSIM_FP64, RSIM_MASK_COMPUTE,
                   RSIM_MASK_INPUT)


def pack_mask(mask: np.ndarray) -> np.ndarray:
    """[N, F] bool -> [N, ceil(F/32)] uint32 with bit f % 32 of word f // 32."""
    mask = np.asarray(mask, bool)
    n, f = mask.shape
    words = (f + 31) // 32
    pad = np.zeros((n, words * 32), bool)
    pad[:, :f] = mask
    return np.packbits(pad, axis=1, bitorder="little").view("<u4").reshape(n, words)


def unpack_mask(words: np.ndarray, n_facets: int) -> np.ndarray:
    w = np.ascontiguousarray(words, dtype="<u4")
    bits = np.unpackbits(w.view(np.uint8).reshape(w.shape[0], -1), axis=1, bitorder="little")
    return bits[:, :n_facets].astype(bool)


class Simulator:
    """One context holding a list of scenes sharing one waveform and array."""

    def __init__(self, scenes: Sequence, waveform, array, device: int = 0):
        self.ctx = Context(device)
        self.ctx.set_waveform(waveform)
        self.ctx.set_array(array.tx, array.rx)
        self.wf = waveform
        self.O = self.ctx.n_channels
        self.scene_ids = [self.ctx.load_scene(s) for s in scenes]
        self.inst_pos0 = [[np.asarray(i.pos0, np.float64) for i in s.instances] for s in scenes]
        self.n_facets = [self.ctx.scene_info(s)[0] for s in self.scene_ids]
        self.mask_words = [self.ctx.scene_info(s)[1] for s in self.scene_ids]
        self.dev = torch.device("cuda", device)
        self.intra_chirp = False  # RadarRDM: delay within the chirp, forward and backward

    def echo_buffer(self, n_scenes: int = 1, precision: int = RSIM_FP32_PHASE64):
        dt = torch.complex128 if precision == RSIM_FP64 else torch.complex64
        return torch.empty((n_scenes, self.O, self.wf.n_chirps, self.wf.n_samples), dtype=dt,
                           device=self.dev)

    def set_intra_chirp(self, enable: bool):
        """RadarRDM's forward takes each facet's delay at the sample times (opts.intra_chirp)
        and its backward differentiates that echo (rsim_set_backward_intra_chirp)."""
        self.intra_chirp = bool(enable)

    def set_ground(self, enable: bool, z_ground: float = 0.0, gamma: complex = -1.0):
        """Ground double bounce on/off; while on, masks hold four path types per scene."""
        self.ctx.set_ground(enable, z_ground, gamma)
        self.mask_types = 4 if enable else 1

    def set_double_bounce(self, enable: bool, gamma: complex = -1.0):
        """Facet-to-facet double bounce on/off; while on, a scene's part of a mask buffer
        is followed by its connection table [2][N][F] int32."""
        self.ctx.set_double_bounce(enable, gamma)
        self.db = bool(enable)

    def _mask_span(self, i):
        types = getattr(self, "mask_types", 1)
        span = types * self.wf.n_chirps * self.mask_words[i]
        if getattr(self, "db", False):
            span += 2 * self.wf.n_chirps * self.n_facets[i]
        return span

    def mask_buffer(self, which: Optional[Sequence[int]] = None):
        which = range(len(self.scene_ids)) if which is None else which
        total = sum(self._mask_span(i) for i in which)
        return torch.zeros(max(1, total), dtype=torch.int32, device=self.dev)

    def connections_numpy(self, mask_tensor, which: Optional[Sequence[int]] = None):
        """The connection tables [2, N, F] (facet B or -1) of a mask buffer (double bounce)."""
        which = list(range(len(self.scene_ids))) if which is None else list(which)
        raw = mask_tensor.cpu().numpy().view("<i4")
        out, off = [], 0
        for i in which:
            words = getattr(self, "mask_types", 1) * self.wf.n_chirps * self.mask_words[i]
            n = 2 * self.wf.n_chirps * self.n_facets[i]
            out.append(raw[off + words:off + words + n].reshape(2, self.wf.n_chirps,
                                                                self.n_facets[i]).copy())
            off += self._mask_span(i)
        return out

    def mask_with_connections(self, masks: Sequence[np.ndarray], tables: Sequence[np.ndarray]):
        """A device mask buffer from per-scene lit masks [N, F] and connection tables
        [2, N, F] (double bounce)."""
        parts = []
        for m, t in zip(masks, tables):
            parts.append(pack_mask(m).reshape(-1).view(np.int32))
            parts.append(np.asarray(t, np.int32).reshape(-1))
        return torch.from_numpy(np.concatenate(parts).copy()).to(self.dev)

    def synthesize(self, which: Optional[Sequence[int]] = None, precision=RSIM_FP32_PHASE64,
                   echo=None, mask=None, mask_mode=RSIM_MASK_COMPUTE, **kw):
        which = list(range(len(self.scene_ids))) if which is None else list(which)
        if echo is None:
            echo = self.echo_buffer(len(which), precision)
        self.ctx.synthesize([self.scene_ids[i] for i in which], echo, mask,
                            precision=precision, mask_mode=mask_mode, **kw)
        return echo

    def form_rdm(self, echo, precision=RSIM_FP32_PHASE64, want_y=False, **kw):
        n_cubes = echo.shape[0]
        rdt = torch.float64 if precision == RSIM_FP64 else torch.float32
        rdm = torch.empty(echo.shape, dtype=rdt, device=self.dev)
        y = torch.empty_like(echo) if want_y else None
        self.ctx.form_rdm(echo, rdm, y, n_cubes=n_cubes, precision=precision, **kw)
        return (rdm, y) if want_y else rdm

    def detect(self, rdm, y, max_points: int = 256, guard=(1, 1), train=(2, 4),
               scale: float = 10.0, na_x: int = 0, na_z: int = 0, want_maps: bool = False):
        """CA-CFAR on the channel-integrated RDM and the angle FFT of each detected cell
        (FP32 RDM and Y from form_rdm). Returns (points, counts[, det_mask, noise_map]):
        points a device uint8 tensor [n_cubes, max_points, 64] of Point records
        (points_numpy() decodes them), counts int32 [n_cubes]."""
        n_cubes = rdm.shape[0]
        pts = torch.zeros((n_cubes, max_points, 64), dtype=torch.uint8, device=self.dev)
        cnt = torch.zeros((n_cubes,), dtype=torch.int32, device=self.dev)
        det = noise = None
        if want_maps:
            det = torch.zeros((n_cubes, self.wf.n_chirps, self.wf.n_samples), dtype=torch.uint8,
                              device=self.dev)
            noise = torch.zeros((n_cubes, self.wf.n_chirps, self.wf.n_samples),
                                dtype=torch.float32, device=self.dev)
        self.ctx.detect(rdm, y, pts, cnt, n_cubes=n_cubes, det_mask=det, noise_map=noise,
                        guard=guard, train=train, scale=scale, na_x=na_x, na_z=na_z)
        return (pts, cnt, det, noise) if want_maps else (pts, cnt)

    @staticmethod
    def points_numpy(points, counts):
        """Per cube, a structured numpy array of the written Point records."""
        raw = points.cpu().numpy()
        c = counts.cpu().numpy()
        return [raw[i, :min(int(c[i]), raw.shape[1])].copy().view(POINT_DTYPE).reshape(-1)
                for i in range(raw.shape[0])]

    def add_noise(self, echo, snr_db: float, seed: int, precision=RSIM_FP32_PHASE64):
        """White Gaussian noise at snr_db added in place to each cube of `echo`."""
        self.ctx.add_noise(echo, snr_db, seed, n_cubes=echo.shape[0], precision=precision)
        return echo

    def masks_numpy(self, mask_tensor, which: Optional[Sequence[int]] = None):
        """Split a device mask buffer into per-scene [N, F] bool arrays."""
        which = list(range(len(self.scene_ids))) if which is None else list(which)
        raw = mask_tensor.cpu().numpy().view("<u4")
        out, off = [], 0
        for i in which:
            cnt = self.wf.n_chirps * self.mask_words[i]
            words = raw[off:off + cnt].reshape(self.wf.n_chirps, self.mask_words[i])
            out.append(unpack_mask(words, self.n_facets[i]))
            off += self._mask_span(i)
        return out

    def mask_from_numpy(self, masks: Sequence[np.ndarray]):
        packed = np.concatenate([pack_mask(m).reshape(-1) for m in masks])
        return torch.from_numpy(packed.view(np.int32).copy()).to(self.dev)
