"""Coherent facet sum: the echo's frequency response per virtual channel and chirp
(test infrastructure; FP64, direct evaluation of every term, no recurrences).

Paper basis:
  * eq. (7)  radar equation: received power P_t G_TX sigma G_RX lambda^2 / ((4 pi)^3 d^4);
  * eq. (8)  complex FMCW chirp; ADC sample m sits at frequency f_m = f0 + m df;
  * eqs. (9)-(11) echo as the target's frequency response (sigma_f from BART per
    chirp) applied to the chirp, brought to the time domain by an inverse transform;
  * eq. (12) round-trip delay tau = 2 (d + v t) / c;
  * eq. (13) beat signal P sigma exp{j 2 pi [f0 tau + mu t tau - mu tau^2 / 2]};
  * Section 3.3: P Tx x Q Rx give O = P Q channels, N chirps of M samples.

Readings where the paper is silent or garbled:
  * Field amplitude per facet from eq. (7) with isotropic unit-gain antennas and
    P_t = 1: the facet term is a(m) = j o I(k_m) / (4 pi R_t R_r), where I is the
    closed-form facet integral (facet_integral.py), o = n . (u_t + u_r) / 2 the
    obliquity and R_t, R_r the exact distances from the facet centroid to the Tx
    and Rx elements. For a flat plate at normal incidence |a|^2 equals eq. (7)
    with sigma = 4 pi A^2 / lambda^2 (the lambda factors cancel since lambda k = 2 pi).
  * Stop-and-hop: the geometry of chirp n is frozen at t_n = n T_c (eq. (12) per chirp).
  * The response carries exp(-j 2 pi (f_m tau - mu tau^2 / 2)), tau = (R_t + R_r)/c,
    so that conj(H) at sample m equals eq. (13) for a point target (beat = conj(H)).
  * Point scatterers: amplitude s / (4 pi R_t R_r) with a constant complex s (m^2)
    and the same phase term.

Output layout: H[o, n, m] complex128, channel o = p * Q + q.
"""
from __future__ import annotations

import numpy as np

from .constants import C0
from .facet_integral import facet_integral
from .geometry import facet_frames, point_positions, world_triangles
from .visibility import visibility


def _phase_turns(freqs, tau, slope):
    """f_m tau - mu tau^2 / 2 in turns, reduced to [0, 1) (subtracting an integer is
    exact in FP64, so only the product's rounding remains)."""
    ph = freqs[None, :] * tau[:, None] - 0.5 * slope * (tau * tau)[:, None]
    return ph - np.floor(ph)


def facet_terms(tri: np.ndarray, wf, array, freqs: np.ndarray, channels):
    """Sum over the given world triangles [F,3,3] of the facet terms for the
    selected channels (list of (p, q)) and frequencies: returns [len(channels), M_sel]."""
    tx = np.asarray(array.tx, np.float64)
    rx = np.asarray(array.rx, np.float64)
    tx_c, rx_c = tx.mean(axis=0), rx.mean(axis=0)
    out = np.zeros((len(channels), freqs.size), np.complex128)
    if tri.shape[0] == 0:
        return out
    c, nrm, area = facet_frames(tri)
    ut = tx_c - c
    ut /= np.linalg.norm(ut, axis=1, keepdims=True)
    ur = rx_c - c
    ur /= np.linalg.norm(ur, axis=1, keepdims=True)
    w = ut + ur
    obl = 0.5 * np.einsum("ij,ij->i", nrm, w)
    beta = np.einsum("fij,fj->fi", tri - c[:, None, :], w)  # [F, 3]
    k = 2.0 * np.pi * freqs / C0
    integ = facet_integral(k[None, :], beta[:, None, :], area[:, None])  # [F, M]
    rt = np.linalg.norm(tx[None, :, :] - c[:, None, :], axis=2)  # [F, P]
    rr = np.linalg.norm(rx[None, :, :] - c[:, None, :], axis=2)  # [F, Q]
    for ci, (p, q) in enumerate(channels):
        tau = (rt[:, p] + rr[:, q]) / C0
        amp = 1j * obl / (4.0 * np.pi * rt[:, p] * rr[:, q])
        ph = _phase_turns(freqs, tau, wf.slope)
        out[ci] = np.sum(amp[:, None] * integ * np.exp(-2j * np.pi * ph), axis=0)
    return out


def point_terms(pos: np.ndarray, amp: np.ndarray, wf, array, freqs, channels):
    """Sum of point-scatterer terms s / (4 pi R_t R_r) exp(-j 2 pi (f tau - mu tau^2/2))."""
    tx = np.asarray(array.tx, np.float64)
    rx = np.asarray(array.rx, np.float64)
    out = np.zeros((len(channels), freqs.size), np.complex128)
    if pos.shape[0] == 0:
        return out
    rt = np.linalg.norm(tx[None, :, :] - pos[:, None, :], axis=2)
    rr = np.linalg.norm(rx[None, :, :] - pos[:, None, :], axis=2)
    for ci, (p, q) in enumerate(channels):
        tau = (rt[:, p] + rr[:, q]) / C0
        a = amp / (4.0 * np.pi * rt[:, p] * rr[:, q])
        ph = _phase_turns(freqs, tau, wf.slope)
        out[ci] = np.sum(a[:, None] * np.exp(-2j * np.pi * ph), axis=0)
    return out


def synthesize(scene, wf, array, mask=None, chirps=None, channels=None, samples=None,
               chunk: int = 2048, return_mask: bool = False):
    """Echo frequency response H[o, n, m] (complex128) of a scene.

    mask: optional lit-facet mask [n_chirps_total, F] (bool) to use instead of the
    brute-force visibility; chirps / channels / samples: optional index subsets
    (channels as flat indices o = p Q + q). Returns H[len(channels), len(chirps),
    len(samples)] (and the per-chirp masks used when return_mask)."""
    P, Q = array.tx.shape[0], array.rx.shape[0]
    chirps = np.arange(wf.n_chirps) if chirps is None else np.asarray(chirps)
    channels = np.arange(P * Q) if channels is None else np.asarray(channels)
    samples = np.arange(wf.n_samples) if samples is None else np.asarray(samples)
    pq = [(int(o) // Q, int(o) % Q) for o in channels]
    df = wf.slope / wf.fs
    freqs = wf.f0 + df * samples.astype(np.float64)
    H = np.zeros((channels.size, chirps.size, samples.size), np.complex128)
    used = []
    for ni, n in enumerate(chirps):
        t = float(n) * wf.chirp_period
        tri, _, _ = world_triangles(scene, t)
        if mask is None:
            lit, _ = visibility(scene, array, wf, chirps=[n])
            lit = lit[0]
        else:
            lit = np.asarray(mask[int(n)], bool)
        used.append(lit)
        idx = np.nonzero(lit)[0]
        for s0 in range(0, idx.size, chunk):
            H[:, ni, :] += facet_terms(tri[idx[s0:s0 + chunk]], wf, array, freqs, pq)
        if scene.points is not None and scene.points.n:
            H[:, ni, :] += point_terms(point_positions(scene, t), scene.points.amp, wf,
                                       array, freqs, pq)
    if return_mask:
        return H, np.array(used)
    return H
