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
    Optionally (intra_chirp=True) the propagation delay of eqs. (12)-(13) is taken at
    each sample time t_n + m / fs: the facet centroid (or point) moves with its velocity
    within the chirp; the amplitude, the facet integral and the lit set stay at t_n
    (eq. (13) holds P sigma constant while tau(t) varies).
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


def _moving_distances(elems, c, vel, dt):
    """|e - (c_f + v_f dt_m)| for elements [E,3], centroids [F,3], velocities [F,3] and
    sample times dt [M_sel]: returns [F, E, M_sel]."""
    pos = c[:, None, :] + vel[:, None, :] * dt[None, :, None]  # [F, M, 3]
    return np.linalg.norm(elems[None, :, None, :] - pos[:, None, :, :], axis=3)


def facet_terms(tri: np.ndarray, wf, array, freqs: np.ndarray, channels, vel=None, dt=None):
    """Sum over the given world triangles [F,3,3] of the facet terms for the
    selected channels (list of (p, q)) and frequencies: returns [len(channels), M_sel].
    With vel [F,3] and dt [M_sel] (seconds after t_n) the delay is taken at the sample
    times; amplitude and facet integral stay at t_n."""
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
    if vel is not None:
        rt_m = _moving_distances(tx, c, vel, dt)  # [F, P, M]
        rr_m = _moving_distances(rx, c, vel, dt)
    for ci, (p, q) in enumerate(channels):
        amp = 1j * obl / (4.0 * np.pi * rt[:, p] * rr[:, q])
        if vel is None:
            ph = _phase_turns(freqs, (rt[:, p] + rr[:, q]) / C0, wf.slope)
        else:
            tau = (rt_m[:, p, :] + rr_m[:, q, :]) / C0  # [F, M]
            ph = freqs[None, :] * tau - 0.5 * wf.slope * tau * tau
            ph -= np.floor(ph)
        out[ci] = np.sum(amp[:, None] * integ * np.exp(-2j * np.pi * ph), axis=0)
    return out


def point_terms(pos: np.ndarray, amp: np.ndarray, wf, array, freqs, channels, vel=None,
                dt=None):
    """Sum of point-scatterer terms s / (4 pi R_t R_r) exp(-j 2 pi (f tau - mu tau^2/2));
    with vel and dt the delay is taken at the sample times (amplitude at t_n)."""
    tx = np.asarray(array.tx, np.float64)
    rx = np.asarray(array.rx, np.float64)
    out = np.zeros((len(channels), freqs.size), np.complex128)
    if pos.shape[0] == 0:
        return out
    rt = np.linalg.norm(tx[None, :, :] - pos[:, None, :], axis=2)
    rr = np.linalg.norm(rx[None, :, :] - pos[:, None, :], axis=2)
    if vel is not None:
        rt_m = _moving_distances(tx, pos, vel, dt)
        rr_m = _moving_distances(rx, pos, vel, dt)
    for ci, (p, q) in enumerate(channels):
        a = amp / (4.0 * np.pi * rt[:, p] * rr[:, q])
        if vel is None:
            ph = _phase_turns(freqs, (rt[:, p] + rr[:, q]) / C0, wf.slope)
        else:
            tau = (rt_m[:, p, :] + rr_m[:, q, :]) / C0
            ph = freqs[None, :] * tau - 0.5 * wf.slope * tau * tau
            ph -= np.floor(ph)
        out[ci] = np.sum(a[:, None] * np.exp(-2j * np.pi * ph), axis=0)
    return out


def synthesize(scene, wf, array, mask=None, chirps=None, channels=None, samples=None,
               chunk: int = 2048, return_mask: bool = False, intra_chirp: bool = False):
    """Echo frequency response H[o, n, m] (complex128) of a scene.

    mask: optional lit-facet mask [n_chirps_total, F] (bool) to use instead of the
    brute-force visibility; chirps / channels / samples: optional index subsets
    (channels as flat indices o = p Q + q). Returns H[len(channels), len(chirps),
    len(samples)] (and the per-chirp masks used when return_mask). intra_chirp: delay at
    each sample time t_n + m / fs instead of t_n."""
    P, Q = array.tx.shape[0], array.rx.shape[0]
    chirps = np.arange(wf.n_chirps) if chirps is None else np.asarray(chirps)
    channels = np.arange(P * Q) if channels is None else np.asarray(channels)
    samples = np.arange(wf.n_samples) if samples is None else np.asarray(samples)
    pq = [(int(o) // Q, int(o) % Q) for o in channels]
    df = wf.slope / wf.fs
    freqs = wf.f0 + df * samples.astype(np.float64)
    H = np.zeros((channels.size, chirps.size, samples.size), np.complex128)
    used = []
    dt = samples.astype(np.float64) / wf.fs if intra_chirp else None
    for ni, n in enumerate(chirps):
        t = float(n) * wf.chirp_period
        tri, inst_of, _ = world_triangles(scene, t)
        fvel = (np.array([scene.instances[i].vel for i in inst_of], np.float64).reshape(-1, 3)
                if intra_chirp else None)
        if mask is None:
            lit, _ = visibility(scene, array, wf, chirps=[n])
            lit = lit[0]
        else:
            lit = np.asarray(mask[int(n)], bool)
        used.append(lit)
        idx = np.nonzero(lit)[0]
        for s0 in range(0, idx.size, chunk):
            sel = idx[s0:s0 + chunk]
            H[:, ni, :] += facet_terms(tri[sel], wf, array, freqs, pq,
                                       vel=None if fvel is None else fvel[sel], dt=dt)
        if scene.points is not None and scene.points.n:
            H[:, ni, :] += point_terms(point_positions(scene, t), scene.points.amp, wf,
                                       array, freqs, pq,
                                       vel=scene.points.vel if intra_chirp else None, dt=dt)
    if return_mask:
        return H, np.array(used)
    return H
