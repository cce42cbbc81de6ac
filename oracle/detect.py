"""CA-CFAR detection on the range-Doppler map, angle FFT across the virtual array and
the point cloud (test infrastructure; FP64).

Section 3.3: after the range and Doppler transforms, constant-false-alarm-rate
detection with the cell-averaging rule (CA-CFAR) finds the target cells; an FFT over
the angle dimension of the channels gives each detected cell's direction (eq. (6):
theta = asin(lambda dphi / (2 pi d))); range and angle together place the point.

Readings where the paper is silent:
  * Detection runs on the channel-integrated map P[n, m] = sum_o |Y_o[n, m]|^2
    (non-coherent integration over the O virtual channels).
  * CA-CFAR window: guard cells g_d (Doppler) x g_r (range) on each side of the cell
    under test, then t_d x t_r training cells beyond the guard band on each side; the
    noise level is the mean of P over the training ring (the full rectangle minus the
    guard rectangle, K cells). Both axes are periodic (both transforms are DFTs), so
    the window wraps. Detected: P[n, m] > scale * noise[n, m], strictly.
  * Detections are listed in ascending row-major order (Doppler row, then range bin).
  * Angle FFT: virtual element o = (p, q) sits at tx_p + rx_q; the positions must lie
    on a half-wavelength grid (lambda_c / 2 at band centre) in the array's x-z plane.
    Channel values at one grid node are averaged; empty nodes are zero; the grid is
    zero-padded to na_x x na_z and transformed by a 2-D unnormalised DFT. The peak of
    |A|^2 (first maximum in row-major order) at signed bins (kx, kz) gives the
    direction cosines u = -2 kx / na_x (along x) and w = -2 kz / na_z (along z): for a
    target in direction d the channel phases of Y follow exp(-j k_c d . v_o), since
    Y is formed from the beat signal conj(H).
  * Point: c_ref + R (u, sqrt(max(0, 1 - u^2 - w^2)), w), with c_ref the midpoint of
    the Tx and Rx phase centres, boresight +y, R from the range bin (eq. (4)) and the
    radial velocity from the Doppler row (eq. (5)).
"""
from __future__ import annotations

import numpy as np

from .waveform import derived, range_axis, velocity_axis


def integrate(P: np.ndarray) -> np.ndarray:
    """Channel-integrated map: P[..., O, N, M] -> sum over O."""
    return np.sum(P, axis=-3)


def ca_cfar(Pi: np.ndarray, guard=(1, 1), train=(2, 4), scale: float = 10.0):
    """CA-CFAR on one integrated map Pi[N, M]. guard = (g_d, g_r), train = (t_d, t_r).
    Returns (detected bool [N, M], noise [N, M], K)."""
    gd, gr = guard
    td, tr = train
    hd, hr = gd + td, gr + tr
    total = np.zeros_like(Pi, dtype=np.float64)
    count = 0
    for dn in range(-hd, hd + 1):
        for dm in range(-hr, hr + 1):
            if abs(dn) <= gd and abs(dm) <= gr:
                continue  # guard rectangle, cell under test included
            # value at (n + dn, m + dm), indices modulo N and M
            total += np.roll(Pi, shift=(-dn, -dm), axis=(0, 1))
            count += 1
    noise = total / count
    return Pi > scale * noise, noise, count


def virtual_grid(arr, wf):
    """Half-wavelength grid indices of the virtual elements tx_p + rx_q (channel
    o = p Q + q) in the x-z plane: returns (ix [O], iz [O], nx, nz, d)."""
    d = 0.5 * derived(wf)["lambda_c"]
    v = (arr.tx[:, None, :] + arr.rx[None, :, :]).reshape(-1, 3)
    gx = (v[:, 0] - v[:, 0].min()) / d
    gz = (v[:, 2] - v[:, 2].min()) / d
    ix, iz = np.rint(gx).astype(np.int64), np.rint(gz).astype(np.int64)
    if np.max(np.abs(gx - ix)) > 1e-6 or np.max(np.abs(gz - iz)) > 1e-6:
        raise ValueError("virtual elements are not on a half-wavelength grid")
    if np.ptp(v[:, 1]) > 1e-9:
        raise ValueError("virtual elements are not in one x-z plane")
    return ix, iz, int(ix.max()) + 1, int(iz.max()) + 1, d


def angle_spectrum(y: np.ndarray, ix, iz, na_x: int, na_z: int) -> np.ndarray:
    """|2-D DFT|^2 [na_z, na_x] of the channel values y[O] placed on the virtual grid
    (duplicates averaged, empty nodes zero, zero-padded)."""
    g = np.zeros((na_z, na_x), dtype=np.complex128)
    c = np.zeros((na_z, na_x))
    for o in range(y.shape[0]):
        g[iz[o], ix[o]] += y[o]
        c[iz[o], ix[o]] += 1.0
    g[c > 0] /= c[c > 0]
    return np.abs(np.fft.fft2(g)) ** 2


def direction_from_peak(A: np.ndarray):
    """(u, w, kx, kz, peak) from an angle spectrum A[na_z, na_x]: first maximum in
    row-major order, signed bins, u = -2 kx / na_x and w = -2 kz / na_z."""
    na_z, na_x = A.shape
    flat = int(np.argmax(A))
    kz, kx = divmod(flat, na_x)
    skx = kx - na_x if kx >= (na_x + 1) // 2 else kx
    skz = kz - na_z if kz >= (na_z + 1) // 2 else kz
    u = -2.0 * skx / na_x
    w = -2.0 * skz / na_z if na_z > 1 else 0.0
    return u, w, skx, skz, float(A.flat[flat])


def point_cloud(P: np.ndarray, Y: np.ndarray, wf, arr, guard=(1, 1), train=(2, 4),
                scale: float = 10.0, na_x: int = 0, na_z: int = 0):
    """Detections and points of one frame: P [O, N, M] power, Y [O, N, M] complex.
    na_x / na_z = 0 pick the smallest 2^a 3^b >= twice the grid extent (1 for a flat
    grid). Returns a list of dicts in row-major (Doppler row, range bin) order."""
    ix, iz, nx, nz, _ = virtual_grid(arr, wf)
    if na_x <= 0:
        na_x = _fft_len(2 * nx)
    if na_z <= 0:
        na_z = 1 if nz == 1 else _fft_len(2 * nz)
    Pi = integrate(P)
    det, noise, _ = ca_cfar(Pi, guard, train, scale)
    rng = range_axis(wf)
    vel = velocity_axis(wf)
    c_ref = 0.5 * (arr.tx.mean(0) + arr.rx.mean(0))
    out = []
    for n, m in zip(*np.nonzero(det)):
        A = angle_spectrum(Y[:, n, m], ix, iz, na_x, na_z)
        u, w, kx, kz, peak = direction_from_peak(A)
        R = rng[m]
        dirv = np.array([u, np.sqrt(max(0.0, 1.0 - u * u - w * w)), w])
        out.append({"row": int(n), "bin": int(m), "power": float(Pi[n, m]),
                    "noise": float(noise[n, m]), "range": float(R), "velocity": float(vel[n]),
                    "u": u, "w": w, "kx": kx, "kz": kz, "angle_peak": peak,
                    "xyz": c_ref + R * dirv})
    return out


def _fft_len(n: int) -> int:
    """Smallest 2^a 3^b >= n."""
    best = None
    p2 = 1
    while p2 < 4 * n:
        p = p2
        while p < 4 * n:
            if p >= n and (best is None or p < best):
                best = p
            p *= 3
        p2 *= 2
    return best
