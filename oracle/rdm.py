"""Beat signal, range FFT, Doppler FFT and range-Doppler map (test infrastructure).

Section 3.3: the O x M x N cube goes through an FFT over the samples of a chirp
(range) and an FFT over the chirps (Doppler); the RDM is read off the result.
eqs. (10)-(11): the paper's inverse transform of the frequency-domain echo is read
as the range transform of the beat signal, beat = conj(H) (eq. (13)), so that
X[o, n, k] = sum_m conj(H[o, n, m]) exp(-j 2 pi m k / M) = M conj(IFFT_m(H)).
Unnormalised forward FFTs, no window, power RDM |Y|^2 with the Doppler axis shifted
so that row l holds Doppler index l' = l - N/2 (eq. (5): positive = receding).
"""
from __future__ import annotations

import numpy as np


def beat(H: np.ndarray) -> np.ndarray:
    """Beat (IF) samples of eq. (13): the conjugate of the frequency response."""
    return np.conj(H)


def range_fft(x: np.ndarray) -> np.ndarray:
    """Unnormalised forward DFT over the last axis (samples within a chirp)."""
    return np.fft.fft(x, axis=-1)


def doppler_fft(X: np.ndarray) -> np.ndarray:
    """Unnormalised forward DFT over the chirp axis (-2), zero Doppler moved to row N/2."""
    return np.fft.fftshift(np.fft.fft(X, axis=-2), axes=-2)


def rdm(Y: np.ndarray) -> np.ndarray:
    """Range-Doppler power map |Y|^2."""
    return np.abs(Y) ** 2


def rdm_from_echo(H: np.ndarray):
    """H[..., N, M] -> (RDM [..., N, M] float64, Y [..., N, M] complex128)."""
    Y = doppler_fft(range_fft(beat(H)))
    return rdm(Y), Y


def rdm_loss(P: np.ndarray, T: np.ndarray) -> float:
    """Sum of squared differences between a power RDM and a target RDM."""
    return float(np.sum((P - T) ** 2))
