"""FMCW waveform quantities (test infrastructure; FP64).

Follows Section 2.1 (eqs. (3)-(5)), Section 3.2 (eq. (8)) and the experiment setup
of Section 4.1 with Table 2. Readings where the paper is silent:
  * frequency grid f_m = f0 + m * df, df = slope / fs, m = 0..M-1 (sweep end excluded);
  * chirp start times t_n = n * T_c (stop-and-hop, see echo.py);
  * wavelength in eq. (5) and in the maximum velocity taken at band centre,
    lambda_c = c / (f0 + B/2), B = M * df (reproduces Table 2's 16.16/11.38/8.78 m/s).
"""
from __future__ import annotations

import numpy as np

from .constants import C0


def derived(wf) -> dict:
    """Derived sweep quantities of a waveform (f0, slope, fs, chirp_period, M, N)."""
    df = wf.slope / wf.fs  # frequency step between ADC samples
    bw = wf.n_samples * df  # swept bandwidth while sampling
    lam_c = C0 / (wf.f0 + 0.5 * bw)
    return {
        "df": df,
        "bandwidth": bw,
        "freqs": wf.f0 + df * np.arange(wf.n_samples),
        "chirp_times": wf.chirp_period * np.arange(wf.n_chirps),
        "range_resolution": C0 / (2.0 * bw),
        # eq. (4) with the largest beat frequency the complex ADC resolves (fs)
        "max_range": C0 * wf.fs / (2.0 * wf.slope),
        "lambda_c": lam_c,
        # eq. (5) with a phase step of +-pi between chirps
        "max_velocity": lam_c / (4.0 * wf.chirp_period),
        "velocity_resolution": lam_c / (2.0 * wf.n_chirps * wf.chirp_period),
    }


def range_axis(wf) -> np.ndarray:
    """Range of each range-FFT bin k: eq. (4) with f_IF = k * fs / M."""
    d = derived(wf)
    return np.arange(wf.n_samples) * d["range_resolution"]


def velocity_axis(wf) -> np.ndarray:
    """Range rate of each Doppler row after the shift: row l holds l' = l - N/2,
    v = l' * lambda_c / (2 N T_c) (eq. (5)); positive = receding."""
    d = derived(wf)
    lp = np.arange(wf.n_chirps) - wf.n_chirps // 2
    return lp * d["velocity_resolution"]


def table2_row(n_samples: int) -> dict:
    """Bandwidth, chirp period, range resolution and max velocity of Table 2 for a
    given number of samples, with fs = 5.12 Msps, slope 12.5 MHz/us, f0 = 77 GHz and a
    10 us idle time per chirp (the experiment setup of Section 4.1)."""
    fs = 5.12e6
    slope = 12.5e12

    class _W:
        pass

    w = _W()
    w.f0, w.slope, w.fs = 77e9, slope, fs
    w.chirp_period = n_samples / fs + 10e-6
    w.n_samples, w.n_chirps = n_samples, 1
    d = derived(w)
    return {"bandwidth": d["bandwidth"], "chirp_period": w.chirp_period,
            "range_resolution": d["range_resolution"],
            "max_velocity": d["max_velocity"], "max_range": d["max_range"]}
