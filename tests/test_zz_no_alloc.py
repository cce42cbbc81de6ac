"""The allocation-free range-Doppler entry point (rsim_form_rdm_noalloc) against
rsim_form_rdm through the C ABI: two calls in a row on one context, the second on a
smaller input, each compared elementwise with the allocating entry point on the same
echo (FP32: the RDM bar of 2e-4 relative RMS, FP64: 1e-12); the first call spans several
groups of planes of the 32 MiB static array, with a ragged last group. Oversized planes
are refused with ERANGE before any launch."""
import sys

import numpy as np
import pytest

import scenes

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_rms(a, b):
    a = np.asarray(a, np.complex128)
    b = np.asarray(b, np.complex128)
    return float(np.sqrt(np.sum(np.abs(a - b) ** 2) / np.sum(np.abs(b) ** 2)))


def _pair(sim, echo, n_cubes, precision):
    import torch
    rdt = torch.float64 if precision else torch.float32
    out = {}
    for name, fn in (("plain", sim.ctx.form_rdm), ("noalloc", sim.ctx.form_rdm_noalloc)):
        rdm = torch.full(echo.shape, -1.0, dtype=rdt, device=echo.device)
        y = torch.zeros_like(echo)
        fn(echo, rdm, y, n_cubes=n_cubes, precision=precision)
        torch.cuda.synchronize()
        out[name] = (rdm.cpu().numpy(), y.cpu().numpy())
    return out


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_rdm_two_calls(precision):
    import torch
    from paper_2208_10939_amd.pipeline import Simulator
    wf = scenes.paper_waveform(256, 128)
    arr = scenes.sparse_mimo_12x16(wf, 3)
    sim = Simulator([scenes.point_scene([20.0], [1.0])], wf, arr)
    dt = torch.complex128 if precision else torch.complex64
    tol = 1e-12 if precision else 2e-4
    rng = np.random.default_rng(11 + precision)
    # call 1: 3 cubes x 192 planes of 256 KiB (FP32) / 512 KiB (FP64) in groups of 127 / 63
    # planes (5 / 10 groups, the last ragged); call 2: one cube (smaller input: 2 / 4 groups)
    for n_cubes in (3, 1):
        _log(f"case noalloc precision={precision} n_cubes={n_cubes} M=256 N=128 O=192")
        shape = (n_cubes, sim.O, wf.n_chirps, wf.n_samples)
        H = rng.normal(size=shape) + 1j * rng.normal(size=shape)
        echo = torch.from_numpy(H).to(dt).cuda()
        out = _pair(sim, echo, n_cubes, precision)
        e_rdm = rel_rms(out["noalloc"][0], out["plain"][0])
        e_y = rel_rms(out["noalloc"][1], out["plain"][1])
        _log(f"  rdm rel_rms={e_rdm:.3e} y rel_rms={e_y:.3e}")
        assert np.all(out["noalloc"][0] >= 0.0)  # every output written
        assert e_rdm <= tol and e_y <= tol


def test_noalloc_rdm_refuses_oversized_plane():
    import torch
    from paper_2208_10939_amd.pipeline import Simulator
    from paper_2208_10939_amd.rsim import RSIM_ERANGE, RsimError
    _log("case noalloc refusal: 2048 x 2048 FP32 plane (32 MiB + twiddles)")
    wf = scenes.paper_waveform(2048, 2048)
    arr = scenes.ula_1tx4rx(wf)
    sim = Simulator([scenes.point_scene([20.0], [1.0])], wf, arr)
    small = torch.zeros(16, dtype=torch.complex64, device="cuda")
    with pytest.raises(RsimError) as ei:
        sim.ctx.form_rdm_noalloc(small, torch.zeros(16, device="cuda"), None, n_cubes=1)
    assert ei.value.code == RSIM_ERANGE
    assert "static work array" in str(ei.value)
