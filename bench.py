"""Benchmark: whole echo-synthesis hot path on one MI355X.

Workload (default, `--workload c3`): the intersection scene, a 60 x 60 m ground grid at
0.25 m (115,200 triangles) plus 20 procedural vehicles of the four classes (car, bus,
truck, motorcycle; ~44k triangles each), 1,000,000 triangles in all, seeded positions
and speeds; 12 Tx x 16 Rx sparse MIMO (192 virtual channels), 512 samples x 256 chirps
(the paper's third waveform), FP32 facet sum with FP64 phase. `--workload c2` runs the
single 50k-triangle vehicle (256 x 128). One step = visibility + compaction + facet sum
+ range FFT + Doppler FFT/RDM of one frame; inputs resident in device memory. Prints
ONE JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload c3|c2] [--no-cpu]
                  [--no-extras] [--calib-copy MiB] [--kernel auto|vector|matrix|nufft]
                  [--tile-m T --tile-f F] [--fwd-bwd-only] [--double-bounce-only]

Extras (unless --no-extras): the two other facet-sum kernels on the same frame, forward +
backward, the same frame with the facet-to-facet double bounce, and batched (persistent +
graph) against plain calls on the 64-scene workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("facet·freq·channel·chirp evals/s + ms per RDM frame; "
          "fwd+bwd vs fwd, batched vs plain")
# Algorithmic work per facet.freq.channel.chirp evaluation: one complex phasor step
# (complex multiply, 6 FLOP) + one complex multiply-accumulate (8 FLOP).
FLOP_PER_EVAL = 14
# What the kernel executes per evaluation: the phasor step as the three-term recurrence
# z_{m+1} = 2 cos(t) z_m - z_{m-1} (2 FMA = 4 FLOP) + the complex MAC (4 FMA = 8 FLOP).
EXECUTED_FLOP_PER_EVAL = 12
# Published FP32 vector peak of MI355X (256 CU x 2.4 GHz; reached with packed FP32).
PEAK_FP32_VECTOR = 157.3e12
# Published dense FP32 matrix-core (MFMA) peak of MI355X.
PEAK_FP32_MFMA = 157.3e12
# What the matrix-core kernel executes per evaluation on the matrix cores: the complex
# multiply-accumulate as four real rank-1 MFMA updates (4 MAC = 8 FLOP); the phasors
# (one per Tx and per Rx element, not per channel) run on the vector units.
MFMA_FLOP_PER_EVAL = 8
# FP32 FMA issue without packed-math instructions, which this build keeps out of all
# device code: 256 CU x 4 SIMD x 16 lanes x 2 FLOP x 2.4 GHz.
PEAK_FP32_NON_PACKED = 256 * 4 * 16 * 2 * 2.4e9
# NUFFT facet sum (type-1 non-uniform FFT over the sample index): every lit (facet or
# point, chirp) record becomes one to three Gaussian grid sources per channel, spread over
# the NUFFT_WIDTH cells within half that width of each source.
NUFFT_WIDTH = 12
# Algorithmic FP32/FP64 FLOP of the spread per (record, channel), by part:
#  * setup, once per (record, channel): the channel's path difference from the record's
#    phase-centre path (two FP64 dot products and the phase in turns, 13), the second-order
#    range corrections, amplitude, phase reduction and grid position (FP32, 35) and the
#    channel's complex factor (cos, sin: 2);
#  * a point source: its complex weight times the channel factor (6), the Gaussian's
#    start value and ratio (8); per cell the Gaussian-weighted complex accumulation
#    (2 FMA, 4) and the Gaussian recurrence (2 multiplies);
#  * a quadratic-weighted source: three complex coefficients times the channel factor
#    (18), the Gaussian start (8); per cell the abscissa (1), the degree-2 complex Horner
#    step (2 x 2 FMA, 8), the accumulation (4) and the recurrence (2).
NUFFT_SETUP_FLOP = 50
NUFFT_POINT_FLOP = 14 + NUFFT_WIDTH * 6
NUFFT_QUAD_FLOP = 26 + NUFFT_WIDTH * 15
# per form of rsim_last_census: none, three points, point + quadratic, one quadratic
NUFFT_FORM_FLOP = {
    "none": 0,
    "three_points": NUFFT_SETUP_FLOP + 3 * NUFFT_POINT_FLOP,
    "point_and_quadratic": NUFFT_SETUP_FLOP + NUFFT_POINT_FLOP + NUFFT_QUAD_FLOP,
    "quadratic": NUFFT_SETUP_FLOP + NUFFT_QUAD_FLOP,
}


def nufft_spread_flop(census, channels):
    """Algorithmic FLOP of the NUFFT spread over one frame: records of each source form
    (the library's census) x channels x the form's FLOP per (record, channel)."""
    return sum(census[k] * channels * NUFFT_FORM_FLOP[k] for k in NUFFT_FORM_FLOP)


PROFILE_TRAFFIC = {"vector": "facet_sum_{w}_traffic.json",
                   "matrix": "facet_sum_mfma_{w}_traffic.json",
                   "nufft": "facet_sum_nufft_{w}_traffic.json"}
KERNEL_SOURCES = {"vector": ("echo.hip", "echo_common.h"),
                  "matrix": ("echo_mfma.hip", "echo_common.h"),
                  "nufft": ("nufft_spread.hip", "nufft_common.h")}
KERNEL_CODES = {"auto": 0, "vector": 1, "matrix": 2, "nufft": 3}


def _c3():
    import scenes
    return scenes.c3()


def _c2():
    import scenes
    return scenes.c2()


WORKLOADS = {
    "c3": ("intersection scene: 0.25 m ground grid (115,200 triangles) + 20 vehicles of 4 "
           "classes, 1,000,000 triangles; 12x16 sparse MIMO (192 ch), 512 samples x 256 "
           "chirps, FP32 sum + FP64 phase", _c3),
    "c2": ("single vehicle hull, 50k triangles, 12x16 sparse MIMO (192 ch), 256 samples x "
           "128 chirps, FP32 sum + FP64 phase", _c2),
}


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def platform_info():
    """GPU name and architecture, HIP runtime and ROCm versions, and the shader clock levels
    the driver lists in sysfs (pp_dpm_sclk, the current one marked '*'; each entry null where
    not available). Read from files: no helper program is started (a child started after
    the GPU is initialised may not exec another program on every host)."""
    import glob
    import torch
    info = {"gpu": None, "arch": None, "hip": getattr(torch.version, "hip", None), "rocm": None,
            "sclk": None}
    try:
        prop = torch.cuda.get_device_properties(0)
        info["gpu"] = prop.name
        info["arch"] = getattr(prop, "gcnArchName", None)
    except Exception:
        pass
    try:
        with open("/opt/rocm/.info/version") as f:
            info["rocm"] = f.read().strip()
    except OSError:
        pass
    for path in sorted(glob.glob("/sys/class/drm/card*/device/pp_dpm_sclk")):
        try:
            with open(path) as f:
                levels = [ln.strip() for ln in f if ln.strip()]
        except OSError:
            continue
        if levels:
            info["sclk"] = levels
            break
    return info


def _src_hash(kernel="vector"):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2208_10939_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(kernel, workload, key=None):
    """HBM bytes of the roofline's unit (direct sums: one facet-sum launch; NUFFT: the
    spread's launches of one frame) from the committed counter summary of this kernel and
    workload, if it was taken on the current kernel source (key: another entry of it)."""
    try:
        with open(os.path.join(ROOT, "profiles", PROFILE_TRAFFIC[kernel].format(w=workload))) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("echo_hip_sha256_16") != _src_hash(kernel):
        return None
    return d.get(key or ("bytes_per_frame" if kernel == "nufft" else "bytes_per_launch"))


def roofline(kernel, evals, fs_ms, shape=None, workload="c3", nufft=None):
    """Roofline object of the facet sum's dominant kernel: algorithmic FLOP per launch
    over the launch's measured duration against the published FP32 peak of the units it
    runs on. Direct sums: FLOP_PER_EVAL per evaluation over the facet-sum launch. NUFFT:
    the spread kernel alone (nufft = {"census", "spread_ms"}: records by source form over
    the frame and the summed event time of the spread's launches in the frame, one per
    chunk of chirps), nufft_spread_flop over that time; weighting each launch by its work
    this is the per-launch figure."""
    rate = evals / (fs_ms * 1e-3)
    achieved = FLOP_PER_EVAL * rate
    if kernel == "nufft":
        O = shape[0]
        census, sp_ms = nufft["census"], nufft["spread_ms"]
        flop = nufft_spread_flop(census, O)
        ach = flop / (sp_ms * 1e-3)
        return {
            "bound": "alu",
            "achieved": ach / 1e12,
            "peak": PEAK_FP32_VECTOR / 1e12,
            "unit": "TFLOP/s",
            "frac": ach / PEAK_FP32_VECTOR,
            "traffic": _traffic("nufft", workload),
            # the same counters resolved by read-request size: FETCH_SIZE's copy-kernel
            # factor of 2 corrects 128-B requests, the spread's reads are 64-B requests
            "traffic_by_request_size": _traffic("nufft", workload,
                                                "bytes_per_frame_by_request_size"),
            "kernel": "rsim::nufft_spread_kernel (type-1 NUFFT spread: each run of "
                      "cell-sorted records adds its Gaussian grid sources into a per-channel "
                      "register window of 32 cells)",
            "spread_ms_per_frame": sp_ms,
            "flop_per_frame": flop,
            "records_by_form": census,
            "flop_per_record_channel": NUFFT_FORM_FLOP,
            "frac_of_non_packed_fp32_peak": ach / PEAK_FP32_NON_PACKED,
            "facet_sum_stage_ms": fs_ms,
            "direct_sum_equivalent_tflops": achieved / 1e12,
        }
    if kernel == "matrix":
        return {
            "bound": "mfma",
            "achieved": achieved / 1e12,
            "peak": PEAK_FP32_MFMA / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_MFMA,
            "traffic": _traffic("matrix", workload),
            "kernel": "rsim::echo_mfma_kernel<3, 4, 16> (FP64 prep + facet integral + "
                      "separable Tx x Rx contraction on v_mfma_f32_4x4x1f32)",
            "flop_per_eval": FLOP_PER_EVAL,
            "evals_per_launch": evals,
            "executed_mfma_flop_per_eval": MFMA_FLOP_PER_EVAL,
            "mfma_utilisation": MFMA_FLOP_PER_EVAL * rate / PEAK_FP32_MFMA,
        }
    return {
        "bound": "alu",
        "achieved": achieved / 1e12,
        "peak": PEAK_FP32_VECTOR / 1e12,
        "unit": "TFLOP/s",
        "frac": achieved / PEAK_FP32_VECTOR,
        "traffic": _traffic("vector", workload),
        "kernel": "rsim::echo_kernel<float> (FP64 prep + facet integral + facet sum)",
        "flop_per_eval": FLOP_PER_EVAL,
        "evals_per_launch": evals,
        "executed_flop_per_eval": EXECUTED_FLOP_PER_EVAL,
        "executed_frac_of_non_packed_fp32_peak":
            EXECUTED_FLOP_PER_EVAL * rate / PEAK_FP32_NON_PACKED,
    }


_CPU_CFG = None  # the workload, shared with forked oracle workers (copy-on-write)


def _cpu_worker(task):
    """One host core: the oracle on chirp n for a seeded sample of facets (visibility)
    and the lit ones among them (facet sum over `channels` x all samples). Returns the
    times of the scene transform alone, of the visibility call and of the sum call."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    import oracle
    n, facets, channels = task
    sc, wf, arr = _CPU_CFG.scenes[0], _CPU_CFG.waveform, _CPU_CFG.array
    with threadpool_limits(1):
        t0 = time.perf_counter()
        oracle.world_triangles(sc, float(n) * wf.chirp_period)
        t_geo = time.perf_counter() - t0
        t0 = time.perf_counter()
        m, _ = oracle.visibility(sc, arr, wf, chirps=[n], facets=facets)
        t_vis = time.perf_counter() - t0
        row = np.zeros(sc.n_tris, bool)
        row[facets[m[0]]] = True
        t0 = time.perf_counter()
        oracle.synthesize(sc, wf, arr, mask={int(n): row}, chirps=[n], channels=channels)
        t_sum = time.perf_counter() - t0
    return t_geo, t_vis, t_sum, int(m[0].sum())


def cpu_baseline(cfg, sample_facets=3000, channels=24, max_workers=16):
    """The FP64 oracle on the host's cores (one forked worker per core, BLAS threads = 1,
    one chirp each): per worker, visibility of a seeded sample of facets and the facet
    sum of the lit ones over `channels` evenly spaced channels x all samples. Whole-frame
    oracle time = chirps x (two scene transforms + all facets' visibility + all lit
    facets' sum over all channels) at the measured per-facet and per-evaluation costs,
    spread over the workers; value = lit-facet evaluations of the frame / that time.
    Must run before the process touches the GPU (the workers are forked)."""
    import multiprocessing as mp
    import numpy as np
    global _CPU_CFG
    _CPU_CFG = cfg
    sc, wf, arr = cfg.scenes[0], cfg.waveform, cfg.array
    F, O, M, N = sc.n_tris, arr.n_channels, wf.n_samples, wf.n_chirps
    workers = max(1, min(os.cpu_count() or 1, max_workers, N))
    rng = np.random.default_rng(cfg.seed + 1000)
    chirps = np.linspace(0, N - 1, workers).astype(int)
    ch = np.linspace(0, O - 1, channels).astype(int)
    tasks = [(int(n), np.sort(rng.choice(F, min(sample_facets, F), replace=False)), ch)
             for n in chirps]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(_cpu_worker, tasks)
    wall = time.perf_counter() - t0
    per_chirp, lit_frac = [], []
    for (t_geo, t_vis, t_sum, lit), (_, fac, _) in zip(res, tasks):
        S = fac.size
        v = max(t_vis - t_geo, 0.0) / S                      # per facet (visibility)
        e = max(t_sum - t_geo, 0.0) / max(1, lit * M * channels)  # per evaluation
        lit_all = F * lit / S
        per_chirp.append(2.0 * t_geo + F * v + lit_all * M * O * e)
        lit_frac.append(lit / S)
    frame_s = N * float(np.mean(per_chirp)) / workers
    evals = N * F * float(np.mean(lit_frac)) * M * O
    return {"value": evals / frame_s, "unit": "evals/s", "cores": workers, "kind": "oracle",
            "sample": (f"{workers} forked workers (numpy float64, BLAS threads 1), one chirp "
                       f"each ({', '.join(str(int(n)) for n in chirps)}): visibility of "
                       f"{tasks[0][1].size} seeded facets of {F}, facet sum of the lit ones "
                       f"over {channels} of {O} channels x {M} samples; scaled to the whole "
                       f"frame ({N} chirps, all facets and channels) on {workers} cores: "
                       f"{frame_s:.0f} s per frame; sample wall time {wall:.1f} s"),
            "host_cpus": os.cpu_count()}


def measure_fwd_bwd(sim, kernel, reps=2):
    """Forward (echo + RDM, the given facet-sum kernel) and forward + backward (RDM adjoint +
    facet-sum adjoint, the library's default for the scene + vertex/velocity gather) for the
    loss sum (RDM - T)^2 with a fixed target T."""
    import numpy as np
    import torch
    echo = sim.echo_buffer(1)
    mask = sim.mask_buffer()
    rdm = torch.empty(echo.shape, dtype=torch.float32, device="cuda")
    y = torch.empty_like(echo)
    sid = sim.scene_ids[0]
    kc = KERNEL_CODES[kernel]
    sim.ctx.synthesize([sid], echo, mask, kernel=kc)
    sim.ctx.form_rdm(echo, rdm, y)
    target = (0.5 * rdm).contiguous()
    ge = torch.empty_like(echo)
    meshes = sim.ctx.scene_meshes[sid]
    gv = [None] * (max(meshes) + 1)
    for mid in meshes:
        nv = sim.ctx.mesh_nverts[mid]
        gv[mid] = torch.zeros((nv, 3), dtype=torch.float32, device="cuda")
    gvel = torch.zeros((len(sim.inst_pos0[0]), 3), dtype=torch.float64, device="cuda")
    fwd, tot, stages = [], [], None
    for _ in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.ctx.synthesize([sid], echo, mask, timing=True, kernel=kc)
        sim.ctx.form_rdm(echo, rdm, y, timing=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        grad = (2.0 * (rdm - target)).contiguous()
        sim.ctx.rdm_backward(grad, y, ge)
        sim.ctx.backward(sid, ge, mask, gv, gvel)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        stages = sim.ctx.last_timings()
        fwd.append(t1 - t0)
        tot.append(t2 - t0)
    fwd_ms = 1e3 * float(np.median(fwd[1:]))
    tot_ms = 1e3 * float(np.median(tot[1:]))
    return {"fwd_ms": fwd_ms, "fwd_bwd_ms": tot_ms, "ratio": tot_ms / fwd_ms,
            "stage_ms": {k: round(v, 4) for k, v in stages.items()}}


def measure_other_kernel(sim, echo, mask, kernel, evals, workload, reps=2):
    """Facet-sum time and roofline of the kernel the autotuner did not pick, on the same
    frame (median of `reps` launches after one warm-up; results compared with the main
    kernel's to the FP32 bar)."""
    import numpy as np
    import torch
    ref = echo.clone()
    kc = KERNEL_CODES[kernel]
    buf = torch.empty_like(echo)
    sim.ctx.synthesize([sim.scene_ids[0]], buf, mask, kernel=kc)
    ts, sp = [], []
    for _ in range(reps):
        sim.ctx.synthesize([sim.scene_ids[0]], buf, mask, timing=True, kernel=kc)
        t = sim.ctx.last_timings()
        ts.append(t["facet_sum"])
        sp.append(t["nufft_spread"])
    torch.cuda.synchronize()
    fs = float(np.median(ts))
    nu = nufft_info(sim, mask, float(np.median(sp))) if kernel == "nufft" else None
    d = (buf - ref).abs().pow(2).sum().sqrt() / ref.abs().pow(2).sum().sqrt()
    wf = sim.wf
    return {"kernel": kernel, "facet_sum_ms": fs,
            "roofline": roofline(kernel, evals, fs, (sim.O, wf.n_chirps, wf.n_samples), workload,
                                 nu),
            "rel_rms_vs_main": float(d)}


def nufft_info(sim, mask, spread_ms):
    """The NUFFT roofline's inputs: the record census of one untimed NUFFT call on the same
    frame (visibility mask as given) and the spread's measured time."""
    echo = sim.echo_buffer(1)
    sim.ctx.synthesize([sim.scene_ids[0]], echo, mask, mask_mode=1, kernel=KERNEL_CODES["nufft"],
                       census=True)
    return {"census": sim.ctx.last_census(), "spread_ms": spread_ms}


def measure_batched(n_scenes=64, reps=2, kernels=("matrix", "nufft")):
    """The batched workload (64 scenes, seeds 400..463, 10k-400k triangles each): for each
    kernel, one call over all scenes with the persistent launch under a captured graph
    against one plain call per scene, timed end to end (visibility, compaction, facet
    sum); the two results are compared bit for bit. A kernel the scenes make ineligible
    is reported as such."""
    import numpy as np
    import torch
    import scenes
    from paper_2208_10939_amd.pipeline import Simulator
    from paper_2208_10939_amd.rsim import RsimError
    cfg = scenes.c4(n_scenes=n_scenes)
    sim = Simulator(cfg.scenes, cfg.waveform, cfg.array)
    n = len(cfg.scenes)
    plain = sim.echo_buffer(n)
    batched = sim.echo_buffer(n)
    mask = sim.mask_buffer()
    out = {"scenes": n, "triangles": int(sum(s.n_tris for s in cfg.scenes)), "legs": []}
    evals = None
    for kernel in kernels:
        kc = KERNEL_CODES[kernel]

        def run_plain():
            for i in range(n):
                sim.ctx.synthesize([sim.scene_ids[i]], plain[i:i + 1], None, kernel=kc)

        def run_batched():
            sim.ctx.synthesize(sim.scene_ids, batched, mask, persistent=True, use_graph=True,
                               kernel=kc)

        leg = {"kernel": kernel}
        try:
            times = {}
            for name, fn in (("plain", run_plain), ("batched", run_batched)):
                fn()
                torch.cuda.synchronize()
                ts = []
                for _ in range(reps):
                    t0 = time.perf_counter()
                    fn()
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t0)
                times[name] = 1e3 * float(np.median(ts))
        except RsimError as e:
            leg["note"] = f"not run: {e}"
            out["legs"].append(leg)
            continue
        if evals is None:
            lit = sum(int(m.sum()) for m in sim.masks_numpy(mask))
            evals = lit * cfg.waveform.n_samples * cfg.array.n_channels
        diff = float((plain - batched).abs().pow(2).sum().sqrt() / plain.abs().pow(2).sum().sqrt())
        leg.update({"plain_ms": times["plain"], "batched_ms": times["batched"],
                    "plain_evals_per_s": evals / (times["plain"] * 1e-3),
                    "batched_evals_per_s": evals / (times["batched"] * 1e-3),
                    "bit_identical": bool(torch.equal(plain, batched)),
                    "rel_rms_difference": diff})
        _log(f"bench: batched {kernel}: plain {times['plain']:.1f} ms, batched "
             f"{times['batched']:.1f} ms, bit-identical {leg['bit_identical']}")
        out["legs"].append(leg)
    return out


def measure_double_bounce(sim, lit_per_step, reps=2):
    """The same frame with the facet-to-facet double bounce on (NUFFT facet sum): frame
    time with its stages (the connection search runs in the compaction stage), the number
    of connections (census records beyond the lit facets), and the time of rsim_backward
    for the loss sum RDM^2 through that echo (NUFFT adjoint, connection table held)."""
    import numpy as np
    import torch
    sim.set_double_bounce(True, -1.0)
    try:
        echo = sim.echo_buffer(1)
        mask = sim.mask_buffer()
        rdm = torch.empty(echo.shape, dtype=torch.float32, device="cuda")
        sid = sim.scene_ids[0]
        sim.ctx.synthesize([sid], echo, mask)
        ts, st = [], []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.ctx.synthesize([sid], echo, mask, timing=True)
            sim.ctx.form_rdm(echo, rdm, None, n_cubes=1, timing=True)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
            st.append(sim.ctx.last_timings())
        sim.ctx.synthesize([sid], echo, mask, mask_mode=1, census=True)
        records = sum(sim.ctx.last_census().values())
        # the backward of sum RDM^2 through this echo (NUFFT adjoint, connections held)
        y = torch.empty_like(echo)
        sim.ctx.form_rdm(echo, rdm, y, n_cubes=1)
        ge = torch.empty_like(echo)
        sim.ctx.rdm_backward((2.0 * rdm).contiguous(), y, ge)
        meshes = sim.ctx.scene_meshes[sid]
        gv = [None] * (max(meshes) + 1)
        for mid in meshes:
            gv[mid] = torch.zeros((sim.ctx.mesh_nverts[mid], 3), dtype=torch.float32,
                                  device="cuda")
        gvel = torch.zeros((len(sim.inst_pos0[0]), 3), dtype=torch.float64, device="cuda")
        bs = []
        for _ in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.ctx.backward(sid, ge, mask, gv, gvel)
            torch.cuda.synchronize()
            bs.append(time.perf_counter() - t0)
        i = int(np.argmin(ts))
        return {"ms_per_frame": 1e3 * float(np.median(ts)),
                "stage_ms": {k: round(v, 4) for k, v in st[i].items()},
                "backward_ms": 1e3 * float(np.median(bs[1:])),
                "connections_per_frame": int(records - lit_per_step),
                "lit_facet_records_per_frame": int(lit_per_step)}
    finally:
        sim.set_double_bounce(False)


def measure_intra_chirp(sim, echo_ref, reps=2):
    """The same frame with the delay within the chirp (rsim_opts.intra_chirp = 1, the
    default facet-sum kernel): frame time with its stages, and the echo's relative RMS
    difference from the stop-and-hop echo echo_ref (the range-Doppler coupling)."""
    import numpy as np
    import torch
    echo = sim.echo_buffer(1)
    mask = sim.mask_buffer()
    rdm = torch.empty(echo.shape, dtype=torch.float32, device="cuda")
    sid = sim.scene_ids[0]
    sim.ctx.synthesize([sid], echo, mask, intra_chirp=1)
    ts, st = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.ctx.synthesize([sid], echo, mask, timing=True, intra_chirp=1)
        sim.ctx.form_rdm(echo, rdm, None, n_cubes=1, timing=True)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
        st.append(sim.ctx.last_timings())
    sim.ctx.synthesize([sid], echo, mask, intra_chirp=1)
    d = float(torch.linalg.vector_norm(echo - echo_ref) / torch.linalg.vector_norm(echo_ref))
    i = int(np.argmin(ts))
    return {"ms_per_frame": 1e3 * float(np.median(ts)),
            "stage_ms": {k: round(v, 4) for k, v in st[i].items()},
            "rel_rms_vs_stop_and_hop": d}


def calib_copy(mib: int):
    """Plain elementwise copy of known size, for scaling FETCH_SIZE / WRITE_SIZE."""
    import torch
    n = mib * 1024 * 1024 // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.add(x, 0.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_mib": mib, "bytes_read": n * 4, "bytes_written": n * 4}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the forward+backward and batched-vs-plain measurements")
    ap.add_argument("--calib-copy", type=int, default=0, metavar="MIB")
    ap.add_argument("--fwd-bwd-only", action="store_true",
                    help="only the forward + backward timing (for kernel traces of the adjoint)")
    ap.add_argument("--double-bounce-only", action="store_true",
                    help="only the frame with the facet-to-facet double bounce")
    ap.add_argument("--tile-m", type=int, default=0)
    ap.add_argument("--tile-f", type=int, default=0)
    ap.add_argument("--workload", choices=tuple(WORKLOADS), default="c3",
                    help="c3: 1M-triangle intersection, 512 x 256 (default); c2: 50k-triangle "
                         "vehicle, 256 x 128")
    ap.add_argument("--kernel", choices=("auto", "vector", "matrix", "nufft"), default="auto",
                    help="facet-sum kernel (auto: the autotuner's choice)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(sharding over chirps is a design note only)", file=sys.stderr)
        sys.exit(2)
    if args.calib_copy:
        calib_copy(args.calib_copy)
        return

    import numpy as np

    import scenes

    desc, make = WORKLOADS[args.workload]
    cfg = make()
    sc, wf, arr = cfg.scenes[0], cfg.waveform, cfg.array
    _log(f"bench: {args.workload} workload, {sc.n_tris} triangles, O={arr.n_channels}, "
         f"M={wf.n_samples}, N={wf.n_chirps}")
    cpu = None
    if not args.no_cpu:
        # the oracle's workers are forked: before anything touches the GPU
        _log("bench: timing the FP64 oracle on the host cores (bounded sample)")
        cpu = cpu_baseline(cfg)
        _log(f"bench: oracle {cpu['value']:.3e} evals/s on {cpu['cores']} cores")

    import torch
    from paper_2208_10939_amd.pipeline import Simulator

    torch.cuda.set_device(0)
    sim = Simulator([sc], wf, arr)
    echo = sim.echo_buffer(1)
    mask = sim.mask_buffer()
    rdm = torch.empty(echo.shape, dtype=torch.float32, device="cuda")
    kw = dict(tile_m=args.tile_m, tile_f=args.tile_f, kernel=KERNEL_CODES[args.kernel])

    def step(timing):
        sim.ctx.synthesize([sim.scene_ids[0]], echo, mask, timing=timing, **kw)
        sim.ctx.form_rdm(echo, rdm, None, n_cubes=1, timing=timing)

    tuned = None
    if not (args.tile_m or args.tile_f) and args.kernel == "auto":
        # tile shapes from the library's autotuner, timed on this workload
        import tempfile
        fd, tune_path = tempfile.mkstemp(suffix=".jsonl")
        os.close(fd)
        sim.ctx.autotune([sim.scene_ids[0]], tune_path)
        with open(tune_path) as f:
            tuned = json.loads(f.read().strip().splitlines()[-1])
        os.remove(tune_path)
        _log(f"bench: autotuned facet-sum kernel {tuned['kernel']}, vector tile "
             f"{tuned['tile_m']} x {tuned['tile_f']}")
    kernel = (tuned["kernel"] if tuned else
              ("vector" if args.kernel == "auto" else args.kernel))
    if args.fwd_bwd_only:
        print(json.dumps({"facet_sum_kernel": kernel, "fwd_bwd": measure_fwd_bwd(sim, kernel)}))
        return
    if args.double_bounce_only:
        step(False)
        torch.cuda.synchronize()
        lit0 = int(sim.masks_numpy(mask)[0].sum())
        print(json.dumps({"double_bounce": measure_double_bounce(sim, lit0)}))
        return
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()

    names = None
    stage_ms = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(True)
        t = sim.ctx.last_timings()  # waits for this step's events
        if stage_ms is None:
            names, stage_ms = list(t.keys()), np.zeros(len(t))
        stage_ms += np.array(list(t.values()))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / args.steps
    # the frame's lit facets (the same every step: the scene and chirp times are fixed)
    lit = sim.masks_numpy(mask)[0].sum(axis=1)
    evals_per_step = int(lit.sum()) * wf.n_samples * arr.n_channels
    _log(f"bench: lit facets per chirp mean {lit.mean():.0f}, evals/step {evals_per_step:.3e}")
    stage_avg = {n: round(float(v / args.steps), 4) for n, v in zip(names, stage_ms)}
    fs_ms = stage_ms[names.index("facet_sum")] / args.steps
    achieved = FLOP_PER_EVAL * evals_per_step / (fs_ms * 1e-3)
    nu = None
    if kernel == "nufft":
        nu = nufft_info(sim, mask, stage_ms[names.index("nufft_spread")] / args.steps)
    rl = roofline(kernel, evals_per_step, fs_ms, (arr.n_channels, wf.n_chirps, wf.n_samples),
                  args.workload, nu)
    _log(f"bench: {ms_per_step:.2f} ms/step, facet sum {fs_ms:.2f} ms "
         f"({achieved / 1e12:.2f} TFLOP/s direct-sum-equivalent); {kernel} kernel "
         f"{'(spread) ' if kernel == 'nufft' else ''}at {rl['achieved']:.2f} {rl['unit']} of "
         f"its own work = {rl['frac']:.3f} of peak")

    out = {
        "metric": METRIC,
        "value": evals_per_step * args.steps / wall,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc,
                   "triangles": int(sc.n_tris), "channels": int(arr.n_channels),
                   "samples": int(wf.n_samples), "chirps": int(wf.n_chirps),
                   "lit_facets_per_chirp": float(lit.mean()), "seed": cfg.seed,
                   "facet_sum_kernel": kernel,
                   "facet_sum_tile": (tuned if tuned else
                                      {"tile_m": args.tile_m, "tile_f": args.tile_f}),
                   # every facet of every chirp, lit or not: F M O N
                   "nominal_evals_per_step": int(sc.n_tris) * wf.n_samples * arr.n_channels *
                                             wf.n_chirps},
        "stage_ms": stage_avg,
        "roofline": rl,
        "platform": platform_info(),
    }
    if not args.no_extras:
        out["other_kernels"] = []
        for other in ("nufft", "matrix", "vector"):
            if other == kernel:
                continue
            _log(f"bench: the {other} kernel's facet sum on the same frame")
            out["other_kernels"].append(
                measure_other_kernel(sim, echo, mask, other, evals_per_step, args.workload))
        _log("bench: forward + backward")
        out["fwd_bwd"] = measure_fwd_bwd(sim, kernel)
        _log("bench: the facet-to-facet double bounce on the same frame")
        out["double_bounce"] = measure_double_bounce(sim, int(lit.sum()))
        _log("bench: the delay within the chirp on the same frame")
        out["intra_chirp"] = measure_intra_chirp(sim, echo)
        _log("bench: batched vs plain (the 64-scene workload)")
        out["batched_vs_plain"] = measure_batched()
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
