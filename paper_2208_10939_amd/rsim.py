"""ctypes binding of librsim (argument marshalling only; every step runs in the HIP
library). Names follow include/rsim.h. Device buffers are torch tensors on the GPU;
streams are torch streams. The binding refuses to run without the built library.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librsim.so")

RSIM_OK = 0
RSIM_EINVAL = -1
RSIM_ENOMEM = -2
RSIM_EDEVICE = -3
RSIM_ESTATE = -4
RSIM_ERANGE = -5
RSIM_FP32_PHASE64 = 0
RSIM_FP64 = 1
RSIM_MASK_COMPUTE = 0
RSIM_MASK_INPUT = 1
RSIM_KERNEL_AUTO = 0
RSIM_KERNEL_VECTOR = 1
RSIM_KERNEL_MATRIX = 2
RSIM_KERNEL_NUFFT = 3
ABI_VERSION = 2
CENSUS_FORMS = ("none", "three_points", "point_and_quadratic", "quadratic")
N_STAGES = 10
STAGES = ("visibility", "compaction", "facet_sum", "range_fft", "doppler_rdm",
          "adjoint_facet_sum", "adjoint_fft", "vertex_gather", "nufft_spread", "nufft_gather")

EXPORTS = (
    "rsim_abi_version", "rsim_create", "rsim_destroy", "rsim_last_error", "rsim_set_mem_limit",
    "rsim_load_mesh", "rsim_create_scene", "rsim_add_instance", "rsim_add_points",
    "rsim_scene_info", "rsim_set_waveform", "rsim_set_array", "rsim_synthesize",
    "rsim_form_rdm", "rsim_last_timings", "rsim_last_census", "rsim_set_double_bounce",
    "rsim_backward", "rsim_rdm_adjoint",
    "rsim_autotune", "rsim_sync", "rsim_update_mesh", "rsim_set_instance_motion",
    "rsim_rdm_backward", "rsim_detect", "rsim_add_noise", "rsim_set_ground",
    "rsim_set_backward_kernel", "rsim_set_backward_intra_chirp", "rsim_set_nufft_chunk",
    "rsim_form_rdm_noalloc",
)


class RsimError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"rsim error {code}: {msg}")
        self.code = code


class Waveform(ctypes.Structure):
    _fields_ = [("f0_hz", ctypes.c_double), ("slope_hz_per_s", ctypes.c_double),
                ("fs_hz", ctypes.c_double), ("chirp_period_s", ctypes.c_double),
                ("n_samples", ctypes.c_int32), ("n_chirps", ctypes.c_int32)]


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("mask_mode", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("timing", ctypes.c_int32), ("tile_m", ctypes.c_int32),
                ("tile_f", ctypes.c_int32), ("intra_chirp", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("census", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


class CfarOpts(ctypes.Structure):
    _fields_ = [("guard_doppler", ctypes.c_int32), ("guard_range", ctypes.c_int32),
                ("train_doppler", ctypes.c_int32), ("train_range", ctypes.c_int32),
                ("scale", ctypes.c_float), ("na_x", ctypes.c_int32), ("na_z", ctypes.c_int32),
                ("max_points", ctypes.c_int32)]


class Point(ctypes.Structure):
    _fields_ = [("row", ctypes.c_int32), ("bin", ctypes.c_int32), ("power", ctypes.c_float),
                ("noise", ctypes.c_float), ("range_m", ctypes.c_float),
                ("velocity_mps", ctypes.c_float), ("u", ctypes.c_float), ("w", ctypes.c_float),
                ("x", ctypes.c_float), ("y", ctypes.c_float), ("z", ctypes.c_float),
                ("angle_power", ctypes.c_float), ("kx", ctypes.c_int32), ("kz", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


# numpy view of an array of Point records (64 bytes each)
POINT_DTYPE = np.dtype([("row", "<i4"), ("bin", "<i4"), ("power", "<f4"), ("noise", "<f4"),
                        ("range_m", "<f4"), ("velocity_mps", "<f4"), ("u", "<f4"), ("w", "<f4"),
                        ("x", "<f4"), ("y", "<f4"), ("z", "<f4"), ("angle_power", "<f4"),
                        ("kx", "<i4"), ("kz", "<i4"), ("reserved", "<i4", (2,))])

_lib = None


def lib() -> ctypes.CDLL:
    """Load librsim.so (built in-tree by paper_2208_10939_amd.build); fails loudly."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2208_10939_amd.build` (there is no fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "rsim_abi_version": ([], i32),
        "rsim_create": ([i32, ctypes.POINTER(vp)], i32),
        "rsim_destroy": ([vp], None),
        "rsim_last_error": ([vp], ctypes.c_char_p),
        "rsim_set_mem_limit": ([vp, u64], i32),
        "rsim_load_mesh": ([vp, vp, i64, vp, i64, ctypes.POINTER(i32)], i32),
        "rsim_create_scene": ([vp, ctypes.POINTER(i32)], i32),
        "rsim_add_instance": ([vp, i32, i32, dp, dp, dp, ctypes.POINTER(i32)], i32),
        "rsim_add_points": ([vp, i32, dp, dp, dp, i64], i32),
        "rsim_scene_info": ([vp, i32, ctypes.POINTER(i64), ctypes.POINTER(i64)], i32),
        "rsim_set_waveform": ([vp, ctypes.POINTER(Waveform)], i32),
        "rsim_set_array": ([vp, dp, i32, dp, i32], i32),
        "rsim_synthesize": ([vp, ctypes.POINTER(i32), i32, vp, vp, vp, ctypes.POINTER(Opts)], i32),
        "rsim_form_rdm": ([vp, vp, i32, vp, vp, vp, ctypes.POINTER(Opts)], i32),
        "rsim_last_timings": ([vp, ctypes.POINTER(ctypes.c_float), i32], i32),
        "rsim_last_census": ([vp, ctypes.POINTER(ctypes.c_int64)], i32),
        "rsim_set_double_bounce": ([vp, i32, ctypes.c_double, ctypes.c_double], i32),
        "rsim_backward": ([vp, i32, vp, vp, ctypes.POINTER(vp), i32, vp, vp], i32),
        "rsim_rdm_adjoint": ([vp, vp, i32, vp, vp], i32),
        "rsim_autotune": ([vp, ctypes.POINTER(i32), i32, ctypes.c_char_p], i32),
        "rsim_sync": ([vp, vp], i32),
        "rsim_update_mesh": ([vp, i32, vp, i64], i32),
        "rsim_set_instance_motion": ([vp, i32, i32, dp, dp], i32),
        "rsim_rdm_backward": ([vp, vp, vp, i32, vp, vp], i32),
        "rsim_detect": ([vp, vp, vp, i32, ctypes.POINTER(CfarOpts), vp, vp, vp, vp, vp], i32),
        "rsim_add_noise": ([vp, vp, i32, ctypes.c_double, u64, vp, ctypes.POINTER(Opts)], i32),
        "rsim_set_ground": ([vp, i32, ctypes.c_double, ctypes.c_double, ctypes.c_double], i32),
        "rsim_set_backward_kernel": ([vp, i32], i32),
        "rsim_set_backward_intra_chirp": ([vp, i32], i32),
        "rsim_set_nufft_chunk": ([vp, i32], i32),
        "rsim_form_rdm_noalloc": ([vp, vp, i32, vp, vp, vp, ctypes.POINTER(Opts)], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    if L.rsim_abi_version() != ABI_VERSION:
        raise RuntimeError(f"{LIB_PATH} has ABI version {L.rsim_abi_version()}, the binding "
                           f"expects {ABI_VERSION}: rebuild it")
    _lib = L
    return L


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ptr(t) -> Optional[int]:
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Context:
    """One librsim context on one HIP device (device=-1: host-only, validation only)."""

    def __init__(self, device: int = 0):
        self._L = lib()
        h = ctypes.c_void_p()
        rc = self._L.rsim_create(int(device), ctypes.byref(h))
        if rc != RSIM_OK:
            raise RsimError(rc, self._L.rsim_last_error(None).decode())
        self._h = h
        self.device = device
        self.n_tx = self.n_rx = 0
        self.waveform = None

    def close(self):
        if getattr(self, "_h", None):
            self._L.rsim_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int):
        if rc != RSIM_OK:
            raise RsimError(rc, self._L.rsim_last_error(self._h).decode())

    # ---- scene -------------------------------------------------------------------
    def set_mem_limit(self, nbytes: int):
        self._check(self._L.rsim_set_mem_limit(self._h, int(nbytes)))

    def load_mesh(self, verts, tris) -> int:
        v = np.ascontiguousarray(verts, dtype=np.float32)
        t = np.ascontiguousarray(tris, dtype=np.int32)
        out = ctypes.c_int32()
        self._check(self._L.rsim_load_mesh(self._h, v.ctypes.data, v.shape[0], t.ctypes.data,
                                           t.shape[0], ctypes.byref(out)))
        if not hasattr(self, "mesh_nverts"):
            self.mesh_nverts = {}
        self.mesh_nverts[out.value] = v.shape[0]
        return out.value

    def create_scene(self) -> int:
        out = ctypes.c_int32()
        self._check(self._L.rsim_create_scene(self._h, ctypes.byref(out)))
        return out.value

    def add_instance(self, scene: int, mesh: int, rot, pos0, vel) -> int:
        r = np.ascontiguousarray(rot, np.float64).reshape(9)
        p = np.ascontiguousarray(pos0, np.float64).reshape(3)
        v = np.ascontiguousarray(vel, np.float64).reshape(3)
        out = ctypes.c_int32()
        self._check(self._L.rsim_add_instance(self._h, scene, mesh, _dptr(r), _dptr(p), _dptr(v),
                                              ctypes.byref(out)))
        return out.value

    def add_points(self, scene: int, pos0, vel, amp):
        p = np.ascontiguousarray(pos0, np.float64).reshape(-1, 3)
        v = np.ascontiguousarray(vel, np.float64).reshape(-1, 3)
        a = np.asarray(amp, np.complex128).reshape(-1)
        ari = np.ascontiguousarray(np.stack([a.real, a.imag], 1))
        self._check(self._L.rsim_add_points(self._h, scene, _dptr(p), _dptr(v), _dptr(ari),
                                            p.shape[0]))

    def update_mesh(self, mesh: int, verts):
        v = np.ascontiguousarray(verts, dtype=np.float32)
        self._check(self._L.rsim_update_mesh(self._h, int(mesh), v.ctypes.data, v.shape[0]))

    def set_instance_motion(self, scene: int, inst: int, pos0, vel):
        p = np.ascontiguousarray(pos0, np.float64).reshape(3)
        v = np.ascontiguousarray(vel, np.float64).reshape(3)
        self._check(self._L.rsim_set_instance_motion(self._h, int(scene), int(inst), _dptr(p),
                                                     _dptr(v)))

    def scene_info(self, scene: int):
        nf, nw = ctypes.c_int64(), ctypes.c_int64()
        self._check(self._L.rsim_scene_info(self._h, scene, ctypes.byref(nf), ctypes.byref(nw)))
        return nf.value, nw.value

    def load_scene(self, scene) -> int:
        """Load an object with .meshes (verts, tris), .instances (mesh, rot, pos0, vel)
        and optional .points (pos0, vel, amp); returns the scene id."""
        mesh_ids = [self.load_mesh(m.verts, m.tris) for m in scene.meshes]
        sid = self.create_scene()
        for inst in scene.instances:
            self.add_instance(sid, mesh_ids[inst.mesh], inst.rot, inst.pos0, inst.vel)
        if getattr(scene, "points", None) is not None and scene.points.n:
            self.add_points(sid, scene.points.pos0, scene.points.vel, scene.points.amp)
        if not hasattr(self, "scene_meshes"):
            self.scene_meshes = {}
        self.scene_meshes[sid] = mesh_ids
        return sid

    # ---- radar -------------------------------------------------------------------
    def set_waveform(self, wf):
        w = Waveform(wf.f0, wf.slope, wf.fs, wf.chirp_period, wf.n_samples, wf.n_chirps)
        self._check(self._L.rsim_set_waveform(self._h, ctypes.byref(w)))
        self.waveform = wf

    def set_array(self, tx, rx):
        t = np.ascontiguousarray(tx, np.float64).reshape(-1, 3)
        r = np.ascontiguousarray(rx, np.float64).reshape(-1, 3)
        self._check(self._L.rsim_set_array(self._h, _dptr(t), t.shape[0], _dptr(r), r.shape[0]))
        self.n_tx, self.n_rx = t.shape[0], r.shape[0]

    def set_ground(self, enable: bool, z_ground: float = 0.0, gamma: complex = -1.0):
        g = complex(gamma)
        self._check(self._L.rsim_set_ground(self._h, int(bool(enable)), float(z_ground), g.real,
                                            g.imag))

    def set_double_bounce(self, enable: bool, gamma: complex = -1.0):
        g = complex(gamma)
        self._check(self._L.rsim_set_double_bounce(self._h, int(bool(enable)), g.real, g.imag))

    def set_backward_kernel(self, kernel: int = RSIM_KERNEL_AUTO):
        self._check(self._L.rsim_set_backward_kernel(self._h, int(kernel)))

    def set_backward_intra_chirp(self, enable: bool):
        self._check(self._L.rsim_set_backward_intra_chirp(self._h, int(bool(enable))))

    def set_nufft_chunk(self, max_chirps: int = 0):
        self._check(self._L.rsim_set_nufft_chunk(self._h, int(max_chirps)))

    @property
    def n_channels(self) -> int:
        return self.n_tx * self.n_rx

    # ---- echo / RDM --------------------------------------------------------------
    @staticmethod
    def opts(precision=RSIM_FP32_PHASE64, mask_mode=RSIM_MASK_COMPUTE, use_graph=False,
             persistent=False, timing=False, tile_m=0, tile_f=0, intra_chirp=False,
             kernel=RSIM_KERNEL_AUTO, census=False) -> Opts:
        return Opts(int(precision), int(mask_mode), int(bool(use_graph)), int(bool(persistent)),
                    int(bool(timing)), int(tile_m), int(tile_f), int(bool(intra_chirp)),
                    int(kernel), int(bool(census)))

    def synthesize(self, scene_ids: Sequence[int], echo, mask=None, stream=None, **kw):
        ids = (ctypes.c_int32 * len(scene_ids))(*[int(s) for s in scene_ids])
        o = self.opts(**kw)
        self._check(self._L.rsim_synthesize(self._h, ids, len(scene_ids), _ptr(echo), _ptr(mask),
                                             _stream(stream), ctypes.byref(o)))

    def form_rdm(self, echo, rdm=None, y=None, n_cubes: int = 1, stream=None, **kw):
        o = self.opts(**kw)
        self._check(self._L.rsim_form_rdm(self._h, _ptr(echo), int(n_cubes), _ptr(rdm), _ptr(y),
                                           _stream(stream), ctypes.byref(o)))

    def form_rdm_noalloc(self, echo, rdm=None, y=None, n_cubes: int = 1, stream=None, **kw):
        """rsim_form_rdm_noalloc: form_rdm with its work memory in the library's static
        per-GPU array (no device allocation)."""
        o = self.opts(**kw)
        self._check(self._L.rsim_form_rdm_noalloc(self._h, _ptr(echo), int(n_cubes), _ptr(rdm),
                                                  _ptr(y), _stream(stream), ctypes.byref(o)))

    def rdm_adjoint(self, grad_y, grad_echo, n_cubes: int = 1, stream=None):
        self._check(self._L.rsim_rdm_adjoint(self._h, _ptr(grad_y), int(n_cubes),
                                              _ptr(grad_echo), _stream(stream)))

    def rdm_backward(self, grad_rdm, y, grad_echo, n_cubes: int = 1, stream=None):
        self._check(self._L.rsim_rdm_backward(self._h, _ptr(grad_rdm), _ptr(y), int(n_cubes),
                                              _ptr(grad_echo), _stream(stream)))

    def backward(self, scene: int, grad_echo, mask, grad_verts: Sequence, grad_vel, stream=None):
        arr = (ctypes.c_void_p * max(1, len(grad_verts)))(*[_ptr(g) for g in grad_verts])
        self._check(self._L.rsim_backward(self._h, int(scene), _ptr(grad_echo), _ptr(mask), arr,
                                          len(grad_verts), _ptr(grad_vel), _stream(stream)))

    def detect(self, rdm, y, points, n_points, n_cubes: int = 1, det_mask=None, noise_map=None,
               guard=(1, 1), train=(2, 4), scale: float = 10.0, na_x: int = 0, na_z: int = 0,
               stream=None):
        """CA-CFAR + angle FFT into `points` (uint8 device tensor of n_cubes x max_points
        x 64 bytes) and `n_points` (int32 device tensor [n_cubes])."""
        max_points = points.numel() // (64 * int(n_cubes))
        o = CfarOpts(int(guard[0]), int(guard[1]), int(train[0]), int(train[1]), float(scale),
                     int(na_x), int(na_z), int(max_points))
        self._check(self._L.rsim_detect(self._h, _ptr(rdm), _ptr(y), int(n_cubes), ctypes.byref(o),
                                        _ptr(det_mask), _ptr(noise_map), _ptr(points),
                                        _ptr(n_points), _stream(stream)))

    def add_noise(self, echo, snr_db: float, seed: int, n_cubes: int = 1, stream=None, **kw):
        o = self.opts(**kw)
        self._check(self._L.rsim_add_noise(self._h, _ptr(echo), int(n_cubes), float(snr_db),
                                           int(seed) & 0xFFFFFFFFFFFFFFFF, _stream(stream),
                                           ctypes.byref(o)))

    def last_timings(self) -> dict:
        buf = (ctypes.c_float * N_STAGES)()
        self._check(self._L.rsim_last_timings(self._h, buf, N_STAGES))
        return {name: float(buf[i]) for i, name in enumerate(STAGES)}

    def last_census(self) -> dict:
        """Record counts by source form of the last NUFFT call made with census=1."""
        buf = (ctypes.c_int64 * 4)()
        self._check(self._L.rsim_last_census(self._h, buf))
        return {name: int(buf[i]) for i, name in enumerate(CENSUS_FORMS)}

    def autotune(self, scene_ids: Sequence[int], cache_path: Optional[str] = None):
        ids = (ctypes.c_int32 * len(scene_ids))(*[int(s) for s in scene_ids])
        self._check(self._L.rsim_autotune(self._h, ids, len(scene_ids),
                                          cache_path.encode() if cache_path else None))

    def sync(self, stream=None):
        self._check(self._L.rsim_sync(self._h, _stream(stream)))
