"""Named synthetic workloads (seeded). Sizes follow the five benchmark workloads:

  c1   one box "car" 4.5x1.8x1.5 m, 1000 triangles, 20 m, 10 m/s approaching;
       77-81 GHz in 128 samples, 1 Tx x 4 Rx ULA, 32 chirps (FP64 path)
  c1p  c1 with the paper's experiment-1 waveform slope (readable RDM)
  c2   one procedural hull, 50k triangles, 10-60 m, +-15 m/s; 12x16 sparse MIMO
       (192 channels), 256 samples, 128 chirps
  c3   intersection: ground grid + 20 vehicles of 4 classes, ~1M triangles;
       192 channels, 512 samples, 256 chirps
  c4   64 scenes, 10k-400k triangles (log-uniform), 1-20 vehicles each;
       192 channels, 256 samples, 128 chirps
  c5   two vehicles of 100k triangles each at 20-40 m (gradient workload)

plus reduced-size variants used by parity tests (`small_*`). Everything is drawn
from numpy.random.default_rng(seed).
"""
from __future__ import annotations

import numpy as np

from .generators import (Config, Instance, RADAR_POS, LANE_CENTRES_X, Scene,
                         VEHICLE_CLASSES, box_mesh, ground_grid, literal_77_81_waveform,
                         paper_waveform, place_many, place_single, sparse_mimo_12x16,
                         ula_1tx4rx, vehicle_mesh, yaw_matrix, _instance_from)


def _c1_scene(seed: int) -> Scene:
    rng = np.random.default_rng(seed)
    L, W, H = 4.5, 1.8, 1.5
    mesh = box_mesh((-0.5 * L, -0.5 * W, 0.0), (0.5 * L, 0.5 * W, H), (16, 6, 7))
    assert mesh.n_tris == 1000
    lane = LANE_CENTRES_X[int(rng.integers(0, 3))]
    dz = RADAR_POS[2] - 0.5 * H
    y = np.sqrt(20.0 ** 2 - lane ** 2 - dz ** 2)
    centre = np.array([lane, y, 0.5 * H])
    los = (centre - RADAR_POS) / np.linalg.norm(centre - RADAR_POS)
    rot = yaw_matrix(np.pi / 2)  # length along the lane (Y)
    inst = Instance(mesh=0, rot=rot, pos0=np.array([lane, y, 0.0]), vel=-10.0 * los)
    return Scene(meshes=[mesh], instances=[inst])


def c1(seed: int = 1) -> Config:
    wf = literal_77_81_waveform(128, 32)
    return Config("c1", [_c1_scene(seed)], wf, ula_1tx4rx(wf), seed)


def c1p(seed: int = 1) -> Config:
    wf = paper_waveform(128, 32)
    return Config("c1p", [_c1_scene(seed)], wf, ula_1tx4rx(wf), seed)


def single_vehicle_scene(seed: int, n_tris: int, cls: str = "car",
                         range_lo=10.0, range_hi=60.0) -> Scene:
    rng = np.random.default_rng(seed)
    mesh = vehicle_mesh(cls, n_tris)
    H = VEHICLE_CLASSES[cls][2]
    x, y, yaw, speed = place_single(rng, H, range_lo, range_hi)
    return Scene(meshes=[mesh], instances=[_instance_from(0, x, y, yaw, speed)])


def c2(seed: int = 2, n_tris: int = 50_000, n_samples: int = 256,
       n_chirps: int = 128) -> Config:
    wf = paper_waveform(n_samples, n_chirps)
    return Config("c2", [single_vehicle_scene(seed, n_tris)], wf,
                  sparse_mimo_12x16(wf, seed), seed)


def intersection_scene(seed: int, n_vehicles: int = 20, per_vehicle: int = 44_250,
                       with_ground: bool = True, ground_cell: float = 0.25,
                       classes=None) -> Scene:
    rng = np.random.default_rng(seed)
    names = list(VEHICLE_CLASSES)
    if classes is None:
        classes = [names[int(rng.integers(0, 4))] for _ in range(n_vehicles)]
    poses = place_many(rng, classes)
    meshes, insts = [], []
    if with_ground:
        meshes.append(ground_grid(-30.0, 30.0, 0.0, 60.0, ground_cell))
        insts.append(Instance(mesh=0, rot=np.eye(3), pos0=np.zeros(3), vel=np.zeros(3)))
    budget = per_vehicle if np.ndim(per_vehicle) == 0 else None
    for k, (cls, (x, y, yaw, speed)) in enumerate(zip(classes, poses)):
        nt = budget if budget is not None else int(per_vehicle[k])
        meshes.append(vehicle_mesh(cls, nt))
        insts.append(_instance_from(len(meshes) - 1, x, y, yaw, speed))
    return Scene(meshes=meshes, instances=insts)


def c3(seed: int = 3) -> Config:
    wf = paper_waveform(512, 256)
    return Config("c3", [intersection_scene(seed)], wf, sparse_mimo_12x16(wf, seed), seed)


def batched_scene(seed: int) -> Scene:
    rng = np.random.default_rng(seed)
    budget = float(np.exp(rng.uniform(np.log(10_000), np.log(400_000))))
    n_v = int(rng.integers(1, 21))
    names = list(VEHICLE_CLASSES)
    classes = [names[int(rng.integers(0, 4))] for _ in range(n_v)]
    per = max(400, int(budget / n_v))
    return intersection_scene(int(rng.integers(0, 2 ** 31)), n_vehicles=n_v,
                              per_vehicle=per, with_ground=False, classes=classes)


def c4(n_scenes: int = 64, first_seed: int = 400, n_samples: int = 256,
       n_chirps: int = 128) -> Config:
    wf = paper_waveform(n_samples, n_chirps)
    scenes = [batched_scene(first_seed + i) for i in range(n_scenes)]
    return Config("c4", scenes, wf, sparse_mimo_12x16(wf, 4), first_seed)


def two_vehicle_scene(seed: int, n_each: int = 100_000) -> Scene:
    rng = np.random.default_rng(seed)
    meshes = [vehicle_mesh("car", n_each), vehicle_mesh("truck", n_each)]
    insts = []
    for k, lane in enumerate((LANE_CENTRES_X[0], LANE_CENTRES_X[2])):
        H = VEHICLE_CLASSES[("car", "truck")[k]][2]
        r = rng.uniform(20.0, 40.0)
        dz = RADAR_POS[2] - 0.5 * H
        y = np.sqrt(max(r * r - lane * lane - dz * dz, 1.0))
        yaw = np.pi / 2 if rng.uniform() < 0.5 else -np.pi / 2
        insts.append(_instance_from(k, lane, y, yaw, rng.uniform(-15.0, 15.0)))
    return Scene(meshes=meshes, instances=insts)


def perturbed(scene: Scene, seed: int, pos_sigma=0.1, vel_sigma=0.5,
              vert_sigma=1e-3) -> Scene:
    """Seeded perturbation of a scene (target RDM of the gradient workload)."""
    rng = np.random.default_rng(seed)
    meshes = []
    for m in scene.meshes:
        v = m.verts.astype(np.float64) + rng.normal(0.0, vert_sigma, m.verts.shape)
        meshes.append(type(m)(verts=v.astype(np.float32), tris=m.tris.copy(), name=m.name))
    insts = []
    for i in scene.instances:
        dp = rng.normal(0.0, pos_sigma, 3)
        dp[2] = 0.0
        dv = rng.normal(0.0, vel_sigma, 3)
        dv[2] = 0.0
        insts.append(Instance(mesh=i.mesh, rot=i.rot.copy(), pos0=i.pos0 + dp,
                              vel=i.vel + dv))
    return Scene(meshes=meshes, instances=insts, points=scene.points)


def c5(seed: int = 5, n_each: int = 100_000, n_samples: int = 256,
       n_chirps: int = 128) -> Config:
    wf = paper_waveform(n_samples, n_chirps)
    sc = two_vehicle_scene(seed, n_each)
    cfg = Config("c5", [sc], wf, sparse_mimo_12x16(wf, seed), seed)
    cfg.notes["target_scene"] = perturbed(sc, seed + 1000)
    return cfg


# ----------------------------------------------------------------------------------
# reduced sizes for parity tests: several tiles and a ragged tail, oracle in seconds
# ----------------------------------------------------------------------------------

def small_single(seed: int = 12, n_tris: int = 1500, n_samples: int = 96,
                 n_chirps: int = 4, mimo: bool = True) -> Config:
    wf = paper_waveform(n_samples, n_chirps)
    arr = sparse_mimo_12x16(wf, seed) if mimo else ula_1tx4rx(wf)
    return Config("small_single", [single_vehicle_scene(seed, n_tris, range_lo=12.0,
                                                        range_hi=40.0)],
                  wf, arr, seed)


def small_intersection(seed: int = 13, n_samples: int = 64, n_chirps: int = 4) -> Config:
    wf = paper_waveform(n_samples, n_chirps)
    sc = intersection_scene(seed, n_vehicles=3, per_vehicle=600, with_ground=True,
                            ground_cell=2.0)
    return Config("small_intersection", [sc], wf, sparse_mimo_12x16(wf, seed), seed)


CONFIGS = {"c1": c1, "c1p": c1p, "c2": c2, "c3": c3, "c4": c4, "c5": c5}
