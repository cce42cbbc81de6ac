"""Seeded synthetic scenes, arrays and waveforms (input data only)."""
from .generators import (Config, Instance, Mesh, Points, RadarArray, Scene, Waveform,
                         RADAR_POS, LANE_CENTRES_X, VEHICLE_CLASSES, box_mesh,
                         cylinder_y_mesh, ground_grid, hull_mesh, literal_77_81_waveform,
                         merge_meshes, paper_waveform, plate_scene, dihedral_scene, point_scene,
                         sparse_mimo_12x16, synthetic_y_cube, ula_1tx4rx, vehicle_mesh,
                         yaw_matrix, scene_digest)
from .configs import (CONFIGS, c1, c1p, c2, c3, c4, c5, perturbed, small_intersection,
                      small_single, single_vehicle_scene, intersection_scene,
                      two_vehicle_scene, batched_scene)
