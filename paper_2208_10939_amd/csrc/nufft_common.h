// Types shared by the NUFFT facet-sum kernels (nufft.hip) and its spread (nufft_spread.hip):
// the forward record and where a launch's (scene, chirp) units keep their work.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "rsim_internal.h"
#include "rsim_launch.h"

namespace rsim {

// Forward record of one lit facet or point of one chirp (128 bytes; 144 with the delay
// within the chirp). Sources sit at grid position (the channel's path position - offset):
//   kind 1: three Gaussians, (offset, weight re, weight im) at s[3j .. 3j + 2], j < 3;
//   kind 2: one Gaussian at s[0 .. 2] and a Gaussian-weighted quadratic at s[3 .. 9]
//           (offset, c0, c1, c2 as re/im pairs, in powers of the cell distance);
//   kind 3: a Gaussian-weighted quadratic at s[3 .. 9];
//   kind 0: no contribution (zero-area facet).
// ext (with the delay within the chirp): velocity (3), its components along ut and ur,
// and the phase-centre path's Doppler shift of the source in cells (included in cell and
// frac).
template <bool INTRA>
struct alignas(16) NuRecF {
  double ut[3], ur[3];  // unit vectors from t_c and r_c to the centroid c at t_n
  double g1;            // (f_c - mu tau_c) / c: turns per metre of dL
  float rt, rr;         // |c - t_c|, |c - r_c|
  float t0;             // f_c tau_c - mu tau_c^2 / 2 reduced to [-1/2, 1/2] turns
  float frac;           // grid position of the phase-centre path minus `cell`
  int32_t cell;         // its grid cell (0 .. n_g - 1)
  int32_t kind;
  float s[10];
  float ext[INTRA ? 6 : 2];
};
static_assert(sizeof(NuRecF<false>) == 128 && sizeof(NuRecF<true>) == 144, "record size");

// Where one (scene, chirp) unit of a launch keeps its work: a plain launch covers chirps
// n0 .. n0 + n_chirps - 1 of one scene at fixed strides; a batched one reads the unit's
// scene, chirp, strides and run bounds from its table.
struct NuWork {
  const DevScene *sc;
  int n;
  int64_t rec;     // first record (and key, position) slot
  int64_t run;     // first run slot
  int64_t stride;  // record slots of the unit
  int32_t max_runs, run_len, b0, kspan;
};

__device__ inline NuWork nu_work(const DevScene &sc, const NuShape &ns, const NuBatch &bt, int u) {
  NuWork w;
  if (!bt.units) {
    w.sc = &sc;
    w.n = ns.n0 + u;
    w.rec = static_cast<int64_t>(u) * ns.rec_stride;
    w.run = static_cast<int64_t>(u) * ns.max_runs;
    w.stride = ns.rec_stride;
    w.max_runs = ns.max_runs;
    w.run_len = ns.run_len;
    w.b0 = ns.b0;
    w.kspan = ns.kspan;
  } else {
    const NuUnit un = load_uniform(bt.units + u);
    w.sc = bt.scenes + un.scene;
    w.n = un.n;
    w.rec = un.rec_base;
    w.run = un.run_base;
    w.stride = un.rec_stride;
    w.max_runs = un.max_runs;
    w.run_len = un.run_len;
    w.b0 = un.b0;
    w.kspan = un.kspan;
  }
  return w;
}

}  // namespace rsim
