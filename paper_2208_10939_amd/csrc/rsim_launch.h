// Host-side entry points of the kernels (implemented in the .hip files).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "rsim_internal.h"

namespace rsim {

// Facet-sum launch shape: a workgroup holds O_w channels x B_w blocks of MB samples
// (n_compute accumulating threads, O_w * B_w rounded up to whole waves; the forward
// kernel adds two staging waves).
struct EchoShape {
  int32_t O, O_w, o_tiles, B_w, M_t, m_tiles, E, n_compute;
  double two_pi_slope;  // 2 pi mu
  int32_t accumulate;   // 0: write the echo; 1: add gamma x (this path's echo) to it
  int32_t pad;
  double gamma_re, gamma_im;
  int32_t slots_tx, slots;  // matrix-core sum: element slots per facet (Tx first, padded)
};

constexpr int kStagingThreads = 128;  // staging waves of the forward facet sum
constexpr int kMaxComputeThreads = 384;  // + staging = 512 threads, 8 waves

int build_bvh(const float *verts, const int32_t *tris, int64_t n_tris,
              std::vector<BvhNode4> &nodes_out, std::vector<float> &leaf_out);

// Lit-facet masks of chirps [n_begin, n_begin + n_chirps), and their compaction into the
// per-chirp lit lists.
hipError_t launch_visibility(const DevScene &sc, const RadarConst &rc, int n_begin, int n_chirps,
                             hipStream_t s);
hipError_t launch_compact(const DevScene &sc, int n_begin, int n_chirps, hipStream_t s);
// Facet-to-facet double bounce: the connection of every (launching end, chirp, facet)
// into pair_b [2][N][F] (the connected facet or -1), then per (end, chirp) the connected
// facets in ascending order into idx [2][N][F] and their counts into cnt [2][N]. ray_len:
// metres a reflected ray is followed (0: pair_b is given; only the compaction runs);
// r_lim: the scene's largest facet radius. With ray_len > 0, sc.mask holds the chirps'
// single-path lit masks (a lit facet sees both phase centres).
hipError_t launch_dbounce(const DevScene &sc, const RadarConst &rc, double ray_len, double r_lim,
                          int32_t *pair_b, int32_t *idx, int32_t *cnt, hipStream_t s);

hipError_t launch_echo_plain(int precision, int mb, int ft, const DevScene &sc,
                             const RadarConst &rc, const double *elem, const EchoShape &sh,
                             hipStream_t s);
hipError_t launch_echo_persistent(int precision, int mb, int ft, const DevScene *scenes,
                                  const int4 *items, int32_t n_items, int32_t *queue,
                                  const RadarConst &rc, const double *elem, const EchoShape &sh,
                                  int n_groups, hipStream_t s);
hipError_t echo_occupancy(int precision, int mb, int ft, const EchoShape &sh, int *groups_per_cu);
bool echo_variant_exists(int precision, int mb, int ft);
size_t echo_smem_bytes(int precision, int mb, int ft, const EchoShape &sh);

// facet sum on the matrix cores (FP32, separable Tx x Rx form without the cross term):
// one workgroup per (chirp, 128-sample tile)
bool mfma_variant(int P, int Q, int *pt, int *qt);
size_t mfma_smem_bytes(const EchoShape &sh);
int mfma_tile_samples();
hipError_t launch_echo_mfma(const DevScene &sc, const RadarConst &rc, const double *elem,
                            const EchoShape &sh, hipStream_t s);
hipError_t launch_echo_mfma_persistent(const DevScene *scenes, const int4 *items, int32_t n_items,
                                       int32_t *queue, const RadarConst &rc, const double *elem,
                                       const EchoShape &sh, int n_groups, hipStream_t s);
hipError_t mfma_occupancy(int P, int Q, const EchoShape &sh, int *groups_per_cu);

// facet sum as a type-1 non-uniform FFT over the sample index (FP32): Gaussian spread
// of kNuWidth cells with standard deviation kNuSigma cells onto n_g >= 2M cells
constexpr int kNuWidth = 12;
constexpr double kNuSigma = 1.1;
// forward spread: register window of kNuSlots grid cells per lane; a run of sorted
// records spans at most `kspan` cells so that all its sources fit one window
constexpr int kNuSlots = 32;
struct NuShape {
  int32_t ng, ld, cb, groups;  // grid cells, LDS row stride, channels per FFT workgroup, groups
  int32_t n0, n_chirps;        // chirps of this launch: n0 .. n0 + n_chirps - 1
  int32_t spread_groups;       // 64-channel groups of the spread
  int32_t pad1;
  int64_t rec_stride;          // records per chirp (forward: lit facets + points)
  double chan_d;               // largest grid offset of a channel from the phase-centre path
  double wave_d;               // largest grid offset of a channel from the first of its wave
  double fc, kc;               // f0 + (M/2) df; 2 pi fc / c
  double cells_per_s;          // df ng: grid cells per second of round-trip delay
  double kappa;                // df ng / c: grid cells per metre of path length
  double sigma;                // kNuSigma
  int32_t accumulate;          // 0: write the echo; 1: add gamma x (this path's echo) to it
  int32_t pad2;
  double gamma_re, gamma_im;
  // forward: sources lie within off_max cells of their record's path position; the
  // window of a run starts b0 cells below its first record's cell; runs hold at most
  // run_len records over at most kspan + 1 cells; max_runs per chirp bounds their count
  double off_max;
  int32_t b0, kspan, run_len, max_runs;
};
// Work buffers of one launch (n_chirps chirps). Forward: per (chirp, entry) the grid cell
// and the position in cell order, the records in that order, per chirp the runs
// (first record, end, window base cell) and their count, and per (chirp, run, channel)
// the window of kNuSlots cells. Adjoint: see launch_nufft_adjoint.
struct NuBuffers {
  int32_t *key;
  int32_t *pos;
  void *srec;
  float2 *grid;      // forward: partial windows [chirp][max_runs][O][kNuSlots]
  size_t rec_bytes;  // record slot size of srec (a launch refuses wider records)
  void *sder;        // adjoint records in the same order (adjoint only)
  int4 *runs;        // forward: [chirp][max_runs]
  int32_t *n_runs;   // forward: [chirp]
  // forward, optional: record counts by source form, kNuCensusSlots rows of 4 (summed by
  // the host); nullptr: no census
  unsigned long long *census;
  int32_t *order;  // adjoint: the class lists ordered by cell [chirp][classes][rec_stride]
  // adjoint with the facet-to-facet double bounce (else null / 0): per connection (chirp,
  // connection j) its seven adjoint sums [chirp][db_stride][kAdjVals] and its per-element
  // distance sums [chirp][db_stride][P + Q] (dL/dR of each Tx, then each Rx element)
  float *part_db;
  float *el_db;
  int64_t db_stride;
};
constexpr int kNuCensusSlots = 64;
// Tx + Rx elements the double-bounce adjoint's gather takes (an LDS column of 256 lanes per
// element beside the 32 KB staging area: 64 KB at most)
constexpr int kNuDbMaxElems = 32;
// One (scene, chirp) unit of a batched NUFFT launch: the scene's index in the launch's
// scene table, the chirp, where its records and runs start in the work buffers and the
// scene's own record capacity, run bound and run cutting (as in NuShape).
struct NuUnit {
  int32_t scene, n;
  int64_t rec_base;
  int64_t rec_stride;
  int64_t run_base;
  int32_t max_runs, run_len, b0, kspan;
};
// Batched NUFFT launch: units[0 .. ns.n_chirps) of scenes[]; {nullptr, nullptr}: a plain
// launch over chirps n0 .. n0 + n_chirps - 1 of one scene.
struct NuBatch {
  const DevScene *scenes;
  const NuUnit *units;
};
size_t nufft_record_bytes(bool intra);
size_t nufft_der_bytes();
size_t nufft_smem_bytes(const NuShape &ns);
size_t nufft_fft_smem_bytes(const NuShape &ns);
size_t nufft_sort_smem_bytes(const NuShape &ns);
int nufft_cells_per_source(const NuShape &ns);  // 14, 16 or 20; 0: channels too far apart
hipError_t launch_fill_zero(float *p, int64_t n, hipStream_t s);
// Forward NUFFT facet sum of ns.n_chirps units (plain: chirps of sc; batched: bt.units,
// with ns.rec_stride and ns.max_runs the largest of the launch's units).
// ev (optional): two events recorded just before and just after the spread kernel.
hipError_t launch_nufft(const DevScene &sc, const RadarConst &rc, const double *elem,
                        const NuShape &ns, const NuBuffers &nb, const void *tw, hipStream_t s,
                        const NuBatch &bt = NuBatch{nullptr, nullptr},
                        const hipEvent_t *ev = nullptr);
// The spread of launch_nufft (nufft_spread.hip): the runs of ns.n_chirps units into the
// partial windows part [unit's runs][O][kNuSlots].
hipError_t launch_nufft_spread(const DevScene &sc, const RadarConst &rc, const NuShape &ns,
                               const double *elem, const void *srec, const int4 *runs,
                               const int32_t *n_runs, float2 *part, const NuBatch &bt,
                               hipStream_t s);
// Floats per (chirp, lit facet, slot) of the adjoint sums: dL/dc through the element
// distances (3), sum Re y, dL/dbeta_v (3), pad.
constexpr int kAdjSlotFloats = 8;
// Per-(chirp, lit facet, slot) sums -> world-vertex gradients (FP64 chain rule) into gxw
// (zero on entry; added to it with sh.accumulate), slots = sh.m_tiles * sh.o_tiles. The
// adjoint launchers below clear gxw first unless sh.accumulate. partial_v / gxv (the
// vector-unit adjoint with the delay within the chirp, else both null): the velocity's
// sums over samples per slot [slot][4], summed into gxv [N][F][3] (as gxw for accumulate).
hipError_t launch_adjoint_finish(const DevScene &sc, const RadarConst &rc, const EchoShape &sh,
                                 const float *partial, float *gxw, hipStream_t s,
                                 const float *partial_v = nullptr, float *gxv = nullptr);
// Adjoint of launch_nufft for one chunk of chirps (stop-and-hop, facets only: sc.n_points
// must be 0): writes the per-(chirp, lit facet) adjoint sums into partial
// [N][n_facets][kAdjVals]. Uses nb.srec and nb.sder (records in entry order, rec_stride per
// chirp), nb.key (per chirp two lists of rec_stride entries: three-point records, others),
// nb.pos (the records' cells beside them), nb.order (the lists ordered by cell), nb.n_runs
// (their two counts per chirp) and nb.grid (grid rows [chirp][O][n_g]); n_g <= 2048.
// ev (optional): two events recorded around the two gather kernels.
// With the facet-to-facet double bounce (sc.db_on): the chirps' connections too (entries
// after the lit facets, rec_stride >= 3 F; classes 2 and 3 of the lists), their sums into
// nb.part_db / nb.el_db (db_stride >= 2 F) and their chain rule added into dbsum / dbtsum
// ([F][9] FP64 per-facet chirp sums, plain and t_n-weighted).
hipError_t launch_nufft_adjoint(const DevScene &sc, const RadarConst &rc, const double *elem,
                                const NuShape &ns, const NuBuffers &nb, const void *tw,
                                const void *grad_echo, float *partial, hipStream_t s,
                                const hipEvent_t *ev = nullptr, double *dbsum = nullptr,
                                double *dbtsum = nullptr);

// Allocation-free range-Doppler processing: a file-scope device array of
// kStaticScratchBytes per GPU, addressed through static_scratch_address (looked up once
// per device with that device current), and twiddle tables written into it by a kernel.
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
hipError_t static_scratch_address(int device, void **out);
hipError_t launch_twiddle_fill(void *tw, int L, int precision, hipStream_t s);

hipError_t launch_range_fft(int precision, const void *in, void *out, int64_t rows, int M,
                            int conj_in, const void *tw, hipStream_t s);
hipError_t launch_doppler_fft(int precision, const void *in, void *y_out, void *rdm,
                              int64_t planes, int N, int M, int mode, const void *tw,
                              hipStream_t s, const void *gp = nullptr);

// detection stage and white Gaussian noise
size_t cfar_smem_bytes(int gd, int gr, int td, int tr);
size_t angle_smem_bytes(int na_x, int na_z);
hipError_t launch_detect(const float *rdm, const void *y, int64_t cubes, int O, int N, int M,
                         int gd, int gr, int td, int tr, float scale, int na_x, int na_z,
                         int max_points, double range_res, double vel_res, const double *c_ref,
                         const int32_t *node_pos, const int32_t *node_off,
                         const int32_t *node_ch, int n_nodes, const void *tw_x, const void *tw_z,
                         float *P, uint8_t *det, float *noise, int32_t *list, int32_t *count,
                         void *points, hipStream_t s);
hipError_t launch_add_noise(int precision, void *echo, int64_t n, int64_t cubes, double snr_db,
                            uint64_t seed, double *part, double *scale, hipStream_t s);
int noise_partials_per_cube();

// adjoint of the facet sum (FP32): partial sums per (chirp, lit facet, tile), then
// per-facet world-vertex gradients gxw [N][F][9]
size_t adjoint_partial_floats(const EchoShape &sh, int64_t N, int64_t F);
size_t adjoint_smem_bytes(const EchoShape &sh, bool intra);
int adjoint_tile_m();
// adjoint on the matrix cores (FP32, separable form): one workgroup per (chirp,
// 64-sample tile); EchoShape with o_tiles = 1 and m_tiles = ceil(M / 64)
int adjoint_mfma_tile_m();
size_t adjoint_mfma_smem_bytes(int P, int Q, int E);
hipError_t launch_adjoint_mfma(const DevScene &sc, const RadarConst &rc, const double *elem,
                               const EchoShape &sh, const void *grad_echo, float *partial,
                               float *gxw, hipStream_t s);
// rc.intra: the delay within the chirp (then partial_v [N][F][slots][4] and gxv [N][F][3]
// are required, else both null).
hipError_t launch_adjoint(const DevScene &sc, const RadarConst &rc, const double *elem,
                          const EchoShape &sh, const void *grad_echo, float *partial, float *gxw,
                          hipStream_t s, float *partial_v = nullptr, float *gxv = nullptr);
// out[i] = conj(gamma) in[i] (complex64): the echo gradient of a path type added times gamma
hipError_t launch_scale_conj(const void *in, void *out, int64_t n, double gr, double gi,
                             hipStream_t s);
// world-vertex gradients [N][F][9] -> per-facet sums over chirps, plain and t_n-weighted;
// gxv (or null): the velocity's sums over samples [N][F][3], a third added to the
// t_n-weighted sum of each corner; dbsum (or null): [2][F][9] sums added to both (the
// double-bounce connections')
hipError_t launch_facet_chirp_sum(const float *gxw, const float *gxv, int64_t n_facets, int N,
                                  double tc, double *gsum, double *gtsum, hipStream_t s,
                                  const double *dbsum = nullptr);
hipError_t launch_vertex_gather(const double *gsum, const double *gtsum, const double *rot_dev,
                                int64_t facet_base, const int32_t *csr_off, const int32_t *csr_ent,
                                int32_t n_verts, float *gv, double *vpart, double *vel_out,
                                hipStream_t s);

}  // namespace rsim
