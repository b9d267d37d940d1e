// Launchers of the gfx950 kernels (kernels.hip); all enqueue on `st`.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "device_types.hpp"

namespace pswf {

constexpr int kQChunk = 8192;   // atoms per block of the charge sums
constexpr int kPrepSmallMax = 2048;  // structures up to this size bin, order and sum in one launch
static_assert(kPrepSmallMax <= kQChunk, "the one-launch charge sums assume a single block");
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;  // workspace of pswflr_execute_noalloc
constexpr int kNoallocMaxDevices = 64;

// device address of this device's no-allocation scratch array (looked up
// once per device, with the device current)
hipError_t noalloc_scratch(void **out);

size_t spread_lds_bytes(const Geo &g, int ncg);
size_t gather_lds_bytes(const Geo &g, int ncg);
bool gather_tile_ok(int bx, int by, int bz, int P);  // halo staging map and LDS fit
size_t zpass_lds_bytes(const Geo &g);
size_t ypass_lds_bytes(const Geo &g);
size_t xpass_lds_bytes(const Geo &g);
int qsum_blocks(const Geo &g);
int spread_max_channels();   // channels per spreading launch
bool x_register_path(const Geo &g);  // the fused x pass runs the 256-point register FFT
bool spread_tile_ok(int bx, int by, int bz);  // tile fits the spreading kernel's blocks and LDS
int spread_candidate_cells(const int *nc, const int *b, int P);  // cells a tile screens
int spread_max_cells();
int spread_flush_cap(int64_t tiles);  // candidates per flush of the vector-ALU spread for a launch of this many tiles

// binning, cell order and the per-channel charge sums (five launches)
hipError_t enqueue_sort(const Geo &g, const Work &w, const float *pos, const float *q, hipStream_t st);
// the same in one launch when prep_small(g)
bool prep_small(const Geo &g);
hipError_t enqueue_prep_small(const Geo &g, const Work &w, const float *pos, const float *q, hipStream_t st);
hipError_t launch_spread(const Geo &g, const Tables &t, const Work &w, int cg0, int ncg, hipStream_t st,
                         const SpreadSrc &src = SpreadSrc{});
hipError_t launch_zfwd(const Geo &g, const Tables &t, const FftAxis &az, const Work &w, hipStream_t st);
hipError_t launch_yfwd(const Geo &g, const Tables &t, const FftAxis &ay, const Work &w, hipStream_t st);
// mode 0: energy only, 1: energy + potential grid, 2: adjoint scaled by grad[c]
hipError_t launch_xmul(const Geo &g, const Tables &t, const FftAxis &ax, const Work &w, int mode,
                       const double *grad, hipStream_t st);
hipError_t launch_yinv(const Geo &g, const Tables &t, const FftAxis &ay, const Work &w, hipStream_t st);
hipError_t launch_zinv(const Geo &g, const Tables &t, const FftAxis &az, const Work &w, hipStream_t st);
hipError_t launch_gather(const Geo &g, const Tables &t, const Work &w, float *forces, float *pot, int mode,
                         const double *grad, hipStream_t st);
// derivatives of sum_i v_i . F_i after a forward call with forces on the
// same workspace (its potential grid is overwritten); qd [3 C N], s2 [C N],
// f2 [N][3] are scratch
hipError_t launch_double_backward(const Geo &g, const Tables &t, const FftAxis &az, const FftAxis &ay,
                                  const FftAxis &ax, const Work &w, const float *v, float *qd, float *s2, float *f2,
                                  float *grad_q, float *grad_pos, hipStream_t st);
// input validation: word w.status[1] gets bit 0 for a non-finite position,
// bit 1 for a non-finite charge
hipError_t launch_check_inputs(const Geo &g, const Work &w, const float *pos, const float *q, hipStream_t st);
hipError_t launch_finalize(const Geo &g, const Tables &t, const Work &w, double *energy, double *virial,
                           hipStream_t st);

// dE/dH = -(H^-T W) from a device virial [6] (xx, yy, zz, xy, xz, yz);
// hinv is H^-1 row-major (host values, passed by value)
struct CellInv {
  double m[9];
};
hipError_t launch_cell_gradient(const CellInv &hinv, const double *virial, double *grad, hipStream_t st);

// real-space complement: binning, ordering, pair sums and the FP64 reduction
// (realspace.hip); grp/gch describe channel groups sharing one exponent
hipError_t launch_realspace(const RsGeo &g, const RsTables &t, const RsWork &w, const int *grp, const int *gch,
                            int ngrp, int cgmax, const float *pos, const float *q, double *energy, float *forces,
                            double *virial, float *pot, hipStream_t st);

// batched execution (one launch per stage over every structure)
int batch_stage_threads(int stage);
// stage_a = kBsBin (with kBsQsum) or kBsScatter (with kBsQreduce) in one launch
hipError_t launch_batch_pair(const BatchItem *d_items, const int *d_prefix_a, int total_a, const int *d_prefix_b,
                             int total_b, int n, int stage_a, hipStream_t st);
int batch_stage_blocks(const BatchItem &it, int stage, bool adjoint);
size_t batch_stage_lds(const BatchItem &it, int stage);
hipError_t launch_batch_stage(const BatchItem *d_items, const int *d_prefix, int n, int stage, int total_blocks,
                              size_t lds, int mode, hipStream_t st);
// the batch's spreading, one launch per kernel variant (batch_spread_variant)
int batch_spread_variant(const Geo &g);
hipError_t launch_batch_spread(const BatchItem *d_items, const int *d_prefix, int n, int total_blocks, size_t lds,
                               int variant, hipStream_t st);

}  // namespace pswf
