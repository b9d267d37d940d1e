// Launchers of the gfx950 kernels (kernels.hip); all enqueue on `st`.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "device_types.hpp"

namespace pswf {

constexpr int kQChunk = 8192;   // atoms per block of the charge sums

size_t spread_lds_bytes(const Geo &g, int ncg);
size_t gather_lds_bytes(const Geo &g, int ncg);
size_t zpass_lds_bytes(const Geo &g);
size_t ypass_lds_bytes(const Geo &g);
size_t xpass_lds_bytes(const Geo &g);
int qsum_blocks(const Geo &g);

hipError_t enqueue_sort(const Geo &g, const Work &w, const float *pos, const float *q, hipStream_t st);
hipError_t enqueue_qsum(const Geo &g, const Work &w, const float *q, hipStream_t st);
hipError_t enqueue_spread(const Geo &g, const Tables &t, const Work &w, hipStream_t st);
hipError_t enqueue_forward_fft(const Geo &g, const Tables &t, const FftAxis &az, const FftAxis &ay,
                               const Work &w, hipStream_t st);
// mode 0: energy only, 1: energy + potential grid, 2: adjoint scaled by grad[c]
hipError_t enqueue_xmul(const Geo &g, const Tables &t, const FftAxis &ax, const Work &w, int mode,
                        const double *grad, hipStream_t st);
hipError_t enqueue_inverse_fft(const Geo &g, const Tables &t, const FftAxis &az, const FftAxis &ay,
                               const Work &w, hipStream_t st);
hipError_t enqueue_gather(const Geo &g, const Tables &t, const Work &w, float *forces, float *pot, int mode,
                          const double *grad, hipStream_t st);
hipError_t enqueue_finalize(const Geo &g, const Tables &t, const Work &w, double *energy, double *virial,
                            hipStream_t st);

}  // namespace pswf
