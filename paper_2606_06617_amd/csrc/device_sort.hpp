// Device helpers shared by the binning of the reciprocal-space path and of
// the real-space pair sum (included by kernels.hip and realspace.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pswf {

constexpr int kSortThreads = 256;  // threads of the ordering kernels

// exclusive scan of count[0..n) into start[0..n], start[n] = total (one
// block of 1024 threads).  Each thread takes kScanPer consecutive counts
// and scans them serially; the threads' sums are scanned inside each wave
// by shuffles, and the waves' totals through LDS: one pass with two
// barriers per 1024 kScanPer counts.  Integer sums, so the result does not
// depend on the grouping.
constexpr int kScanPer = 8;
__device__ inline void scan_counts(const int *count, int *start, int n, int64_t total) {
  __shared__ int wsum[1024 / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int carry = 0;
  for (int base = 0; base < n; base += 1024 * kScanPer) {
    const int i0 = base + tid * kScanPer;
    int v[kScanPer], s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      v[k] = i0 + k < n ? count[i0 + k] : 0;
      s += v[k];
    }
    int x = s;  // inclusive scan of the threads' sums within the wave
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    int before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < 1024 / 64; ++k) {
      before += k < wave ? wsum[k] : 0;
      all += wsum[k];
    }
    int e = carry + before + x - s;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      if (i0 + k < n) start[i0 + k] = e;
      e += v[k];
    }
    carry += all;
    __syncthreads();  // wsum is rewritten by the next round
  }
  if (tid == 0) start[n] = int(total);
}

// Crowded cell (more keys than fit the LDS rank): stable least-significant-
// digit radix sort of its caller indices, 8 bits per pass, between two
// key buffers.  A pass takes the keys 256 at a time;
// inside a wave, lanes with equal digits are found by ballots over the 8
// digit bits and ranked by lane, waves in order, so every pass is stable and
// the cost is linear in the cell's size.  src and dst are the cell's
// ranges of two key arrays; returns the one holding the sorted keys.
__device__ inline int *order_radix(int64_t N, int *src, int *dst, int n) {
  __shared__ int hist[256];
  __shared__ int wcnt[kSortThreads / 64][256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int bits = N > 1 ? 32 - __clz(int(N - 1)) : 1;
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int shift = 0; shift < bits; shift += 8) {
    for (int d = tid; d < 256; d += kSortThreads) hist[d] = 0;
    __syncthreads();
    for (int k = tid; k < n; k += kSortThreads) atomicAdd(&hist[(src[k] >> shift) & 255], 1);
    __syncthreads();
    if (tid == 0) {  // exclusive prefix: the first slot of every digit
      int acc = 0;
      for (int d = 0; d < 256; ++d) {
        const int v = hist[d];
        hist[d] = acc;
        acc += v;
      }
    }
    __syncthreads();
    for (int k0 = 0; k0 < n; k0 += kSortThreads) {
      for (int e = tid; e < (kSortThreads / 64) * 256; e += kSortThreads) (&wcnt[0][0])[e] = 0;
      __syncthreads();
      const int k = k0 + tid;
      const bool valid = k < n;
      const int key = valid ? src[k] : 0;
      const int d = (key >> shift) & 255;
      unsigned long long eq = __ballot(valid);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const unsigned long long on = __ballot(valid && ((d >> b) & 1));
        eq &= ((d >> b) & 1) ? on : ~on;
      }
      const int rank = __popcll(eq & below);
      if (valid && rank == 0) wcnt[wave][d] = __popcll(eq);
      __syncthreads();
      if (valid) {
        int off = hist[d] + rank;
        for (int wq = 0; wq < wave; ++wq) off += wcnt[wq][d];
        dst[off] = key;
      }
      __syncthreads();
      for (int dd = tid; dd < 256; dd += kSortThreads) {
        int t = 0;
        for (int wq = 0; wq < kSortThreads / 64; ++wq) t += wcnt[wq][dd];
        hist[dd] += t;
      }
      __syncthreads();
    }
    int *tmp = src;
    src = dst;
    dst = tmp;
  }
  return src;
}

}  // namespace pswf
