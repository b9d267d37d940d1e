// Device helpers shared by the binning of the reciprocal-space path and of
// the real-space pair sum (included by kernels.hip and realspace.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pswf {

constexpr int kSortThreads = 256;  // threads of the ordering kernels

// exclusive scan of count[0..n) into start[0..n], start[n] = total (one
// block of 1024 threads)
__device__ inline void scan_counts(const int *count, int *start, int n, int64_t total) {
  __shared__ int part[1024];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < n; base += 1024) {
    int i = base + threadIdx.x;
    int v = i < n ? count[i] : 0;
    part[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      int t = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
      __syncthreads();
      part[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < n) start[i] = carry + part[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += part[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) start[n] = int(total);
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
