// Real-space complement of the PSWF split on gfx950 (Eq. realLR with the
// mollifier of Eqs. G1, G6, G; Methods, "Implementation details"):
//
//   E_real^(c) = 1/2 sum_n sum'_{i,j} q_i q_j K_p(|r_j - r_i + n H|),
//   K_p(r) = (1 - G_p(r / r_c)) / r^p  for 0 < r < r_c, 0 beyond,
//
// with potentials dE/dq_i, forces -dE/dr_i and the virial -dE/d(strain).
// 1 - G_p is tabulated on rho = r / r_c in [0, 1] as a piecewise polynomial
// (16 segments of degree 11, fitted on the host in FP64), its derivative
// taken from the same polynomial.
//
// The cell may be triclinic (lattice vectors as the rows of H).  Atoms are
// binned on their fractional coordinates into cells whose widths across the
// lattice planes are >= r_c (the whole cell along an axis narrower than r_c)
// by a counting sort with a deterministic order inside each cell (ascending
// caller index).  One wave per cell: lane l takes home atom l / 4 of a group
// of 16 and every fourth atom of each neighbour cell (offsets -R..R per
// axis, each one periodic image of the cell it wraps to, shifted by lattice
// vectors),
// so the four lanes of an atom read the same neighbour record as the lanes
// of the other atoms (broadcast loads).  Every lane accumulates only its own
// atom: no atomics, a fixed summation order, bitwise reproducible results.
// Channels are processed in groups sharing one exponent, so the pair kernel
// is evaluated once per pair and group.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "device_sort.hpp"
#include "device_types.hpp"
#include "kernels.hpp"

namespace pswf {

namespace {

constexpr int kRsThreads = 64;   // one wave per cell
constexpr int kRsGroup = kRsThreads / 4;  // home atoms per pass

__global__ __launch_bounds__(256) void k_rs_zero(RsWork w, int ncell) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < ncell) w.count[i] = 0;
}

// wrapped position and cell per atom; the record [x, y, z, 0, q_0 .. q_{C-1}]
// in caller order.  The fractional coordinates s = H^-T r pick the cell and
// the whole cells k = floor(s) to remove: r - k H with the lattice vectors
// as FP32 double words.
__global__ __launch_bounds__(256) void k_rs_bin(RsGeo g, RsWork w, const float *__restrict__ pos,
                                                const float *__restrict__ q) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= g.N) return;
  float r[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    r[a] = pos[3 * i + a];
    if (!isfinite(r[a])) r[a] = 0.0f;
  }
  float kf[3];
  int cc[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float sa = fmaf(g.Binv[3 * a], r[0], fmaf(g.Binv[3 * a + 1], r[1], g.Binv[3 * a + 2] * r[2]));
    kf[a] = floorf(sa);
    float f = sa - kf[a];
    if (!(f >= 0.0f)) f = 0.0f;
    cc[a] = min(int(f * g.nc[a]), g.nc[a] - 1);
  }
  float xw[3];
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    float v = fmaf(-kf[2], g.A_hi[6 + b], fmaf(-kf[1], g.A_hi[3 + b], fmaf(-kf[0], g.A_hi[b], r[b])));
    v = fmaf(-kf[2], g.A_lo[6 + b], fmaf(-kf[1], g.A_lo[3 + b], fmaf(-kf[0], g.A_lo[b], v)));
    xw[b] = v;
  }
  float *rec = w.rec_b + i * g.srec;
  *reinterpret_cast<float4 *>(rec) = make_float4(xw[0], xw[1], xw[2], 0.0f);
  for (int c = 0; c < g.C; ++c) rec[4 + c] = q[int64_t(c) * g.N + i];
  const int cell = (cc[0] * g.nc[1] + cc[1]) * g.nc[2] + cc[2];
  w.cell_of[i] = cell;
  w.slot[i] = atomicAdd(&w.count[cell], 1);
}

__global__ __launch_bounds__(1024) void k_rs_scan(RsWork w, int ncell, int64_t N) {
  scan_counts(w.count, w.start, ncell, N);
}

__global__ __launch_bounds__(256) void k_rs_scatter(RsGeo g, RsWork w) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= g.N) return;
  w.perm_b[w.start[w.cell_of[i]] + w.slot[i]] = int(i);
}

__device__ __forceinline__ void rs_move(const RsGeo &g, const RsWork &w, int key, int dst) {
  const float4 *src = reinterpret_cast<const float4 *>(w.rec_b + int64_t(key) * g.srec);
  float4 *out = reinterpret_cast<float4 *>(w.rec_a + int64_t(dst) * g.srec);
  for (int v = 0; v < g.srec / 4; ++v) out[v] = src[v];
  w.perm_a[dst] = key;
}

// ascending caller index inside each cell
__global__ __launch_bounds__(kSortThreads) void k_rs_order(RsGeo g, RsWork w) {
  __shared__ int keys[2048];
  const int cell = blockIdx.x;
  const int s = w.start[cell], n = w.start[cell + 1] - s;
  if (n <= 0) return;
  if (n > 2048) {
    const int *sorted = order_radix(g.N, w.perm_b + s, w.perm_a + s, n);
    for (int k = threadIdx.x; k < n; k += kSortThreads) rs_move(g, w, sorted[k], s + k);
    return;
  }
  for (int k = threadIdx.x; k < n; k += kSortThreads) keys[k] = w.perm_b[s + k];
  __syncthreads();
  for (int k = threadIdx.x; k < n; k += kSortThreads) {
    const int key = keys[k];
    int rank = 0;
    for (int m = 0; m < n; ++m) rank += keys[m] < key;
    rs_move(g, w, key, s + rank);
  }
}

// 1 - G_p(rho) and its rho-derivative from the segment polynomial
__device__ __forceinline__ float2 rs_complement(const float *__restrict__ coef, float rho) {
  const float y = rho * kRsSeg;
  const int sg = min(int(y), kRsSeg - 1);
  const float tau = 2.0f * (y - sg) - 1.0f;
  const float4 *c4 = reinterpret_cast<const float4 *>(coef + sg * (kRsDeg + 1));
  const float4 a = c4[0], b = c4[1], d = c4[2];
  const float c[12] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, d.x, d.y, d.z, d.w};
  float r = c[kRsDeg], dr = 0.0f;
#pragma unroll
  for (int k = kRsDeg - 1; k >= 0; --k) {
    dr = fmaf(dr, tau, r);
    r = fmaf(r, tau, c[k]);
  }
  return make_float2(r, dr * (2.0f * kRsSeg));
}

// One wave per cell.  Channel groups (one exponent each) are described by
// grp[4 * gidx] = {p, first entry in gch, count, table index}; gch lists
// channels.  Potentials are written per channel; forces after all groups.
template <int CG>
__global__ __launch_bounds__(kRsThreads) void k_rs_pairs(RsGeo g, RsTables t, RsWork w, const int *__restrict__ grp,
                                                         const int *__restrict__ gch, int ngrp,
                                                         float *__restrict__ forces, float *__restrict__ pot) {
  const int cell = blockIdx.x;
  const int s0 = w.start[cell], n = w.start[cell + 1] - s0;
  const int lane = threadIdx.x, part = lane & 3;
  const int cz = cell % g.nc[2], cy = (cell / g.nc[2]) % g.nc[1], cx = cell / (g.nc[2] * g.nc[1]);
  double vir[6] = {0, 0, 0, 0, 0, 0};
  for (int g0 = 0; g0 < n; g0 += kRsGroup) {
    const int ia = g0 + (lane >> 2);
    const bool act = ia < n;
    const int i = s0 + min(ia, n - 1);
    const float4 xi = *reinterpret_cast<const float4 *>(w.rec_a + int64_t(i) * g.srec);
    float f[3] = {0.f, 0.f, 0.f};
    float wv[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int gi = 0; gi < ngrp; ++gi) {
      const int p = grp[4 * gi], gb = grp[4 * gi + 1], gn = grp[4 * gi + 2];
      const float *coef = t.ucoef + grp[4 * gi + 3] * kRsCoef;
      int ch[CG];
      float qi[CG], phi[CG];
#pragma unroll
      for (int k = 0; k < CG; ++k) {
        ch[k] = gch[gb + min(k, gn - 1)];
        qi[k] = k < gn ? w.rec_a[int64_t(i) * g.srec + 4 + ch[k]] : 0.0f;
        phi[k] = 0.0f;
      }
      for (int dx = -g.R[0]; dx <= g.R[0]; ++dx) {
        int ax = cx + dx, kx = 0;
        while (ax < 0) { ax += g.nc[0]; --kx; }
        while (ax >= g.nc[0]) { ax -= g.nc[0]; ++kx; }
        for (int dy = -g.R[1]; dy <= g.R[1]; ++dy) {
          int ay = cy + dy, ky = 0;
          while (ay < 0) { ay += g.nc[1]; --ky; }
          while (ay >= g.nc[1]) { ay -= g.nc[1]; ++ky; }
          for (int dz = -g.R[2]; dz <= g.R[2]; ++dz) {
            int az = cz + dz, kz = 0;
            while (az < 0) { az += g.nc[2]; --kz; }
            while (az >= g.nc[2]) { az -= g.nc[2]; ++kz; }
            const int nb = (ax * g.nc[1] + ay) * g.nc[2] + az;
            const int js = w.start[nb], je = w.start[nb + 1];
            // the image shift k H (lattice vectors as double words): hi
            // part added to r_j, then r_i subtracted, then the lo part
            const float kv[3] = {float(kx), float(ky), float(kz)};
            float shi[3], slo[3];
#pragma unroll
            for (int b = 0; b < 3; ++b) {
              const float th[3] = {g.A_hi[b], g.A_hi[3 + b], g.A_hi[6 + b]};
              const float tl[3] = {g.A_lo[b], g.A_lo[3 + b], g.A_lo[6 + b]};
              grid_coord(kv, th, tl, &shi[b], &slo[b]);
            }
            for (int j = js + part; j < je; j += 4) {
              const float *rj = w.rec_a + int64_t(j) * g.srec;
              const float4 xj = *reinterpret_cast<const float4 *>(rj);
              const float dxv = ((xj.x + shi[0]) - xi.x) + slo[0];
              const float dyv = ((xj.y + shi[1]) - xi.y) + slo[1];
              const float dzv = ((xj.z + shi[2]) - xi.z) + slo[2];
              const float r2 = fmaf(dxv, dxv, fmaf(dyv, dyv, dzv * dzv));
              if (!(r2 < g.rc2) || !(r2 > 0.0f)) continue;
              const float rinv = rsqrtf(r2);
              const float r = r2 * rinv;
              const float2 u = rs_complement(coef, r * g.inv_rc);
              float rp = rinv;
              for (int e = 1; e < p; ++e) rp *= rinv;
              const float K = u.x * rp;
              const float Kd = u.y * g.inv_rc * rp - float(p) * K * rinv;   // dK/dr
              float qk = 0.0f;
#pragma unroll
              for (int k = 0; k < CG; ++k) {
                if (k < gn) {
                  const float qj = rj[4 + ch[k]];
                  phi[k] = fmaf(qj, K, phi[k]);
                  qk = fmaf(qi[k] * qj, Kd, qk);
                }
              }
              const float s = qk * rinv;   // q_i q_j K' / r
              f[0] = fmaf(s, dxv, f[0]);
              f[1] = fmaf(s, dyv, f[1]);
              f[2] = fmaf(s, dzv, f[2]);
              wv[0] = fmaf(s * dxv, dxv, wv[0]);
              wv[1] = fmaf(s * dyv, dyv, wv[1]);
              wv[2] = fmaf(s * dzv, dzv, wv[2]);
              wv[3] = fmaf(s * dxv, dyv, wv[3]);
              wv[4] = fmaf(s * dxv, dzv, wv[4]);
              wv[5] = fmaf(s * dyv, dzv, wv[5]);
            }
          }
        }
      }
      // the four lanes of an atom hold parts of its sums
#pragma unroll
      for (int k = 0; k < CG; ++k) {
        phi[k] += __shfl_xor(phi[k], 1, 4);
        phi[k] += __shfl_xor(phi[k], 2, 4);
      }
      const int dst = w.perm_a[i];
#pragma unroll
      for (int k = 0; k < CG; ++k) {
        if (k < gn) {
          if (act && part == 0 && pot) pot[int64_t(ch[k]) * g.N + dst] = phi[k];
          // energy of this wave's atoms: 1/2 sum_i q_i phi_i, summed in lane order
          float e = (act && part == 0) ? 0.5f * qi[k] * phi[k] : 0.0f;
          for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
          if (lane == 0) w.part[int64_t(cell) * (g.C + 6) + ch[k]] += double(e);
        }
      }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      f[a] += __shfl_xor(f[a], 1, 4);
      f[a] += __shfl_xor(f[a], 2, 4);
    }
    if (act && part == 0 && forces) {
      const int64_t o = 3 * int64_t(w.perm_a[i]);
      forces[o] = f[0];
      forces[o + 1] = f[1];
      forces[o + 2] = f[2];
    }
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      float v = act ? wv[a] : 0.0f;
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      vir[a] += double(v);
    }
  }
  if (lane < 6) {
    double v = 0.0;
#pragma unroll
    for (int a = 0; a < 6; ++a)
      if (lane == a) v = vir[a];
    w.part[int64_t(cell) * (g.C + 6) + g.C + lane] = -0.5 * v;   // W = -1/2 sum q_i q_j K' d d / r
  }
}

__global__ __launch_bounds__(256) void k_rs_clear_part(RsGeo g, RsWork w) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < int64_t(g.ncell) * (g.C + 6)) w.part[i] = 0.0;
}

// energy [C] and virial [6]: per-cell partials summed in cell order
__global__ __launch_bounds__(256) void k_rs_finalize(RsGeo g, RsWork w, double *energy, double *virial) {
  __shared__ double red[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int col = 0; col < g.C + 6; ++col) {
    double a = 0.0;
    for (int c = tid; c < g.ncell; c += 256) a += w.part[int64_t(c) * (g.C + 6) + col];
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    if (lane == 0) red[wave] = a;
    __syncthreads();
    if (tid == 0) {
      const double v = red[0] + red[1] + red[2] + red[3];
      if (col < g.C) energy[col] = v;
      else if (virial) virial[col - g.C] = v;
    }
    __syncthreads();
  }
}

}  // namespace

#define RS_CHECK()                              \
  do {                                          \
    hipError_t e__ = hipGetLastError();         \
    if (e__ != hipSuccess) return e__;          \
  } while (0)

hipError_t launch_realspace(const RsGeo &g, const RsTables &t, const RsWork &w, const int *grp, const int *gch,
                            int ngrp, int cgmax, const float *pos, const float *q, double *energy, float *forces,
                            double *virial, float *pot, hipStream_t st) {
  const unsigned nb_c = unsigned((g.ncell + 255) / 256);
  const unsigned nb_n = unsigned((g.N + 255) / 256);
  hipLaunchKernelGGL(k_rs_zero, dim3(nb_c), dim3(256), 0, st, w, g.ncell);
  RS_CHECK();
  if (g.N > 0) {
    hipLaunchKernelGGL(k_rs_bin, dim3(nb_n), dim3(256), 0, st, g, w, pos, q);
    RS_CHECK();
  }
  hipLaunchKernelGGL(k_rs_scan, dim3(1), dim3(1024), 0, st, w, g.ncell, g.N);
  RS_CHECK();
  const int64_t nparts = int64_t(g.ncell) * (g.C + 6);
  hipLaunchKernelGGL(k_rs_clear_part, dim3(unsigned((nparts + 255) / 256)), dim3(256), 0, st, g, w);
  RS_CHECK();
  if (g.N > 0) {
    hipLaunchKernelGGL(k_rs_scatter, dim3(nb_n), dim3(256), 0, st, g, w);
    RS_CHECK();
    hipLaunchKernelGGL(k_rs_order, dim3(g.ncell), dim3(kSortThreads), 0, st, g, w);
    RS_CHECK();
    if (cgmax <= 2)
      hipLaunchKernelGGL(k_rs_pairs<2>, dim3(g.ncell), dim3(kRsThreads), 0, st, g, t, w, grp, gch, ngrp, forces, pot);
    else if (cgmax <= 4)
      hipLaunchKernelGGL(k_rs_pairs<4>, dim3(g.ncell), dim3(kRsThreads), 0, st, g, t, w, grp, gch, ngrp, forces, pot);
    else
      hipLaunchKernelGGL(k_rs_pairs<16>, dim3(g.ncell), dim3(kRsThreads), 0, st, g, t, w, grp, gch, ngrp, forces, pot);
    RS_CHECK();
  }
  hipLaunchKernelGGL(k_rs_finalize, dim3(1), dim3(256), 0, st, g, w, energy, virial);
  RS_CHECK();
  return hipSuccess;
}

}  // namespace pswf
