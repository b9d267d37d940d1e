// gfx950 kernels of the PSWF-LR reciprocal-space path.
//
// Pipeline (Methods, "Accelerating atom-grid spreading with PSWFs"):
//   bin/sort  -> spread (step i) -> z R2C, y FFT (step ii)
//   -> fused [x FFT, diagonal scaling + energy/virial partials (steps iii,
//      iv), inverse x FFT] -> inverse y, z C2R -> gather (adjoint of i)
//   -> FP64 reductions.
// The spectrum is pruned to the k-ball: only |k_z| <= k_c columns leave the
// z transform and only |k_y| <= k_c rows leave the y transform, since the
// kernel Phi_p vanishes beyond k_c (Eq. Fourier truncation).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

#include "device_sort.hpp"
#include "device_types.hpp"
#include "kernels.hpp"

namespace pswf {

#define PSWF_THREADS 256
static_assert(PSWF_THREADS == kSortThreads, "the ordering kernels run with the sort's block size");

// ---------------------------------------------------------------------------
// Streaming stores: results that the next pass reads once, written with the
// nontemporal hint so they do not linger in the caches as dirty lines the
// next pass's reads must wait behind (measured on the 256^3 passes: y, x
// and inverse y 5-15 % faster, the following z C2R 11 %).
typedef float nt_f2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void st_stream(float2 *p, float2 v) {
  const nt_f2 x = {v.x, v.y};
  __builtin_nontemporal_store(x, reinterpret_cast<nt_f2 *>(p));
}
__device__ __forceinline__ void st_stream(float4 *p, float4 v) {
  const nt_f4 x = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(x, reinterpret_cast<nt_f4 *>(p));
}

// Workgroups are dealt to the 8 XCDs round-robin by index; give each XCD a
// contiguous range of b in [0, n), so that neighbouring work runs behind the
// same L2.
__device__ __forceinline__ int xcd_contiguous(int b, int n) {
  const int q = n >> 3, r = n & 7, xcd = b & 7, j = b >> 3;
  return xcd * q + min(xcd, r) + j;
}
// the same for a 2D grid, returned as (x, y) block coordinates
__device__ __forceinline__ int2 xcd_contiguous_2d() {
  const int n = gridDim.x * gridDim.y, m = xcd_contiguous(blockIdx.y * gridDim.x + blockIdx.x, n);
  return make_int2(m % gridDim.x, m / gridDim.x);
}

// complex helpers
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ int fdiv(int n, const FastDiv &f) {
  return int((__umulhi(unsigned(n), f.m) + unsigned(n)) >> f.s);
}
// multiply by i*sigma (sigma = +-1)
template <int S>
__device__ __forceinline__ float2 mul_isig(float2 a) {
  return S > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// Small DFTs y_k = sum_j x_j w^(jk), w = exp(S 2 pi i / R), in place.
template <int R, int S>
struct Dft;

template <int S>
struct Dft<2, S> {
  __device__ __forceinline__ static void run(float2 *x) {
    float2 a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  }
};

template <int S>
struct Dft<3, S> {
  __device__ __forceinline__ static void run(float2 *x) {
    const float h = 0.86602540378443864676f;  // sqrt(3)/2
    float2 s = cadd(x[1], x[2]), d = csub(x[1], x[2]);
    float2 m = make_float2(x[0].x - 0.5f * s.x, x[0].y - 0.5f * s.y);
    float2 r = cscale(mul_isig<S>(d), h);
    x[0] = cadd(x[0], s);
    x[1] = cadd(m, r);
    x[2] = csub(m, r);
  }
};

template <int S>
struct Dft<4, S> {
  __device__ __forceinline__ static void run(float2 *x) {
    float2 a0 = cadd(x[0], x[2]), a1 = csub(x[0], x[2]);
    float2 b0 = cadd(x[1], x[3]), b1 = mul_isig<S>(csub(x[1], x[3]));
    x[0] = cadd(a0, b0);
    x[2] = csub(a0, b0);
    x[1] = cadd(a1, b1);
    x[3] = csub(a1, b1);
  }
};

template <int S>
struct Dft<5, S> {
  __device__ __forceinline__ static void run(float2 *x) {
    const float c1 = 0.30901699437494742410f, c2 = -0.80901699437494742410f;
    const float s1 = 0.95105651629515357212f, s2 = 0.58778525229247312917f;
    float2 a1 = cadd(x[1], x[4]), b1 = csub(x[1], x[4]);
    float2 a2 = cadd(x[2], x[3]), b2 = csub(x[2], x[3]);
    float2 x0 = x[0];
    float2 r1 = make_float2(x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y);
    float2 r2 = make_float2(x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y);
    float2 i1 = mul_isig<S>(make_float2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y));
    float2 i2 = mul_isig<S>(make_float2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y));
    x[0] = cadd(x0, cadd(a1, a2));
    x[1] = cadd(r1, i1);
    x[4] = csub(r1, i1);
    x[2] = cadd(r2, i2);
    x[3] = csub(r2, i2);
  }
};

template <int S>
struct Dft<8, S> {
  __device__ __forceinline__ static void run(float2 *x) {
    const float r = 0.70710678118654752440f;
    float2 e[4] = {x[0], x[2], x[4], x[6]};
    float2 o[4] = {x[1], x[3], x[5], x[7]};
    Dft<4, S>::run(e);
    Dft<4, S>::run(o);
    // w8^k = exp(S 2 pi i k / 8)
    float2 t1 = cscale(make_float2(o[1].x - S * o[1].y, o[1].y + S * o[1].x), r);   // (1 + iS)/sqrt2
    float2 t2 = mul_isig<S>(o[2]);
    float2 t3 = cscale(make_float2(-o[3].x - S * o[3].y, -o[3].y + S * o[3].x), r); // (-1 + iS)/sqrt2
    x[0] = cadd(e[0], o[0]);
    x[4] = csub(e[0], o[0]);
    x[1] = cadd(e[1], t1);
    x[5] = csub(e[1], t1);
    x[2] = cadd(e[2], t2);
    x[6] = csub(e[2], t2);
    x[3] = cadd(e[3], t3);
    x[7] = csub(e[3], t3);
  }
};

template <int S>
struct Dft<16, S> {
  // 16 = 4 x 4: DFT-4 over the stride-4 subsequences, twiddles w16^(n2 k1),
  // DFT-4 across them; output in natural order
  __device__ __forceinline__ static void run(float2 *x) {
    const float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f;  // cos, sin (pi/8)
    const float r = 0.70710678118654752440f;
    float2 a[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      a[n2][0] = x[n2];
      a[n2][1] = x[4 + n2];
      a[n2][2] = x[8 + n2];
      a[n2][3] = x[12 + n2];
      Dft<4, S>::run(a[n2]);
    }
    // w16^e = (cos(2 pi e / 16), S sin(2 pi e / 16))
    a[1][1] = cmul(a[1][1], make_float2(c1, S * s1));
    a[1][2] = cmul(a[1][2], make_float2(r, S * r));
    a[1][3] = cmul(a[1][3], make_float2(s1, S * c1));
    a[2][1] = cmul(a[2][1], make_float2(r, S * r));
    a[2][2] = mul_isig<S>(a[2][2]);
    a[2][3] = cmul(a[2][3], make_float2(-r, S * r));
    a[3][1] = cmul(a[3][1], make_float2(s1, S * c1));
    a[3][2] = cmul(a[3][2], make_float2(-r, S * r));
    a[3][3] = cmul(a[3][3], make_float2(-c1, -S * s1));
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      float2 b[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
      Dft<4, S>::run(b);
      x[k1] = b[0];
      x[k1 + 4] = b[1];
      x[k1 + 8] = b[2];
      x[k1 + 12] = b[3];
    }
  }
};

// One Stockham stage over the lines owned by one wave (LW = 2^lw_log2
// lines, wave w owns lines [w LW, (w + 1) LW)), each of length n stored in
// LDS as buf[idx * ld + line].  Butterfly j of a line reads x[j + r n/R],
// twiddles by exp(S 2 pi i r k / (ns R)) with k = j mod ns, and writes
// y[(j / ns) ns R + k + u ns]: the output of the last stage is in natural
// order.  Results are held in registers across a wave-scope fence, so the
// stage is in place and waves never wait for each other.  Each lane owns at
// most MAXE elements.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Copy `count` elements with every load of a thread in flight at once:
// load(e) for e = tid, tid + 256, ... (up to 16 per thread per round) into
// registers, then store(e, v).  Loads of the staging loops otherwise issue
// one at a time behind a wait each.
template <typename LoadF, typename StoreF>
__device__ __forceinline__ void staged16(int count, LoadF &&load, StoreF &&store) {
  for (int base = 0; base < count; base += 16 * PSWF_THREADS) {
    float2 v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int e = base + int(threadIdx.x) + r * PSWF_THREADS;
      v[r] = e < count ? load(e) : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int e = base + int(threadIdx.x) + r * PSWF_THREADS;
      if (e < count) store(e, v[r]);
    }
  }
}

template <int R, int S, int MAXE>
__device__ __forceinline__ void fft_stage(float2 *buf, int n, int ns, const FastDiv &nsd, int lw_log2, int ld,
                                          const float2 *tw, int lane, int wave) {
  constexpr int MAXB = (MAXE + R - 1) / R;
  const int nb = n / R;
  const int total = nb << lw_log2;
  const int twstep = n / (ns * R);
  const int line0 = wave << lw_log2;
  float2 v[MAXB][R];
  int oidx[MAXB];
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int b = lane + i * 64;
    oidx[i] = -1;
    if (b < total) {
      const int line = line0 + (b & ((1 << lw_log2) - 1));
      const int j = b >> lw_log2;
      const int jq = fdiv(j, nsd);
      const int k = j - jq * ns;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = buf[(j + r * nb) * ld + line];
      if (ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float2 w = tw[r * k * twstep];
          if (S > 0) w.y = -w.y;
          v[i][r] = cmul(v[i][r], w);
        }
      }
      Dft<R, S>::run(v[i]);
      oidx[i] = (jq * ns * R + k) * ld + line;
    }
  }
  wave_sync();
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    if (oidx[i] >= 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) buf[oidx[i] + r * ns * ld] = v[i][r];
    }
  }
  wave_sync();
}

// Full transform of the wave's lines.  S = -1 forward, +1 inverse
// (unnormalised in both directions).  tw[m] = exp(-2 pi i m / n).  The
// caller synchronises the workgroup before (data loaded) and after.
template <int S, int MAXE>
__device__ __forceinline__ void lds_fft(float2 *buf, const FftAxis &ax, int lw_log2, int ld, const float2 *tw, int tid) {
  const int lane = tid & 63, wave = tid >> 6;
  int ns = 1;
  for (int s = 0; s < ax.nst; ++s) {
    const int R = ax.rad[s];
    const FastDiv &nsd = ax.nsdiv[s];
    switch (R) {
      case 2: fft_stage<2, S, MAXE>(buf, ax.n, ns, nsd, lw_log2, ld, tw, lane, wave); break;
      case 3: fft_stage<3, S, MAXE>(buf, ax.n, ns, nsd, lw_log2, ld, tw, lane, wave); break;
      case 4: fft_stage<4, S, MAXE>(buf, ax.n, ns, nsd, lw_log2, ld, tw, lane, wave); break;
      case 5: fft_stage<5, S, MAXE>(buf, ax.n, ns, nsd, lw_log2, ld, tw, lane, wave); break;
      default: fft_stage<8, S, MAXE>(buf, ax.n, ns, nsd, lw_log2, ld, tw, lane, wave); break;
    }
    ns *= R;
  }
}

// Register FFTs of lines of N = N1 N2 points (N1 a multiple of N2) by the
// four-step split n = N2 n1 + n2, k = k1 + N1 k2:
//   X[k1 + N1 k2] = sum_n2 w_N2^(n2 k2) w_N^(n2 k1) sum_n1 w_N1^(n1 k1) x[N2 n1 + n2].
// A line is served by N2 threads.  Thread j enters with v[n1] = x[N2 n1 + j],
// does the inner DFT and the twiddles in registers (rfft_inner), passes
// v[k1] through LDS to the thread that owns column k1 = j + N2 q (q < N1/N2)
// and does the outer DFTs there (rfft_outer), leaving
// v[q N2 + k2] = X[j + N2 q + N1 k2].  With N1 = N2 the output layout is the
// input layout of the next transform.  tw[m] = exp(-2 pi i m / N).
template <int N1, int S>
__device__ __forceinline__ void rfft_inner(float2 *v, int j, const float2 *tw) {
  Dft<N1, S>::run(v);
#pragma unroll
  for (int k1 = 1; k1 < N1; ++k1) {
    float2 w = tw[j * k1];
    if (S > 0) w.y = -w.y;
    v[k1] = cmul(v[k1], w);
  }
}

template <int N1, int N2, int S>
__device__ __forceinline__ void rfft_outer(float2 *v) {
#pragma unroll
  for (int q = 0; q < N1 / N2; ++q) Dft<N2, S>::run(v + q * N2);
}

// geometry served by the register FFTs: 256-point x / y lines in blocks of
// 16 columns, 128-point (packed 256-real) z lines in blocks of 32
__host__ __device__ __forceinline__ bool zreg_ok(const Geo &g) { return g.Nz == 128 && g.zlines == 32; }
__host__ __device__ __forceinline__ bool yreg_ok(const Geo &g) { return g.M[1] == 256 && g.kb == 16; }
__host__ __device__ __forceinline__ bool xreg_ok(const Geo &g) { return g.M[0] == 256 && g.kb == 16; }
constexpr int kZregLine = 152;  // LDS float2 per z line: 16 x 9 exchange slots, padded to 8 (mod 16)

// ---------------------------------------------------------------------------
// Window psi_s(t), t in [-1, 1): piecewise polynomial in |t| (even function).
// The 12 coefficients of a segment are read as three 16-byte LDS loads
// (the table is 16-byte aligned), all in flight before the Horner chain.
static_assert(kWinDeg + 1 == 12, "window segments are read as three float4");
__device__ __forceinline__ void win_coef(const float *wc, int s, float (&c)[12]) {
  const float4 *c4 = reinterpret_cast<const float4 *>(wc + s * (kWinDeg + 1));
  const float4 a = c4[0], b = c4[1], d = c4[2];
  c[0] = a.x; c[1] = a.y; c[2] = a.z; c[3] = a.w;
  c[4] = b.x; c[5] = b.y; c[6] = b.z; c[7] = b.w;
  c[8] = d.x; c[9] = d.y; c[10] = d.z; c[11] = d.w;
}
__device__ __forceinline__ float win_eval(const float *wc, float t) {
  float a = fabsf(t);
  float y = a * kWinSeg;
  int s = min(int(y), kWinSeg - 1);
  float tau = 2.0f * (y - s) - 1.0f;
  float c[12];
  win_coef(wc, s, c);
  float r = c[kWinDeg];
#pragma unroll
  for (int d = kWinDeg - 1; d >= 0; --d) r = fmaf(r, tau, c[d]);
  return r;
}
// value and d/dt
__device__ __forceinline__ float2 win_eval_d(const float *wc, float t) {
  float a = fabsf(t);
  float y = a * kWinSeg;
  int s = min(int(y), kWinSeg - 1);
  float tau = 2.0f * (y - s) - 1.0f;
  float c[12];
  win_coef(wc, s, c);
  float r = c[kWinDeg], dr = 0.0f;
#pragma unroll
  for (int d = kWinDeg - 1; d >= 0; --d) {
    dr = fmaf(dr, tau, r);
    r = fmaf(r, tau, c[d]);
  }
  float dv = dr * (2.0f * kWinSeg);
  return make_float2(r, t < 0.0f ? -dv : dv);
}

// value, d/dt and d^2/dt^2
__device__ __forceinline__ float3 win_eval_dd(const float *wc, float t) {
  float a = fabsf(t);
  float y = a * kWinSeg;
  int s = min(int(y), kWinSeg - 1);
  float tau = 2.0f * (y - s) - 1.0f;
  float c[12];
  win_coef(wc, s, c);
  float r = c[kWinDeg], d1 = 0.0f, d2 = 0.0f;   // d2 accumulates p'' / 2
#pragma unroll
  for (int d = kWinDeg - 1; d >= 0; --d) {
    d2 = fmaf(d2, tau, d1);
    d1 = fmaf(d1, tau, r);
    r = fmaf(r, tau, c[d]);
  }
  const float sc = 2.0f * kWinSeg;
  return make_float3(r, (t < 0.0f ? -d1 : d1) * sc, 2.0f * d2 * sc * sc);
}

__device__ __forceinline__ int unpack_n0(unsigned v, int a) { return int((v >> (10 * a)) & 1023u); }

// ---------------------------------------------------------------------------
// Binning: each atom is assigned to the tile holding the first node of its
// window, n0 = ceil(x/h - P/2) (mod M); delta = n0 - (x/h - P/2) in [0, 1).
__device__ __forceinline__ void zero_body(const Geo &g, const Work &w, int bx) {
  int i = bx * PSWF_THREADS + threadIdx.x;
  if (i < g.ncell) w.cell_count[i] = 0;
  if (i == 0) w.status[0] = 0;
}

__global__ __launch_bounds__(PSWF_THREADS) void k_zero(Geo g, Work w) { zero_body(g, w, blockIdx.x); }

// one atom: its record (window offsets and packed window start), its tile
// and its slot in the tile (arbitrary order; the ordering pass fixes it)
__device__ __forceinline__ void bin_atom(const Geo &g, const Work &w, const float *__restrict__ pos, int64_t i) {
  unsigned packed = 0;
  float dl[3];
  int cell[3];
  bool bad = false;
  float rp[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    rp[a] = pos[3 * i + a];
    if (!isfinite(rp[a])) {  // reported through the status word; placed at 0
      bad = true;
      rp[a] = 0.0f;
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float uh, ul;
    grid_coord(rp, g.T_hi + 3 * a, g.T_lo + 3 * a, &uh, &ul);
    int n0;
    float delta;
    window_start_dw(uh, ul, g.M[a], g.P, &n0, &delta);
    dl[a] = delta;
    packed |= unsigned(n0) << (10 * a);
    cell[a] = n0 / g.B[a];
  }
  if (bad) atomicOr(w.status, 1);
  const int c = (cell[0] * g.nc[1] + cell[1]) * g.nc[2] + cell[2];
  w.cell_of[i] = c;
  w.slot[i] = atomicAdd(&w.cell_count[c], 1);
  float4 r = make_float4(dl[0], dl[1], dl[2], __uint_as_float(packed));
  *reinterpret_cast<float4 *>(w.q_b + i * g.srec) = r;
}

constexpr int kBinQChunk = 16;  // channels staged through LDS at a time by the binning
__device__ __forceinline__ void bin_body(const Geo &g, const Work &w, const float *__restrict__ pos,
                                         const float *__restrict__ q, int bx) {
  // atoms staged in caller order as records of g.srec floats: window
  // offsets and packed start, then the C charges (padded to a multiple of
  // four), so the reorder reads one aligned record per atom.  The charges
  // pass through LDS, up to kBinQChunk channels at a time: each channel's
  // run of the block's charges is read coalesced, then consecutive threads
  // write consecutive charge words of the block's records
  __shared__ float qs[kBinQChunk][PSWF_THREADS + 1];
  const int64_t b0 = int64_t(bx) * PSWF_THREADS;
  const int nrow = g.N - b0 < PSWF_THREADS ? int(g.N - b0) : PSWF_THREADS;
  const int tid = threadIdx.x;
  for (int c0 = 0; c0 < g.C; c0 += kBinQChunk) {
    const int nc = min(kBinQChunk, g.C - c0);
    if (tid < nrow)
      for (int k = 0; k < nc; ++k) qs[k][tid] = q[int64_t(c0 + k) * g.N + b0 + tid];
    __syncthreads();
    for (int f = tid; f < nrow * nc; f += PSWF_THREADS) {
      const int a = f / nc, ch = f - a * nc;
      w.q_b[(b0 + a) * g.srec + 4 + c0 + ch] = qs[ch][a];
    }
    __syncthreads();
  }
  const int64_t i = b0 + threadIdx.x;
  if (i < g.N) bin_atom(g, w, pos, i);
}

// exclusive scan of cell counts (single block)
__device__ __forceinline__ void scan_body(const Work &w, int ncell, int64_t N) {
  scan_counts(w.cell_count, w.cell_start, ncell, N);
}

__global__ __launch_bounds__(1024) void k_scan(Work w, int ncell, int64_t N) { scan_body(w, ncell, N); }

// scatter the caller index into cell order (arbitrary order inside a cell);
// records and charges follow in the per-cell ordering pass
__device__ __forceinline__ void scatter_body(const Geo &g, const Work &w, int bx) {
  const int64_t i = int64_t(bx) * PSWF_THREADS + threadIdx.x;
  if (i >= g.N) return;
  const int dst = w.cell_start[w.cell_of[i]] + w.slot[i];
  w.perm_b[dst] = int(i);
}

// move atom `key` (caller index) to cell-order position dst: its record,
// its charges and the permutation entry
__device__ __forceinline__ void order_move(const Geo &g, const Work &w, int key, int dst) {
  const float4 *rec = reinterpret_cast<const float4 *>(w.q_b + int64_t(key) * g.srec);
  reinterpret_cast<float4 *>(w.rec_a)[dst] = rec[0];
  w.perm_a[dst] = key;
  for (int c4 = 0; 4 * c4 < g.C; ++c4) {
    const float4 v = rec[1 + c4];
    const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (4 * c4 + j < g.C) w.q_a[int64_t(4 * c4 + j) * g.N + dst] = vv[j];
  }
}

// deterministic order inside each cell: ascending caller index
__device__ __forceinline__ void order_body(const Geo &g, const Work &w, int bx) {
  __shared__ int keys[2048];
  const int cell = bx;
  const int s = w.cell_start[cell], e = w.cell_start[cell + 1];
  const int n = e - s;
  if (n <= 0) return;
  if (n > 2048) {
    const int *sorted = order_radix(g.N, w.perm_b + s, w.perm_a + s, n);
    for (int k = threadIdx.x; k < n; k += PSWF_THREADS) order_move(g, w, sorted[k], s + k);
    return;
  }
  for (int k = threadIdx.x; k < n; k += PSWF_THREADS) keys[k] = w.perm_b[s + k];
  __syncthreads();
  for (int k = threadIdx.x; k < n; k += PSWF_THREADS) {
    const int key = keys[k];
    int rank = 0;
    for (int m = 0; m < n; ++m) rank += keys[m] < key;
    order_move(g, w, key, s + rank);
  }
}

__global__ __launch_bounds__(PSWF_THREADS) void k_order(Geo g, Work w) { order_body(g, w, blockIdx.x); }

// per-channel sum q and sum q^2 (FP64 block partials, fixed order)
__device__ __forceinline__ void qsum_body(const Geo &g, const Work &w, const float *__restrict__ q, int chunk, int bx, int by) {
  __shared__ double s0[PSWF_THREADS], s1[PSWF_THREADS];
  const int c = by;
  const int64_t b0 = int64_t(bx) * chunk;
  double a = 0.0, b = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < min(b0 + chunk, g.N); i += PSWF_THREADS) {
    double v = double(q[int64_t(c) * g.N + i]);
    a += v;
    b += v * v;
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  __syncthreads();
  for (int off = PSWF_THREADS / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      s0[threadIdx.x] += s0[threadIdx.x + off];
      s1[threadIdx.x] += s1[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    w.qpart[(int64_t(bx) * g.C + c) * 2 + 0] = s0[0];
    w.qpart[(int64_t(bx) * g.C + c) * 2 + 1] = s1[0];
  }
}

__device__ __forceinline__ void qreduce_body(const Geo &g, const Work &w, int nblk) {
  __shared__ double s0[PSWF_THREADS], s1[PSWF_THREADS];
  for (int c = 0; c < g.C; ++c) {
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < nblk; k += PSWF_THREADS) {
      a += w.qpart[(int64_t(k) * g.C + c) * 2 + 0];
      b += w.qpart[(int64_t(k) * g.C + c) * 2 + 1];
    }
    s0[threadIdx.x] = a;
    s1[threadIdx.x] = b;
    __syncthreads();
    for (int off = PSWF_THREADS / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) {
        s0[threadIdx.x] += s0[threadIdx.x + off];
        s1[threadIdx.x] += s1[threadIdx.x + off];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      w.qsum[2 * c] = s0[0];
      w.qsum[2 * c + 1] = s1[0];
    }
    __syncthreads();
  }
}

// The charge sums need only the charges, so they share launches with the
// sort: their per-block partials ride beside the binning (blocks nbin ..
// of the grid, chunk-major per channel), their reduction beside the
// scatter (the grid's first block).  Two launches fewer per call.
__global__ __launch_bounds__(PSWF_THREADS) void k_bin_qsum(Geo g, Work w, const float *__restrict__ pos,
                                                           const float *__restrict__ q, int nbin, int nq) {
  const int b = blockIdx.x;
  if (b < nbin) {
    bin_body(g, w, pos, q, b);
  } else {
    const int k = b - nbin;
    qsum_body(g, w, q, kQChunk, k % nq, k / nq);
  }
}

// the reduction is block 0, so that its serial channel loop starts first
// and overlaps the scatter blocks
__global__ __launch_bounds__(PSWF_THREADS) void k_scatter_qreduce(Geo g, Work w, int nscatter, int nq) {
  (void)nscatter;
  if (blockIdx.x == 0)
    qreduce_body(g, w, nq);
  else
    scatter_body(g, w, blockIdx.x - 1);
}

// Small structures (N <= kPrepSmallMax): the steps above in one workgroup
// of 1024 threads and one launch, with the same results bit for bit --
// records, tile counts and starts, the order inside each tile (ascending
// caller index) and the charge sums.  Phases are separated by workgroup
// barriers.  The order inside a tile is found by counting, for each atom,
// the atoms of its tile with a smaller caller index: quadratic in the
// tile's size, bounded by N^2 / 1024 reads per thread.
constexpr int kPrepThreads = 1024;
__global__ __launch_bounds__(kPrepThreads) void k_prep_small(Geo g, Work w, const float *__restrict__ pos,
                                                             const float *__restrict__ q) {
  __shared__ double s0[PSWF_THREADS], s1[PSWF_THREADS];
  __shared__ int lperm[kPrepSmallMax];
  const int tid = threadIdx.x;
  const int N = int(g.N);
  for (int i = tid; i < g.ncell; i += kPrepThreads) w.cell_count[i] = 0;
  if (tid == 0) w.status[0] = 0;
  __syncthreads();
  for (int f = tid; f < N * g.C; f += kPrepThreads) {
    const int a = f / g.C, ch = f - a * g.C;
    w.q_b[int64_t(a) * g.srec + 4 + ch] = q[int64_t(ch) * N + a];
  }
  for (int i = tid; i < N; i += kPrepThreads) bin_atom(g, w, pos, i);
  __syncthreads();
  scan_counts(w.cell_count, w.cell_start, g.ncell, g.N);
  __syncthreads();
  // caller indices in tile order (arbitrary inside a tile), kept in LDS
  for (int i = tid; i < N; i += kPrepThreads) lperm[w.cell_start[w.cell_of[i]] + w.slot[i]] = i;
  __syncthreads();
  for (int k = tid; k < N; k += kPrepThreads) {
    const int key = lperm[k];
    const int c = w.cell_of[key];
    const int s = w.cell_start[c], e = w.cell_start[c + 1];
    int rank = 0;
    for (int m = s; m < e; ++m) rank += lperm[m] < key;
    order_move(g, w, key, s + rank);
  }
  // charge sums per channel, in the order of qsum_body (one block of 256
  // threads, as N <= kQChunk) followed by qreduce_body over that one block
  for (int c = 0; c < g.C; ++c) {
    for (int pass = 0; pass < 2; ++pass) {
      double a = 0.0, b = 0.0;
      if (pass == 0) {
        if (tid < PSWF_THREADS)
          for (int i = tid; i < N; i += PSWF_THREADS) {
            const double v = double(q[int64_t(c) * N + i]);
            a += v;
            b += v * v;
          }
      } else if (tid == 0) {
        a = w.qpart[2 * c];
        b = w.qpart[2 * c + 1];
      }
      if (tid < PSWF_THREADS) {
        s0[tid] = a;
        s1[tid] = b;
      }
      __syncthreads();
      for (int off = PSWF_THREADS / 2; off > 0; off >>= 1) {
        if (tid < off) {
          s0[tid] += s0[tid + off];
          s1[tid] += s1[tid + off];
        }
        __syncthreads();
      }
      if (tid == 0) {
        double *dst = pass == 0 ? w.qpart + 2 * c : w.qsum + 2 * c;
        dst[0] = s0[0];
        dst[1] = s1[0];
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// Spread (step i), output-stationary.  One workgroup of 8 waves per tile.
// The tile is cut into 4 x 4 x 4 blocks.  Each wave owns four of them: NBZ
// consecutive blocks along z (the whole z extent of the tile) in each of
// 4 / NBZ neighbouring columns along y, and every lane owns one point of
// each block, with one accumulator per channel in registers.  Atoms of the
// candidate cells are screened in chunks; the ones whose window reaches
// into the tile are staged in LDS with their charges and, per axis, the
// window weights laid out over the tile's coordinates (zero outside the
// window; the z weights transposed so that a lane's NBZ values are
// adjacent), so a lane reads its weights with one load per axis and no
// index arithmetic.  A wave tests 64 staged candidates at a time against
// each of its blocks (ballot) and walks only the candidates that meet a
// block, with the LDS reads of the next one in flight while the current one
// is accumulated.  No atomics, no read-modify-write of shared memory; the
// summation order is fixed, so the result is bitwise reproducible.
constexpr int kSpreadThreads = 512;
constexpr int kSpreadCap = 256;     // candidates staged per flush (matrix-core variant; at most)
constexpr int kSpreadCapV = 128;    // the vector-ALU variants' smaller flush
constexpr int kSpreadScreenPer = 1; // atoms screened per thread per round
constexpr int kSpreadMaxCells = 64; // candidate cells of a tile
constexpr int kSpreadCGM = 16;      // channels per launch (most)
// accumulator counts the spread is instantiated for: 2 or 4 channels on the
// vector ALUs, up to 16 on the matrix cores
__host__ __device__ constexpr int spread_cg4(int cg) { return (cg + 3) / 4 * 4; }
__host__ __device__ constexpr int spread_cg_template(int ncg) { return ncg <= 2 ? 2 : (ncg <= 4 ? 4 : kSpreadCGM); }
__host__ __device__ constexpr bool spread_mfma(int cg) { return cg == kSpreadCGM; }
// Candidates per flush.  The vector-ALU variants (2 or 4 channels: the
// small grids of training batches and serving) take the plan's choice
// (Geo::scap): 128 when a launch has many more tiles than the chip holds at
// once, so their LDS footprint (about 36 KB at the largest tile) lets four
// workgroups share a CU, the most their registers allow; 256 when all its
// tiles are resident anyway, which saves a second flush on crowded tiles.
// Flush boundaries do not change the summation order.
__host__ __device__ constexpr int spread_cap(int cg, int scap) { return spread_mfma(cg) ? kSpreadCap : scap; }
// screened-candidate list: an unflushed tail (< cap) plus one screening round
__host__ __device__ constexpr int spread_list(int cap) { return cap + kSpreadScreenPer * kSpreadThreads; }
constexpr int kSpreadNBW = 4;       // 4x4x4 blocks per wave
constexpr int kSpreadMaxS = 64;     // padded tile edges Sx + Sy + Sz
constexpr int kSpreadBias = 8;      // packed window offsets are stored + bias
constexpr int kSpreadMaxPts = kSpreadNBW * (kSpreadThreads / 64) * 64;  // tile points
constexpr int kSpreadOutMax = (kSpreadMaxPts + kSpreadThreads - 1) / kSpreadThreads;  // scalar elements/thread

// LDS floats of the candidate staging area (charges and weights) for padded
// edges summing to S; the screened-candidate list, the candidate-cell table
// and the window coefficients follow it
// (one row past the staged candidates holds zeros: the padding of the
// matrix-core hit groups points there)
constexpr int kSpreadHitList = 68;  // per wave and block: 64 hits padded to whole groups of four
// staged charges per candidate: 16 for the matrix-core variant, the
// accumulator count rounded to 4 otherwise
__host__ __device__ constexpr int spread_qstride(int cg) { return spread_mfma(cg) ? kSpreadCGM : spread_cg4(cg); }
__host__ __device__ __forceinline__ int spread_stage_floats(int S, int cg, int cap) {
  return (cap + 1) * (spread_qstride(cg) + S);
}
// the block bits and hit lists only exist for the matrix-core variant
__host__ __device__ __forceinline__ int spread_lds_floats(int S, int cg, int cap) {
  return spread_stage_floats(S, cg, cap) + 5 * spread_list(cap) + 2 * kSpreadMaxCells + 1 + 3 + kWinSeg * (kWinDeg + 1) +
         (spread_mfma(cg) ? 2 * kSpreadCap + (kSpreadThreads / 64) * kSpreadNBW * kSpreadHitList / 2 : 0);
}
__host__ __device__ __forceinline__ int spread_pad4(int b) { return (b + 3) & ~3; }
// blocks along z of a tile edge (1, 2 or 4 supported); 0 if unsupported
__host__ __device__ __forceinline__ int spread_nbz(int bz) {
  const int n = spread_pad4(bz) >> 2;
  return (n == 1 || n == 2 || n == 4) ? n : 0;
}

// window [d, d + P) (mod M) meets block [o, o + S) ?  (0 <= d, o < M)
__device__ __forceinline__ bool win_meets(int o, int S, int d, int P, int M) {
  int a = o - d;
  if (a < 0) a += M;
  int b = d - o;
  if (b < 0) b += M;
  return a < P || b < S;
}

// one staged candidate as a lane needs it: its window weights at the lane's
// x, at its y in each column and at its z in each z block
template <int NBZ>
struct SpreadCand {
  static constexpr int CPW = kSpreadNBW / NBZ;
  float wx, wy[CPW], wz[NBZ];
};

template <int NBZ>
__device__ __forceinline__ void spread_load(const float *cw, int S, int kk, int xa, int ya, int za,
                                            SpreadCand<NBZ> &o) {
  constexpr int CPW = kSpreadNBW / NBZ;
  const char *wk = reinterpret_cast<const char *>(cw + kk * S);
  o.wx = *reinterpret_cast<const float *>(wk + xa);
#pragma unroll
  for (int c = 0; c < CPW; ++c) o.wy[c] = *reinterpret_cast<const float *>(wk + ya + 16 * c);
  if constexpr (NBZ == 4) {
    const float4 z4 = *reinterpret_cast<const float4 *>(wk + za);
    o.wz[0] = z4.x;
    o.wz[1] = z4.y;
    o.wz[2] = z4.z;
    o.wz[3] = z4.w;
  } else if constexpr (NBZ == 2) {
    const float2 z2 = *reinterpret_cast<const float2 *>(wk + za);
    o.wz[0] = z2.x;
    o.wz[1] = z2.y;
  } else {
    o.wz[0] = *reinterpret_cast<const float *>(wk + za);
  }
}

typedef float spread_f4 __attribute__((ext_vector_type(4)));
// Accumulators of a lane.  Vector-ALU variants: one per point of each of
// the wave's four blocks and per channel.  Matrix-core variant: per block
// and x slice of it, the lane's part of a 16 x 16 product tile (16 points of
// the 4 x 4 (y, z) slice by 16 channels): rows 4 (lane / 16) .. + 3, i.e.
// y = lane / 16 and z = 0..3, of channel lane % 16.
template <int CG>
struct SpreadAcc {
  float v[kSpreadNBW][CG];
};
template <>
struct SpreadAcc<kSpreadCGM> {
  spread_f4 v[kSpreadNBW][4];
};

__device__ __forceinline__ int spread_take(unsigned long long &u) {
  const int bit = __builtin_ctzll(u);
  u &= u - 1ull;
  return bit;
}

// add candidate `bit` of the current 64 to the blocks whose hit mask has
// it; its charges come from lane `bit` of the per-lane charge registers
// (v_readlane into SGPRs: a uniform operand of the FMAs, no LDS traffic)
template <int NBZ, int CG>
__device__ __forceinline__ void spread_accumulate(const SpreadCand<NBZ> &cnd, int bit, const float (&qreg)[spread_cg4(CG)],
                                                  const unsigned long long (&m)[kSpreadNBW],
                                                  float (&acc)[kSpreadNBW][CG]) {
  constexpr int CPW = kSpreadNBW / NBZ;
  float q[CG];
#pragma unroll
  for (int c = 0; c < CG; ++c)
    q[c] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(qreg[c]), bit));
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const float wxy = cnd.wx * cnd.wy[c];
#pragma unroll
    for (int z = 0; z < NBZ; ++z) {
      const int j = c * NBZ + z;
      if (!((m[j] >> bit) & 1ull)) continue;
      const float wv = wxy * cnd.wz[z];
#pragma unroll
      for (int qq = 0; qq < CG; ++qq) acc[j][qq] = fmaf(wv, q[qq], acc[j][qq]);
    }
  }
}

template <int P, int NBZ, int CG>
__device__ __forceinline__ void spread_flush(const Geo &g, const Work &w, int cg0, int ncg, int ncand, const int *sz,
                                             float *cq, float *cw, const int *cd, const float *cf, const int *ci,
                                             const float *wcf, const int (&bo)[3], bool wval, unsigned short *cbits,
                                             unsigned short *hl, SpreadAcc<CG> &accs, const SpreadSrc &src) {
  constexpr int CPW = kSpreadNBW / NBZ;
  constexpr bool MF = spread_mfma(CG);
  const int tid = threadIdx.x, lane = tid & 63;
  const int S = sz[0] + sz[1] + sz[2];
  const int soff[3] = {0, sz[0], sz[0] + sz[1]};
  // (1) per candidate and axis, the window weights over the padded tile
  // edge (zero outside the window); for the vector-ALU variants z position
  // zz is stored at (zz % 4) NBZ + zz / 4.  The window positions of one candidate are
  // distinct (P <= M), so they are plain stores after a zero fill whose
  // start rotates with the candidate (no bank conflicts between lanes).
  const int cap = spread_cap(CG, g.scap);
  for (int t = tid; t < 3 * cap; t += kSpreadThreads) {
    const int a = t / cap, k = t - a * cap;
    if (k >= ncand) continue;
    float qv[spread_cg4(CG)];
    if (a == 0) {
      // all charge loads in flight at once (channel index clamped, unused
      // channels zeroed when stored)
      const int i = ci[k];
      const float *qs = src.q ? src.q : w.q_a;
#pragma unroll
      for (int c = 0; c < spread_cg4(CG); ++c) qv[c] = qs[int64_t(cg0 + min(c, ncg - 1)) * g.N + i];
    }
    const int d = ((cd[k] >> (10 * a)) & 1023) - kSpreadBias;  // tile-relative window start
    const float r = cf[3 * k + a];
    float *dst = cw + k * S + soff[a];
    const int sa = sz[a];
    for (int x = 0, xx = k % sa; x < sa; ++x) {
      dst[xx] = 0.0f;
      if (++xx == sa) xx = 0;
    }
    const int Ma = g.M[a], Ba = g.B[a];
    unsigned bits = 0;  // 4-point blocks of this axis the window reaches
#pragma unroll
    for (int l = 0; l < P; ++l) {
      int x = d + l;
      if (x < 0) x += Ma;
      if (x >= Ma) x -= Ma;
      if (x < Ba) {
        const float tt = (2.0f * (l + r)) / P - 1.0f;
        // the derivative factor d psi / dt * 2 / P (per grid unit) on the
        // chosen axis (dipole grids of the second derivatives), psi elsewhere
        dst[(a == 2 && !MF) ? (x & 3) * NBZ + (x >> 2) : x] =
            a == src.dax ? win_eval_d(wcf, tt).y * (2.0f / P) : win_eval(wcf, tt);
        bits |= 1u << (x >> 2);
      }
    }
    if constexpr (MF) cbits[4 * k + a] = static_cast<unsigned short>(bits);
    if (a == 0) {
#pragma unroll
      for (int c = 0; c < spread_cg4(CG); c += 4)
        *reinterpret_cast<float4 *>(cq + k * spread_qstride(CG) + c) =
            make_float4(c < ncg ? qv[c] : 0.0f, c + 1 < ncg ? qv[c + 1] : 0.0f, c + 2 < ncg ? qv[c + 2] : 0.0f,
                        c + 3 < ncg ? qv[c + 3] : 0.0f);
    }
  }
  __syncthreads();
  // (2) accumulate: 64 candidates per ballot, scalar walk over the hits
  const int lx = lane >> 4, ly = (lane >> 2) & 3, lz = lane & 3;
  const int xa = (bo[0] + lx) * 4, ya = (soff[1] + bo[1] + ly) * 4, za = (soff[2] + lz * NBZ) * 4;
  if constexpr (MF) {
    // Matrix cores.  Per 64 candidates, each of the wave's blocks gets the
    // list of candidates whose window meets it (from the per-axis block bits
    // of the staging), padded to whole groups of four with the zero row; the
    // groups of all four blocks are walked as one sequence.  A group is one
    // 16x16x4 product per x slice of its block: (16 points of the slice) x
    // (4 hits) weights times (4 hits) x (16 channels) charges; lane l
    // supplies the weight of point l % 16 for hit l / 16 and the charge of
    // channel l % 16 of hit l / 16.  The next group's index and operands are
    // read while the current group's products run.
    const int i16 = lane & 15, kq = lane >> 4;
    unsigned short *hw = hl + __builtin_amdgcn_readfirstlane(tid >> 6) * (kSpreadNBW * kSpreadHitList);
    const unsigned long long below = (1ull << lane) - 1ull;
    const int bxi = bo[0] >> 2, byi = bo[1] >> 2;
    for (int k0 = 0; k0 < ncand; k0 += 64) {
      const int k = k0 + lane;
      const bool valid = wval && k < ncand;
      const uint2 bv = valid ? *reinterpret_cast<const uint2 *>(cbits + 4 * k) : make_uint2(0u, 0u);
      const bool inx = (bv.x >> bxi) & 1u;
      int ng[kSpreadNBW], tot = 0;
#pragma unroll
      for (int j = 0; j < kSpreadNBW; ++j) {
        const bool hit = inx && ((bv.x >> (16 + byi + j / NBZ)) & 1u) && ((bv.y >> (j % NBZ)) & 1u);
        const unsigned long long mj = __ballot(hit);
        const int n = __popcll(mj);
        if (hit) hw[4 * tot + __popcll(mj & below)] = static_cast<unsigned short>(k);
        const int pad = (4 - (n & 3)) & 3;
        if (lane < pad) hw[4 * tot + n + lane] = static_cast<unsigned short>(kSpreadCap);
        ng[j] = (n + 3) >> 2;
        tot += ng[j];
      }
      if (tot == 0) continue;
      // the groups of the four blocks lie one after another in the list;
      // the index of the next group is read one group ahead, and the
      // operand reads of a group overlap the previous group's products
      int t = 0;
      int idx = hw[kq];
      int idxn = tot > 1 ? hw[4 + kq] : kSpreadCap;
#pragma unroll
      for (int j = 0; j < kSpreadNBW; ++j) {
        const int yoff = soff[1] + bo[1] + 4 * (j / NBZ) + (i16 >> 2);
        const int zoff = soff[2] + 4 * (j % NBZ) + (i16 & 3);
        for (int gq = 0; gq < ng[j]; ++gq, ++t) {
          const float *row = cw + __umul24(idx, S);
          const float4 wx4 = *reinterpret_cast<const float4 *>(row + bo[0]);
          const float wyz = row[yoff] * row[zoff];
          const float qv = cq[idx * kSpreadCGM + i16];
          idx = idxn;
          idxn = t + 2 < tot ? hw[4 * (t + 2) + kq] : kSpreadCap;
          accs.v[j][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(wx4.x * wyz, qv, accs.v[j][0], 0, 0, 0);
          accs.v[j][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(wx4.y * wyz, qv, accs.v[j][1], 0, 0, 0);
          accs.v[j][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(wx4.z * wyz, qv, accs.v[j][2], 0, 0, 0);
          accs.v[j][3] = __builtin_amdgcn_mfma_f32_16x16x4f32(wx4.w * wyz, qv, accs.v[j][3], 0, 0, 0);
        }
      }
    }
  } else {
  for (int k0 = 0; k0 < ncand; k0 += 64) {
    const int k = k0 + lane;
    const bool valid = wval && k < ncand;
    const int pk = valid ? cd[k] : 0;
    int dd[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      dd[a] = ((pk >> (10 * a)) & 1023) - kSpreadBias;
      if (dd[a] < 0) dd[a] += g.M[a];
    }
    const bool inx = win_meets(bo[0], 4, dd[0], P, g.M[0]);
    bool iny[CPW], inz[NBZ];
#pragma unroll
    for (int c = 0; c < CPW; ++c) iny[c] = win_meets(bo[1] + 4 * c, 4, dd[1], P, g.M[1]);
#pragma unroll
    for (int z = 0; z < NBZ; ++z) inz[z] = win_meets(4 * z, 4, dd[2], P, g.M[2]);
    unsigned long long m[kSpreadNBW];
    unsigned long long u = 0ull;
#pragma unroll
    for (int j = 0; j < kSpreadNBW; ++j) {
      m[j] = __ballot(valid && inx && iny[j / NBZ] && inz[j % NBZ]);
      u |= m[j];
    }
    if (!u) continue;
    {
    auto &acc = accs.v;
    // software-pipelined walk over the hits, unrolled by two with two
    // register sets: the LDS reads of the next hit are in flight while the
    // current one is accumulated
    float qreg[spread_cg4(CG)];
    {
      const int kq = min(k, ncand - 1);
#pragma unroll
      for (int c = 0; c < spread_cg4(CG); c += 4) {
        const float4 q4 = *reinterpret_cast<const float4 *>(cq + kq * spread_qstride(CG) + c);
        qreg[c] = q4.x;
        qreg[c + 1] = q4.y;
        qreg[c + 2] = q4.z;
        qreg[c + 3] = q4.w;
      }
    }
    // (the loads are unconditional -- past the last hit they re-read the
    // current candidate -- so the wait before each accumulation counts
    // exactly the reads issued after its own)
    SpreadCand<NBZ> ca, cb;
    int ba = spread_take(u), bb = 0;
    spread_load<NBZ>(cw, S, k0 + ba, xa, ya, za, ca);
    while (true) {
      const bool hb = u != 0ull;
      bb = hb ? spread_take(u) : ba;
      spread_load<NBZ>(cw, S, k0 + bb, xa, ya, za, cb);
      spread_accumulate<NBZ, CG>(ca, ba, qreg, m, acc);
      if (!hb) break;
      const bool ha = u != 0ull;
      ba = ha ? spread_take(u) : bb;
      spread_load<NBZ>(cw, S, k0 + ba, xa, ya, za, ca);
      spread_accumulate<NBZ, CG>(cb, bb, qreg, m, acc);
      if (!ha) break;
    }
    }
  }
  }
  __syncthreads();
}

template <int P, int NBZ, int CG>
__device__ __forceinline__ void spread_body(const Geo &g, const Tables &t, const Work &w, int cg0, int ncg, int bx,
                                            const SpreadSrc &src) {
  constexpr int CPW = kSpreadNBW / NBZ;
  extern __shared__ float smem[];
  const int Bx = g.B[0], By = g.B[1], Bz = g.B[2];
  const int sz[3] = {spread_pad4(Bx), spread_pad4(By), spread_pad4(Bz)};
  const int S = sz[0] + sz[1] + sz[2];
  float *cq = smem;                                                 // [cap + 1][CGM]
  const int cap = spread_cap(CG, g.scap);
  float *cw = cq + (cap + 1) * spread_qstride(CG);           // [cap + 1][S]
  float *lf = cw + (cap + 1) * S;                            // [list][3] window offsets delta
  int *ld = reinterpret_cast<int *>(lf + 3 * spread_list(cap));          // [list] packed window starts
  int *li = ld + spread_list(cap);                                       // [list] atom index
  int *rb = li + spread_list(cap);                                       // [cells] first atom of a candidate cell
  int *rs = rb + kSpreadMaxCells;                                   // [cells + 1] prefix of their sizes
  float *wcf = smem + ((int(reinterpret_cast<float *>(rs + kSpreadMaxCells + 1) - smem) + 3) & ~3);  // window coefficients, 16-byte aligned
  unsigned short *cbits = reinterpret_cast<unsigned short *>(wcf + kWinSeg * (kWinDeg + 1));  // [cap][4] block bits per axis
  unsigned short *hl = cbits + 4 * cap;                      // [waves][blocks][68] hit lists
  // (the write-out stage below reuses the cq and cw area)
  __shared__ int wcount[kSpreadScreenPer * (kSpreadThreads / 64)];

  const int tid = threadIdx.x, lane = tid & 63;
  // the zero row past the staged candidates (padding of the hit groups)
  for (int e = tid; e < spread_qstride(CG); e += kSpreadThreads) cq[cap * spread_qstride(CG) + e] = 0.0f;
  for (int e = tid; e < S; e += kSpreadThreads) cw[cap * S + e] = 0.0f;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: keeps block bookkeeping scalar
  const int cell = bx;
  const int cz = cell % g.nc[2], cy = (cell / g.nc[2]) % g.nc[1], cx = cell / (g.nc[2] * g.nc[1]);
  const int t0[3] = {cx * Bx, cy * By, cz * Bz};
  const int ctile[3] = {cx, cy, cz};

  for (int e = tid; e < kWinSeg * (kWinDeg + 1); e += kSpreadThreads) wcf[e] = t.win[e];

  // columns (x, y) of blocks, y fastest; wave w owns columns [CPW w, CPW w + CPW)
  const int nby = sz[1] >> 2, ncol = (sz[0] >> 2) * nby;
  const int col0 = wave * CPW;
  const bool wval = col0 < ncol;
  const int bo[3] = {wval ? (col0 / nby) * 4 : 0, wval ? (col0 % nby) * 4 : 0, 0};
  constexpr bool MF = spread_mfma(CG);
  SpreadAcc<CG> acc;
#pragma unroll
  for (int j = 0; j < kSpreadNBW; ++j) {
    if constexpr (MF) {
#pragma unroll
      for (int sl = 0; sl < 4; ++sl) acc.v[j][sl] = spread_f4{0.0f, 0.0f, 0.0f, 0.0f};
    } else {
#pragma unroll
      for (int c = 0; c < CG; ++c) acc.v[j][c] = 0.0f;
    }
  }

  // candidate cells: this tile's cell and the ones before it along each
  // axis that can hold a window start reaching into the tile.  Their atom
  // ranges (consecutive in the cell-sorted order) are tabulated with a
  // prefix of their sizes, so the whole candidate set is screened with
  // every load of a round in flight at once.
  int ccount[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) ccount[a] = min(min(g.nc[a] - 1, (P - 2) / g.B[a] + 1) + 1, 8);
  const int ncells = ccount[0] * ccount[1] * ccount[2];  // <= kSpreadMaxCells
  for (int ic = tid; ic < ncells; ic += kSpreadThreads) {
    const int iz = ic % ccount[2], iy = (ic / ccount[2]) % ccount[1], ix = ic / (ccount[2] * ccount[1]);
    const int cc = (((ctile[0] - ix + 8 * g.nc[0]) % g.nc[0]) * g.nc[1] + (ctile[1] - iy + 8 * g.nc[1]) % g.nc[1]) *
                       g.nc[2] +
                   (ctile[2] - iz + 8 * g.nc[2]) % g.nc[2];
    rb[ic] = w.cell_start[cc];
    rs[ic + 1] = w.cell_start[cc + 1] - w.cell_start[cc];
  }
  __syncthreads();
  if (tid == 0) {
    int acc_n = 0;
    rs[0] = 0;
    for (int ic = 0; ic < ncells; ++ic) {
      acc_n += rs[ic + 1];
      rs[ic + 1] = acc_n;
    }
  }
  __syncthreads();
  const int total = rs[ncells];

  // rounds of up to kSpreadScreenPer atoms per thread: screened candidates
  // are appended to the list in screening order (deterministic); the list
  // is flushed cap candidates at a time
  int nlist = 0, c0 = 0;
  for (int base = 0; base < total || c0 < nlist; base += kSpreadScreenPer * kSpreadThreads) {
    if (base < total) {
      float4 rr[kSpreadScreenPer];
      int ai[kSpreadScreenPer];
#pragma unroll
      for (int j = 0; j < kSpreadScreenPer; ++j) {
        const int e = base + tid + j * kSpreadThreads;
        int i = -1;
        if (e < total) {
          int lo = 0, hi = ncells;  // rs[lo] <= e < rs[hi]
          while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (rs[mid] <= e) lo = mid;
            else hi = mid;
          }
          i = rb[lo] + (e - rs[lo]);
        }
        ai[j] = i;
        rr[j] = i >= 0 ? reinterpret_cast<const float4 *>(w.rec_a)[i] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
      unsigned long long mk[kSpreadScreenPer];
      int dk[kSpreadScreenPer];
#pragma unroll
      for (int j = 0; j < kSpreadScreenPer; ++j) {
        bool ok = ai[j] >= 0;
        int pk = 0;
        const unsigned pn = __float_as_uint(rr[j].w);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          int dd = unpack_n0(pn, a) - t0[a];
          if (dd < 0) dd += g.M[a];
          const bool in = dd < g.B[a];
          ok = ok && (in || dd > g.M[a] - P);
          pk |= ((in ? dd : dd - g.M[a]) + kSpreadBias) << (10 * a);
        }
        dk[j] = ok ? pk : -1;
        mk[j] = __ballot(ok);
        if (lane == 0) wcount[j * (kSpreadThreads / 64) + wave] = __popcll(mk[j]);
      }
      __syncthreads();
      // slot = list length + candidates of earlier parts j' < j of this
      // round + those of earlier waves in part j
      int before = nlist;
#pragma unroll
      for (int j = 0; j < kSpreadScreenPer; ++j) {
        int off = before;
        for (int wq = 0; wq < wave; ++wq) off += wcount[j * (kSpreadThreads / 64) + wq];
        if (dk[j] >= 0) {
          const int slot = off + __popcll(mk[j] & ((1ull << lane) - 1ull));
          ld[slot] = dk[j];
          lf[3 * slot] = rr[j].x;
          lf[3 * slot + 1] = rr[j].y;
          lf[3 * slot + 2] = rr[j].z;
          li[slot] = ai[j];
        }
        for (int wq = 0; wq < kSpreadThreads / 64; ++wq) before += wcount[j * (kSpreadThreads / 64) + wq];
      }
      nlist = before;
      __syncthreads();
    }
    const bool last = base + kSpreadScreenPer * kSpreadThreads >= total;
    while (nlist - c0 >= cap || (last && c0 < nlist)) {
      const int n = min(cap, nlist - c0);
      spread_flush<P, NBZ, CG>(g, w, cg0, ncg, n, sz, cq, cw, ld + c0, lf + 3 * c0, li + c0, wcf, bo, wval, cbits, hl,
                               acc, src);
      c0 += n;
    }
    // keep the unflushed tail (fewer than cap <= threads entries)
    // at the front of the list
    if (c0 > 0) {
      const int rem = nlist - c0;
      int dv = 0, iv = 0;
      float f0 = 0.f, f1 = 0.f, f2 = 0.f;
      if (tid < rem) {
        dv = ld[c0 + tid];
        iv = li[c0 + tid];
        f0 = lf[3 * (c0 + tid)];
        f1 = lf[3 * (c0 + tid) + 1];
        f2 = lf[3 * (c0 + tid) + 2];
      }
      __syncthreads();
      if (tid < rem) {
        ld[tid] = dv;
        li[tid] = iv;
        lf[3 * tid] = f0;
        lf[3 * tid + 1] = f1;
        lf[3 * tid + 2] = f2;
      }
      nlist = rem;
      c0 = 0;
      __syncthreads();
    }
  }

  // write the tile through LDS, several channels per pass, as coalesced
  // rows; every grid value belongs to exactly one tile.  A thread moves the
  // same (x, y, z) element(s) of every channel.
  float *stage = smem;  // reuses the candidate area
  const int nt = Bx * By * Bz;
  const int cpp = max(1, min(ncg, spread_stage_floats(S, CG, cap) / nt));
  const bool vec = (Bz & 3) == 0;
  const int epr = vec ? 4 : 1;                       // floats per element
  const int nel = nt / epr;                          // elements per channel
  int goff[kSpreadOutMax], soffs[kSpreadOutMax];
#pragma unroll
  for (int r = 0; r < kSpreadOutMax; ++r) {
    const int el = tid + r * kSpreadThreads;
    const int f = min(el, nel - 1) * epr;            // first float of the element in the tile
    const int x = f / (By * Bz), rem = f - x * (By * Bz), y = rem / Bz, z = rem - y * Bz;
    goff[r] = el < nel ? ((t0[0] + x) * g.M[1] + t0[1] + y) * g.M[2] + t0[2] + z : -1;
    soffs[r] = f;
  }
  const int64_t chan = int64_t(g.M[0]) * g.M[1] * g.M[2];
  const int lx = lane >> 4, ly = (lane >> 2) & 3, lz = lane & 3;
  for (int c0 = 0; c0 < ncg; c0 += cpp) {
    const int nc = min(cpp, ncg - c0);
    if (wval) {
      if constexpr (MF) {
        // lane: channel lane % 16, row y = lane / 16 of the slice, z = 0..3
        const int ch = (lane & 15) - c0, y0 = lane >> 4;
        if (ch >= 0 && ch < nc) {
#pragma unroll
          for (int j = 0; j < kSpreadNBW; ++j) {
            const int y = bo[1] + 4 * (j / NBZ) + y0, z0 = 4 * (j % NBZ);
#pragma unroll
            for (int sl = 0; sl < 4; ++sl) {
              const int x = bo[0] + sl;
              if (x < Bx && y < By) {
                float *dst = stage + ch * nt + (x * By + y) * Bz + z0;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                  if (z0 + r < Bz) dst[r] = acc.v[j][sl][r];
              }
            }
          }
        }
      } else {
#pragma unroll
        for (int j = 0; j < kSpreadNBW; ++j) {
          const int x = bo[0] + lx, y = bo[1] + 4 * (j / NBZ) + ly, z = 4 * (j % NBZ) + lz;
          if (x < Bx && y < By && z < Bz) {
            float *dst = stage + (x * By + y) * Bz + z;
#pragma unroll
            for (int cc = 0; cc < CG; ++cc)
              if (cc >= c0 && cc < c0 + nc) dst[(cc - c0) * nt] = acc.v[j][cc];
          }
        }
      }
    }
    __syncthreads();
    for (int c = 0; c < nc; ++c) {
      float *gch = w.grid + int64_t(cg0 + c0 + c) * chan;
      const float *sch = stage + c * nt;
#pragma unroll
      for (int r = 0; r < kSpreadOutMax; ++r) {
        if (goff[r] < 0) continue;
        if (vec) {
          float4 v = *reinterpret_cast<const float4 *>(sch + soffs[r]);
          if (src.acc) {
            const float4 o = *reinterpret_cast<const float4 *>(gch + goff[r]);
            v = make_float4(v.x + o.x, v.y + o.y, v.z + o.z, v.w + o.w);
          }
          st_stream(reinterpret_cast<float4 *>(gch + goff[r]), v);
        } else {
          gch[goff[r]] = src.acc ? sch[soffs[r]] + gch[goff[r]] : sch[soffs[r]];
        }
      }
    }
    __syncthreads();
  }
}

// CG: channel accumulators per point (2, 4 or 12); a launch covers ncg <= CG
template <int P, int NBZ, int CG>
__global__ __launch_bounds__(kSpreadThreads, 4) void k_spread(Geo g, Tables t, Work w, int cg0, int ncg, SpreadSrc src) {
  spread_body<P, NBZ, CG>(g, t, w, cg0, ncg, blockIdx.x, src);
}

// ---------------------------------------------------------------------------
// z R2C on the register FFT: 32 lines of Nz = 128 per workgroup, 8 threads
// per line (one wave holds 8 whole lines, so the exchanges are wave-local).
__device__ __forceinline__ void zfwd_reg(const Geo &g, const Tables &t, const Work &w, int64_t nlines_total, int bx) {
  extern __shared__ float smem[];
  constexpr int Nz = 128;
  float2 *ex = reinterpret_cast<float2 *>(smem);
  float2 *tw = ex + 32 * kZregLine;
  float2 *twr = tw + Nz;
  const int tid = threadIdx.x, j = tid & 7, l = tid >> 3;
  const int64_t line0 = int64_t(bx) * 32;
  const bool on = line0 + l < nlines_total;
  const float2 *src = reinterpret_cast<const float2 *>(w.grid) + (line0 + l) * Nz + j;
  float2 v[16];
#pragma unroll
  for (int n1 = 0; n1 < 16; ++n1) v[n1] = on ? src[8 * n1] : make_float2(0.f, 0.f);
  for (int e = tid; e < Nz; e += PSWF_THREADS) tw[e] = reinterpret_cast<const float2 *>(t.tw_z)[e];
  for (int e = tid; e <= Nz; e += PSWF_THREADS) twr[e] = reinterpret_cast<const float2 *>(t.tw_zr)[e];
  __syncthreads();
  float2 *xl = ex + l * kZregLine;
  rfft_inner<16, -1>(v, j, tw);
#pragma unroll
  for (int k1 = 0; k1 < 16; ++k1) xl[k1 * 9 + j] = v[k1];
  wave_sync();
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int n2 = 0; n2 < 8; ++n2) v[q * 8 + n2] = xl[(j + 8 * q) * 9 + n2];
  rfft_outer<16, 8, -1>(v);
  wave_sync();
  // natural order for the real-to-complex split
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) xl[j + 8 * q + 16 * k2] = v[q * 8 + k2];
  wave_sync();
  if (!on) return;
  float2 *dst = reinterpret_cast<float2 *>(w.s1) + (line0 + l) * g.KZP;
  for (int k = j; k < g.KZ; k += 8) {
    const float2 zk = xl[k == Nz ? 0 : k];
    const float2 zc = xl[(Nz - k) & (Nz - 1)];
    // E = (Z_k + conj Z_{N-k}) / 2, O = (Z_k - conj Z_{N-k}) / (2i)
    const float2 E = make_float2(0.5f * (zk.x + zc.x), 0.5f * (zk.y - zc.y));
    const float2 O = make_float2(0.5f * (zk.y + zc.y), -0.5f * (zk.x - zc.x));
    st_stream(&dst[k], cadd(E, cmul(twr[k], O)));
  }
}

// z R2C (step ii, first axis): lines of M_z reals -> KZ complex columns.
// The real line is packed as z_n = x_2n + i x_2n+1, transformed with length
// Nz = M_z / 2 and split: X_k = E_k + exp(-2 pi i k / M_z) O_k.
__device__ __forceinline__ void zfwd_body(const Geo &g, const Tables &t, const FftAxis &ax, const Work &w, int64_t nlines_total, int bx) {
  extern __shared__ float smem[];
  const int L = g.zlines, ld = L + 1, Nz = g.Nz;
  int llog = 0;
  while ((1 << llog) < L) ++llog;
  float2 *buf = reinterpret_cast<float2 *>(smem);
  float2 *tw = buf + Nz * ld;
  float2 *twr = tw + Nz;
  const int tid = threadIdx.x;
  const int64_t line0 = int64_t(bx) * L;
  const int nl = int(min(int64_t(L), nlines_total - line0));
  for (int e = tid; e < Nz; e += PSWF_THREADS) tw[e] = reinterpret_cast<const float2 *>(t.tw_z)[e];
  for (int e = tid; e <= Nz; e += PSWF_THREADS) twr[e] = reinterpret_cast<const float2 *>(t.tw_zr)[e];
  const float2 *src = reinterpret_cast<const float2 *>(w.grid) + line0 * Nz;
  staged16(
      L * Nz,
      [&](int e) { return fdiv(e, g.div_nz) < nl ? src[e] : make_float2(0.f, 0.f); },
      [&](int e, float2 v) {
        const int line = fdiv(e, g.div_nz), n = e - line * Nz;
        buf[n * ld + line] = v;
      });
  __syncthreads();
  lds_fft<-1, 16>(buf, ax, llog - 2, ld, tw, tid);
  __syncthreads();
  float2 *dst = reinterpret_cast<float2 *>(w.s1) + line0 * g.KZP;
  for (int e = tid; e < nl * g.KZ; e += PSWF_THREADS) {
    const int line = fdiv(e, g.div_kz), k = e - line * g.KZ;
    const float2 zk = buf[(k == Nz ? 0 : k) * ld + line];
    const int km = (Nz - k) % Nz;
    const float2 zc = buf[(km < 0 ? km + Nz : km) * ld + line];
    // E = (Z_k + conj Z_{N-k}) / 2, O = (Z_k - conj Z_{N-k}) / (2i)
    const float2 E = make_float2(0.5f * (zk.x + zc.x), 0.5f * (zk.y - zc.y));
    const float2 O = make_float2(0.5f * (zk.y + zc.y), -0.5f * (zk.x - zc.x));
    dst[line * g.KZP + k] = cadd(E, cmul(twr[k], O));
  }
}

// REG: the register FFT path (the planner's 256-point geometry)
template <bool REG>
__global__ __launch_bounds__(PSWF_THREADS) void k_zfwd(Geo g, Tables t, FftAxis ax, Work w, int64_t nlines_total) {
  if (REG)
    zfwd_reg(g, t, w, nlines_total, blockIdx.x);
  else
    zfwd_body(g, t, ax, w, nlines_total, blockIdx.x);
}

// y forward on the register FFT (M_y = 256, 16 columns per workgroup):
// thread (col, j) loads rows 16 n1 + j of its column; the exchange crosses
// waves, so it is a workgroup barrier.
__device__ __forceinline__ void yfwd_reg(const Geo &g, const Tables &t, const Work &w, int bx, int by) {
  extern __shared__ float smem[];
  float2 *ex = reinterpret_cast<float2 *>(smem);  // [k1][n2][col]
  float2 *tw = ex + 256 * 16;
  const int tid = threadIdx.x, col = tid & 15, j = tid >> 4;
  const int kz0 = bx * 16;
  const int64_t plane = by;
  const bool on = kz0 + col < g.KZ;
  const float2 *src = reinterpret_cast<const float2 *>(w.s1) + plane * 256 * g.KZP + kz0 + col;
  float2 v[16];
#pragma unroll
  for (int n1 = 0; n1 < 16; ++n1) v[n1] = on ? src[int64_t(16 * n1 + j) * g.KZP] : make_float2(0.f, 0.f);
  tw[tid] = reinterpret_cast<const float2 *>(t.tw_y)[tid];
  __syncthreads();
  rfft_inner<16, -1>(v, j, tw);
#pragma unroll
  for (int k1 = 0; k1 < 16; ++k1) ex[(k1 * 16 + j) * 16 + col] = v[k1];
  __syncthreads();
#pragma unroll
  for (int n2 = 0; n2 < 16; ++n2) v[n2] = ex[(j * 16 + n2) * 16 + col];
  rfft_outer<16, 16, -1>(v);
  if (!on) return;
  // v[k2] = X[j + 16 k2]; keep |f_y| <= FY
  float2 *dst = reinterpret_cast<float2 *>(w.s2) + plane * g.NY * g.KZP + kz0 + col;
#pragma unroll
  for (int k2 = 0; k2 < 16; ++k2) {
    const int k = j + 16 * k2;
    if (k <= g.FY) st_stream(&dst[int64_t(k) * g.KZP], v[k2]);
    else if (k >= 256 - g.FY) st_stream(&dst[int64_t(k - 256 + g.NY) * g.KZP], v[k2]);
  }
}

// y forward (step ii, second axis): plane (c, x), a block of kb z columns;
// keeps only |f_y| <= FY.
__device__ __forceinline__ void yfwd_body(const Geo &g, const Tables &t, const FftAxis &ax, const Work &w, int bx, int by) {
  extern __shared__ float smem[];
  const int kb = g.kby, ld = kb + 1, My = g.M[1];
  float2 *buf = reinterpret_cast<float2 *>(smem);
  float2 *tw = buf + My * ld;
  const int tid = threadIdx.x;
  const int kz0 = bx * g.kzq;
  const int64_t plane0 = int64_t(by) * g.ypl;  // planes c * Mx + x
  const int64_t nplane = int64_t(g.C) * g.M[0];
  // column j: plane plane0 + (j >> kzq_log2), k_z = kz0 + (j & (kzq - 1))
  auto col_ok = [&](int j) {
    return kz0 + (j & (g.kzq - 1)) < g.KZ && plane0 + (j >> g.kzq_log2) < nplane;
  };
  auto col_off = [&](int j, int64_t rows) {
    return (plane0 + (j >> g.kzq_log2)) * rows * g.KZP + kz0 + (j & (g.kzq - 1));
  };
  for (int e = tid; e < My; e += PSWF_THREADS) tw[e] = reinterpret_cast<const float2 *>(t.tw_y)[e];
  const float2 *src = reinterpret_cast<const float2 *>(w.s1);
  staged16(
      My * kb,
      [&](int e) {
        const int y = e >> g.kby_log2, col = e & (kb - 1);
        return col_ok(col) ? src[col_off(col, My) + int64_t(y) * g.KZP] : make_float2(0.f, 0.f);
      },
      [&](int e, float2 v) { buf[(e >> g.kby_log2) * ld + (e & (kb - 1))] = v; });
  __syncthreads();
  lds_fft<-1, 16>(buf, ax, g.kby_log2 - 2, ld, tw, tid);
  __syncthreads();
  float2 *dst = reinterpret_cast<float2 *>(w.s2);
  for (int e = tid; e < g.NY * kb; e += PSWF_THREADS) {
    const int iy = e >> g.kby_log2, col = e & (kb - 1);
    if (!col_ok(col)) continue;
    const int my = iy <= g.FY ? iy : My - g.NY + iy;
    dst[col_off(col, g.NY) + int64_t(iy) * g.KZP] = buf[my * ld + col];
  }
}

// REG: the register FFT path (the planner's 256-point geometry)
template <bool REG>
__global__ __launch_bounds__(PSWF_THREADS) void k_yfwd(Geo g, Tables t, FftAxis ax, Work w) {
  if (REG) {
    // consecutive column blocks of a plane on one XCD
    const int2 m = xcd_contiguous_2d();
    yfwd_reg(g, t, w, m.x, m.y);
  } else {
    yfwd_body(g, t, ax, w, blockIdx.x, blockIdx.y);
  }
}

// Fourier kernel at kappa: (Phi, Phi'/k) from the per-channel polynomials.
__device__ __forceinline__ float kpow(float kap, float inv, int e) {
  float r = 1.0f;
  if (e >= 0) {
    for (int i = 0; i < e; ++i) r *= kap;
  } else {
    for (int i = 0; i < -e; ++i) r *= inv;
  }
  return r;
}
__device__ __forceinline__ float2 kernel_eval(const float *fc, const float *gc, const KChan &kc, float kap) {
  float y = kap * kKerSeg;
  int s = min(int(y), kKerSeg - 1);
  float tau = 2.0f * (y - s) - 1.0f;
  // both coefficient sets of the segment as 16-byte loads (tables 16-byte
  // aligned), all in flight before the Horner chains
  static_assert(kKerDeg + 1 == 12, "kernel segments are read as three float4");
  float a[12], b[12];
  win_coef(fc, s, a);
  win_coef(gc, s, b);
  float fv = a[kKerDeg], gv = b[kKerDeg];
#pragma unroll
  for (int d = kKerDeg - 1; d >= 0; --d) {
    fv = fmaf(fv, tau, a[d]);
    gv = fmaf(gv, tau, b[d]);
  }
  const float inv = 1.0f / kap;
  float phi = kc.A * kpow(kap, inv, kc.eA) * fv;
  float dph = kc.Cc * kpow(kap, inv, kc.eC) * gv;
  if (kc.B != 0.0f || kc.D != 0.0f) {
    const float lg = logf(kap);
    phi += kc.B * kpow(kap, inv, kc.eB) * lg;
    dph += kc.D * kpow(kap, inv, kc.eD) * lg;
  }
  return make_float2(phi, dph);
}

// Fused x pass on the register FFT (M_x = 256, 16 columns per workgroup).
// The forward transform leaves thread (col, j) with X[j + 16 k2], which is
// both where the multiply needs it and the input layout of the inverse.
__device__ __forceinline__ void xmul_reg(const Geo &g, const Tables &t, const Work &w, int mode, const double *__restrict__ grad, int bx, int by) {
  extern __shared__ float smem[];
  float2 *ex = reinterpret_cast<float2 *>(smem);  // [k1][n2][col]
  float2 *tw = ex + 256 * 16;
  float *fc = reinterpret_cast<float *>(tw + 256);
  float *gc = fc + kKerCoef;
  __shared__ double red[7][PSWF_THREADS / 64];
  const int tid = threadIdx.x, col = tid & 15, j = tid >> 4;
  const int blk = bx, c = by;
  const int run = t.xgrp[blk];  // one run per block on this path
  const int iy = t.xblk[4 * run], kz0 = t.xblk[4 * run + 1], ncol = t.xblk[4 * run + 2];
  const bool on = col < ncol;
  const int64_t xstride = int64_t(g.NY) * g.KZP;
  float2 *col0 = reinterpret_cast<float2 *>(w.s2) + int64_t(c) * 256 * xstride + int64_t(iy) * g.KZP + kz0 + col;
  float2 v[16];
#pragma unroll
  for (int n1 = 0; n1 < 16; ++n1) v[n1] = on ? col0[(16 * n1 + j) * xstride] : make_float2(0.f, 0.f);
  const KChan kc = t.kch[c];
  tw[tid] = reinterpret_cast<const float2 *>(t.tw_x)[tid];
  for (int e = tid; e < kKerCoef; e += PSWF_THREADS) {
    fc[e] = t.kf[c * kKerCoef + e];
    gc[e] = t.kg[c * kKerCoef + e];
  }
  __syncthreads();
  rfft_inner<16, -1>(v, j, tw);
#pragma unroll
  for (int k1 = 0; k1 < 16; ++k1) ex[(k1 * 16 + j) * 16 + col] = v[k1];
  __syncthreads();
#pragma unroll
  for (int n2 = 0; n2 < 16; ++n2) v[n2] = ex[(j * 16 + n2) * 16 + col];
  rfft_outer<16, 16, -1>(v);

  const int fy = iy <= g.FY ? iy : iy - g.NY;
  const float dy = t.Dy[iy];
  const int kz = kz0 + col;
  // k = 2 pi H^-1 m: the column's (m_y, m_z) part, then m_x per mode
  const float cyx = fmaf(g.kmat[1], float(fy), g.kmat[2] * kz);
  const float cyy = fmaf(g.kmat[4], float(fy), g.kmat[5] * kz);
  const float cyz = fmaf(g.kmat[7], float(fy), g.kmat[8] * kz);
  const float dyz = on ? dy * t.Dz[kz] : 0.0f;
  const float wz = (kz == 0) ? 1.0f : 2.0f;
  const float scale = (mode == 2 ? float(grad[c]) : 1.0f) * g.invV;
  float acc[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k2 = 0; k2 < 16; ++k2) {
    const int mx = j + 16 * k2;
    const int fx = mx <= 128 ? mx : mx - 256;
    const float kx = fmaf(g.kmat[0], float(fx), cyx);
    const float ky = fmaf(g.kmat[3], float(fx), cyy);
    const float kzv = fmaf(g.kmat[6], float(fx), cyz);
    const float k2v = kx * kx + ky * ky + kzv * kzv;
    float mult = 0.0f;
    if (on && k2v > 0.0f && k2v <= g.kc2 && mx != 128) {
      const float k = sqrtf(k2v);
      const float2 ph = kernel_eval(fc, gc, kc, k * g.kinv);
      const float D = t.Dx[mx] * dyz;
      const float s2 = (v[k2].x * v[k2].x + v[k2].y * v[k2].y) * D * wz;
      acc[0] += ph.x * s2;
      const float vd = ph.y * s2;
      acc[1] += vd * kx * kx;
      acc[2] += vd * ky * ky;
      acc[3] += vd * kzv * kzv;
      acc[4] += vd * kx * ky;
      acc[5] += vd * kx * kzv;
      acc[6] += vd * ky * kzv;
      mult = ph.x * D * scale;
    }
    v[k2] = cscale(v[k2], mult);
  }
  // block reduction in FP64, fixed order
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    double d = double(acc[i]);
    for (int off = 32; off > 0; off >>= 1) d += __shfl_down(d, off, 64);
    if (lane == 0) red[i][wave] = d;
  }
  __syncthreads();
  if (tid < 7) {
    double sum = 0.0;
    for (int k = 0; k < PSWF_THREADS / 64; ++k) sum += red[tid][k];
    w.epart[(int64_t(c) * g.nxblk + blk) * 8 + tid] = sum;
  }
  if (mode == 0) return;
  rfft_inner<16, 1>(v, j, tw);
#pragma unroll
  for (int k1 = 0; k1 < 16; ++k1) ex[(k1 * 16 + j) * 16 + col] = v[k1];
  __syncthreads();
#pragma unroll
  for (int n2 = 0; n2 < 16; ++n2) v[n2] = ex[(j * 16 + n2) * 16 + col];
  rfft_outer<16, 16, 1>(v);
  if (!on) return;
#pragma unroll
  for (int k2 = 0; k2 < 16; ++k2) st_stream(&col0[(j + 16 * k2) * xstride], v[k2]);
}

// Fused x pass (steps ii-iv and the first inverse axis): x transform of one
// block of (f_y, k_z) columns, diagonal scaling by Phi_p h^6 / What^2 / V,
// FP64 block partials of the energy and virial, inverse x transform.
// mode 0: energy only (no write-back), 1: full, 2: adjoint with the scale
// grad[c] folded into the kernel.
__device__ __forceinline__ void xmul_body(const Geo &g, const Tables &t, const FftAxis &ax, const Work &w, int mode, const double *__restrict__ grad, int bx, int by) {
  extern __shared__ float smem[];
  const int kb = g.kbx, ld = kb + 1, Mx = g.M[0];
  float2 *buf = reinterpret_cast<float2 *>(smem);
  float2 *tw = buf + Mx * ld;
  float *fc = reinterpret_cast<float *>(tw + Mx + ((Mx * ld + Mx) & 1));  // 16-byte aligned
  float *gc = fc + kKerCoef;
  __shared__ double red[7][PSWF_THREADS / 64];
  __shared__ int ciy[64], ckz[64];  // k_y row and k_z of each column of the block
  const int tid = threadIdx.x;
  const int blk = bx, c = by;
  const int r0 = t.xgrp[blk], r1 = t.xgrp[blk + 1];
  const int ncol = t.xblk[4 * (r1 - 1) + 3] + t.xblk[4 * (r1 - 1) + 2];
  for (int r = r0 + tid; r < r1; r += PSWF_THREADS) {
    const int iy = t.xblk[4 * r], kz0 = t.xblk[4 * r + 1], n = t.xblk[4 * r + 2], o = t.xblk[4 * r + 3];
    for (int j = 0; j < n; ++j) {
      ciy[o + j] = iy;
      ckz[o + j] = kz0 + j;
    }
  }
  const KChan kc = t.kch[c];
  for (int e = tid; e < Mx; e += PSWF_THREADS) tw[e] = reinterpret_cast<const float2 *>(t.tw_x)[e];
  for (int e = tid; e < kKerCoef; e += PSWF_THREADS) {
    fc[e] = t.kf[c * kKerCoef + e];
    gc[e] = t.kg[c * kKerCoef + e];
  }
  __syncthreads();
  const int64_t xstride = int64_t(g.NY) * g.KZP;
  float2 *chan0 = reinterpret_cast<float2 *>(w.s2) + int64_t(c) * Mx * xstride;
  staged16(
      Mx * kb,
      [&](int e) {
        const int x = e >> g.kbx_log2, col = e & (kb - 1);
        return col < ncol ? chan0[x * xstride + int64_t(ciy[col]) * g.KZP + ckz[col]] : make_float2(0.f, 0.f);
      },
      [&](int e, float2 v) { buf[(e >> g.kbx_log2) * ld + (e & (kb - 1))] = v; });
  __syncthreads();
  lds_fft<-1, 16>(buf, ax, g.kbx_log2 - 2, ld, tw, tid);
  __syncthreads();

  const float scale = (mode == 2 ? float(grad[c]) : 1.0f) * g.invV;
  float acc[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int e = tid; e < Mx * kb; e += PSWF_THREADS) {
    const int mx = e >> g.kbx_log2, col = e & (kb - 1);
    float2 v = buf[mx * ld + col];
    float mult = 0.0f;
    if (col < ncol) {
      const int iy = ciy[col], kz = ckz[col];
      const int fy = iy <= g.FY ? iy : iy - g.NY;
      const int fx = mx <= Mx / 2 ? mx : mx - Mx;
      // k = 2 pi H^-1 m
      const float kx = fmaf(g.kmat[0], float(fx), fmaf(g.kmat[1], float(fy), g.kmat[2] * kz));
      const float ky = fmaf(g.kmat[3], float(fx), fmaf(g.kmat[4], float(fy), g.kmat[5] * kz));
      const float kzv = fmaf(g.kmat[6], float(fx), fmaf(g.kmat[7], float(fy), g.kmat[8] * kz));
      const float k2 = kx * kx + ky * ky + kzv * kzv;
      if (k2 > 0.0f && k2 <= g.kc2 && 2 * abs(fx) != Mx) {
        const float k = sqrtf(k2);
        const float2 ph = kernel_eval(fc, gc, kc, k * g.kinv);
        const float D = t.Dx[mx] * t.Dy[iy] * t.Dz[kz];
        const float wz = (kz == 0) ? 1.0f : 2.0f;
        const float s2 = (v.x * v.x + v.y * v.y) * D * wz;
        acc[0] += ph.x * s2;
        const float vd = ph.y * s2;
        acc[1] += vd * kx * kx;
        acc[2] += vd * ky * ky;
        acc[3] += vd * kzv * kzv;
        acc[4] += vd * kx * ky;
        acc[5] += vd * kx * kzv;
        acc[6] += vd * ky * kzv;
        mult = ph.x * D * scale;
      }
    }
    buf[mx * ld + col] = cscale(v, mult);
  }
  // block reduction in FP64, fixed order
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    double v = double(acc[i]);
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[i][wave] = v;
  }
  __syncthreads();
  if (tid < 7) {
    double sum = 0.0;
    for (int k = 0; k < PSWF_THREADS / 64; ++k) sum += red[tid][k];
    w.epart[(int64_t(c) * g.nxblk + blk) * 8 + tid] = sum;
  }
  if (mode == 0) return;
  lds_fft<1, 16>(buf, ax, g.kbx_log2 - 2, ld, tw, tid);
  __syncthreads();
  for (int e = tid; e < Mx * kb; e += PSWF_THREADS) {
    const int x = e >> g.kbx_log2, col = e & (kb - 1);
    if (col < ncol) chan0[x * xstride + int64_t(ciy[col]) * g.KZP + ckz[col]] = buf[x * ld + col];
  }
}

// REG: the register FFT path (the planner's 256-point geometry)
template <bool REG>
__global__ __launch_bounds__(PSWF_THREADS, REG ? 4 : 1) void k_xmul(Geo g, Tables t, FftAxis ax, Work w, int mode,
                                                        const double *__restrict__ grad) {
  if (REG)
    xmul_reg(g, t, w, mode, grad, blockIdx.x, blockIdx.y);
  else
    xmul_body(g, t, ax, w, mode, grad, blockIdx.x, blockIdx.y);
}

// inverse y on the register FFT (M_y = 256, 16 columns per workgroup)
__device__ __forceinline__ void yinv_reg(const Geo &g, const Tables &t, const Work &w, int bx, int by) {
  extern __shared__ float smem[];
  float2 *ex = reinterpret_cast<float2 *>(smem);  // [k1][n2][col]
  float2 *tw = ex + 256 * 16;
  const int tid = threadIdx.x, col = tid & 15, j = tid >> 4;
  const int kz0 = bx * 16;
  const int64_t plane = by;
  const int kz = kz0 + col;
  const bool on = kz < g.KZ;
  const float2 *src = reinterpret_cast<const float2 *>(w.s2) + plane * g.NY * g.KZP + kz;
  // row m = 16 n1 + j holds f_y = m (m <= FY) or m - 256 (m >= 256 - FY),
  // stored at iy = m or m - 256 + NY; the other rows are zero
  float2 v[16];
#pragma unroll
  for (int n1 = 0; n1 < 16; ++n1) {
    const int m = 16 * n1 + j;
    const int iy = m <= g.FY ? m : m - 256 + g.NY;
    const bool kept = on && (m <= g.FY || m >= 256 - g.FY);
    v[n1] = kept ? src[int64_t(iy) * g.KZP] : make_float2(0.f, 0.f);
  }
  tw[tid] = reinterpret_cast<const float2 *>(t.tw_y)[tid];
  // columns the x pass skipped (k_z >= blim) still hold forward data
#pragma unroll
  for (int n1 = 0; n1 < 16; ++n1) {
    const int m = 16 * n1 + j;
    const int iy = m <= g.FY ? m : m - 256 + g.NY;
    if ((m <= g.FY || m >= 256 - g.FY) && kz >= t.blim[iy]) v[n1] = make_float2(0.f, 0.f);
  }
  __syncthreads();
  rfft_inner<16, 1>(v, j, tw);
#pragma unroll
  for (int k1 = 0; k1 < 16; ++k1) ex[(k1 * 16 + j) * 16 + col] = v[k1];
  __syncthreads();
#pragma unroll
  for (int n2 = 0; n2 < 16; ++n2) v[n2] = ex[(j * 16 + n2) * 16 + col];
  rfft_outer<16, 16, 1>(v);
  if (!on) return;
  float2 *dst = reinterpret_cast<float2 *>(w.s1) + plane * 256 * g.KZP + kz;
#pragma unroll
  for (int k2 = 0; k2 < 16; ++k2) st_stream(&dst[int64_t(j + 16 * k2) * g.KZP], v[k2]);
}

// inverse y: kept rows (zero elsewhere and for columns the x pass skipped)
__device__ __forceinline__ void yinv_body(const Geo &g, const Tables &t, const FftAxis &ax, const Work &w, int bx, int by) {
  extern __shared__ float smem[];
  const int kb = g.kby, ld = kb + 1, My = g.M[1];
  float2 *buf = reinterpret_cast<float2 *>(smem);
  float2 *tw = buf + My * ld;
  const int tid = threadIdx.x;
  const int kz0 = bx * g.kzq;
  const int64_t plane0 = int64_t(by) * g.ypl;
  const int64_t nplane = int64_t(g.C) * g.M[0];
  auto col_ok = [&](int j) {
    return kz0 + (j & (g.kzq - 1)) < g.KZ && plane0 + (j >> g.kzq_log2) < nplane;
  };
  auto col_off = [&](int j, int64_t rows) {
    return (plane0 + (j >> g.kzq_log2)) * rows * g.KZP + kz0 + (j & (g.kzq - 1));
  };
  for (int e = tid; e < My; e += PSWF_THREADS) tw[e] = reinterpret_cast<const float2 *>(t.tw_y)[e];
  // rows |f_y| > FY are zero; the kept rows are all loaded below
  const int ngap = My - g.NY;
  for (int e = tid; e < ngap * kb; e += PSWF_THREADS)
    buf[(g.FY + 1 + (e >> g.kby_log2)) * ld + (e & (kb - 1))] = make_float2(0.f, 0.f);
  const float2 *src = reinterpret_cast<const float2 *>(w.s2);
  // the loads do not wait for the column limits: columns the x pass skipped
  // (k_z >= blim) still hold forward data and are masked after the load
  staged16(
      g.NY * kb,
      [&](int e) {
        const int iy = e >> g.kby_log2, col = e & (kb - 1);
        return col_ok(col) ? src[col_off(col, g.NY) + int64_t(iy) * g.KZP] : make_float2(0.f, 0.f);
      },
      [&](int e, float2 v) {
        const int iy = e >> g.kby_log2, col = e & (kb - 1);
        const int my = iy <= g.FY ? iy : My - g.NY + iy;
        buf[my * ld + col] = kz0 + (col & (g.kzq - 1)) < t.blim[iy] ? v : make_float2(0.f, 0.f);
      });
  __syncthreads();
  lds_fft<1, 16>(buf, ax, g.kby_log2 - 2, ld, tw, tid);
  __syncthreads();
  float2 *dst = reinterpret_cast<float2 *>(w.s1);
  for (int e = tid; e < My * kb; e += PSWF_THREADS) {
    const int y = e >> g.kby_log2, col = e & (kb - 1);
    if (col_ok(col)) dst[col_off(col, My) + int64_t(y) * g.KZP] = buf[y * ld + col];
  }
}

// REG: the register FFT path (the planner's 256-point geometry)
template <bool REG>
__global__ __launch_bounds__(PSWF_THREADS) void k_yinv(Geo g, Tables t, FftAxis ax, Work w) {
  if (REG) {
    // consecutive column blocks of a plane on one XCD
    const int2 m = xcd_contiguous_2d();
    yinv_reg(g, t, w, m.x, m.y);
  } else {
    yinv_body(g, t, ax, w, blockIdx.x, blockIdx.y);
  }
}

// z C2R on the register FFT: 32 lines of Nz = 128 per workgroup
__device__ __forceinline__ void zinv_reg(const Geo &g, const Tables &t, const Work &w, int64_t nlines_total, int bx) {
  extern __shared__ float smem[];
  constexpr int Nz = 128;
  float2 *ex = reinterpret_cast<float2 *>(smem);
  float2 *tw = ex + 32 * kZregLine;
  float2 *twr = tw + Nz;
  const int tid = threadIdx.x, j = tid & 7, l = tid >> 3;
  const int64_t line0 = int64_t(bx) * 32;
  const bool on = line0 + l < nlines_total;
  float2 *xl = ex + l * kZregLine;
  // stored modes k < KZ of the line, zero up to and including k = Nz
  const float2 *src = reinterpret_cast<const float2 *>(w.s1) + (line0 + l) * g.KZP;
  float2 x[17];
#pragma unroll
  for (int i = 0; i < 17; ++i) {
    const int k = j + 8 * i;
    x[i] = (on && k < g.KZ) ? src[k] : make_float2(0.f, 0.f);
  }
  for (int e = tid; e < Nz; e += PSWF_THREADS) tw[e] = reinterpret_cast<const float2 *>(t.tw_z)[e];
  for (int e = tid; e <= Nz; e += PSWF_THREADS) twr[e] = reinterpret_cast<const float2 *>(t.tw_zr)[e];
#pragma unroll
  for (int i = 0; i < 17; ++i)
    if (j + 8 * i <= Nz) xl[j + 8 * i] = x[i];
  __syncthreads();
  // Z'_k = (X_k + conj X_{N-k}) + i exp(+2 pi i k / M_z) (X_k - conj X_{N-k}), k = 8 n1 + j
  float2 v[16];
#pragma unroll
  for (int n1 = 0; n1 < 16; ++n1) {
    const int k = 8 * n1 + j;
    const float2 xa = xl[k], xb = xl[Nz - k];
    const float2 a = make_float2(xa.x + xb.x, xa.y - xb.y);
    const float2 b = make_float2(xa.x - xb.x, xa.y + xb.y);
    float2 wv = twr[k];
    wv.y = -wv.y;
    const float2 ib = cmul(wv, b);
    v[n1] = make_float2(a.x - ib.y, a.y + ib.x);
  }
  rfft_inner<16, 1>(v, j, tw);
  wave_sync();
#pragma unroll
  for (int k1 = 0; k1 < 16; ++k1) xl[k1 * 9 + j] = v[k1];
  wave_sync();
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int n2 = 0; n2 < 8; ++n2) v[q * 8 + n2] = xl[(j + 8 * q) * 9 + n2];
  rfft_outer<16, 8, 1>(v);
  if (!on) return;
  float2 *dst = reinterpret_cast<float2 *>(w.grid) + (line0 + l) * Nz + j;
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) dst[8 * q + 16 * k2] = v[q * 8 + k2];
}

// z C2R: Z'_k = (X_k + conj X_{N-k}) + i exp(+2 pi i k / M_z)(X_k - conj X_{N-k}),
// inverse transform of length Nz gives x_2m + i x_2m+1.
__device__ __forceinline__ void zinv_body(const Geo &g, const Tables &t, const FftAxis &ax, const Work &w, int64_t nlines_total, int bx) {
  extern __shared__ float smem[];
  const int L = g.zlines, ld = L + 1, Nz = g.Nz;
  int llog = 0;
  while ((1 << llog) < L) ++llog;
  float2 *buf = reinterpret_cast<float2 *>(smem);
  float2 *tw = buf + Nz * ld;
  float2 *twr = tw + Nz;
  const int tid = threadIdx.x;
  const int64_t line0 = int64_t(bx) * L;
  const int nl = int(min(int64_t(L), nlines_total - line0));
  for (int e = tid; e < Nz; e += PSWF_THREADS) tw[e] = reinterpret_cast<const float2 *>(t.tw_z)[e];
  for (int e = tid; e <= Nz; e += PSWF_THREADS) twr[e] = reinterpret_cast<const float2 *>(t.tw_zr)[e];
  __syncthreads();
  // stage the KZ stored modes of each line (coalesced rows), then form the
  // packed half-length spectrum in place, one (k, N - k) pair per thread
  const float2 *src = reinterpret_cast<const float2 *>(w.s1) + line0 * g.KZP;
  staged16(
      L * g.KZ,
      [&](int e) {
        const int line = fdiv(e, g.div_kz);
        return line < nl ? src[line * g.KZP + (e - line * g.KZ)] : make_float2(0.f, 0.f);
      },
      [&](int e, float2 v) {
        const int line = fdiv(e, g.div_kz), k = e - line * g.KZ;
        buf[k * ld + line] = v;
      });
  __syncthreads();
  const int half = Nz / 2;
  for (int e = tid; e < L * (half + 1); e += PSWF_THREADS) {
    const int line = e & (L - 1), k = e >> llog;  // k in [0, Nz/2]
    const int km = Nz - k;                        // partner; Nz itself is the dropped Nyquist mode
    const float2 xk = k < g.KZ ? buf[k * ld + line] : make_float2(0.f, 0.f);
    const float2 xm = km < g.KZ ? buf[km * ld + line] : make_float2(0.f, 0.f);
    // Z'_j = (X_j + conj X_{N-j}) + i exp(+2 pi i j / M_z) (X_j - conj X_{N-j})
    auto zmode = [&](float2 xa, float2 xb, int j) {
      const float2 a = make_float2(xa.x + xb.x, xa.y - xb.y);
      const float2 b = make_float2(xa.x - xb.x, xa.y + xb.y);
      float2 wv = twr[j];
      wv.y = -wv.y;
      const float2 ib = cmul(wv, b);
      return make_float2(a.x - ib.y, a.y + ib.x);
    };
    const float2 zk = zmode(xk, xm, k);
    if (km < Nz && km != k) buf[km * ld + line] = zmode(xm, xk, km);
    buf[k * ld + line] = zk;
  }
  __syncthreads();
  lds_fft<1, 16>(buf, ax, llog - 2, ld, tw, tid);
  __syncthreads();
  float2 *dst = reinterpret_cast<float2 *>(w.grid) + line0 * Nz;
  for (int e = tid; e < nl * Nz; e += PSWF_THREADS) {
    const int line = fdiv(e, g.div_nz), n = e - line * Nz;
    dst[e] = buf[n * ld + line];
  }
}

// REG: the register FFT path (the planner's 256-point geometry)
template <bool REG>
__global__ __launch_bounds__(PSWF_THREADS) void k_zinv(Geo g, Tables t, FftAxis ax, Work w, int64_t nlines_total) {
  if (REG)
    zinv_reg(g, t, w, nlines_total, xcd_contiguous(blockIdx.x, gridDim.x));
  else
    zinv_body(g, t, ax, w, nlines_total, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Gather (adjoint of step i): one workgroup per tile.  The tile's atoms are
// taken in passes of up to kGatherAtoms; four lanes serve one atom, lane l
// owning the window rows at y-offsets l and l + 4.  Each lane evaluates the
// window and its derivative at its own offsets and the four exchange them
// once per pass, so every lane holds the atom's x and z weights in
// registers across all channels.  Per channel the tile's grid region plus a
// P-1 halo is staged in LDS (one channel at a time keeps the workgroup small
// enough for several to share a CU); each lane contracts its rows -- z
// first, then x -- and the lanes are reduced once per atom for the forces
// (per channel only for the potential).
//   phi_i   = sum_n pg(n) W(n h - r_i)
//   F_i     = q_i sum_n pg(n) grad W(n h - r_i)
// mode 1: forces/potentials; mode 2: adjoint (grad_q = g phi, grad_r = -g F);
// mode 3: as 1 without the zero-frequency term in the potentials (grids that
// are not the charge grid's potential).
constexpr int kGatherThreads = 512;
constexpr int kGatherLanes = 4;                                 // lanes per atom
constexpr int kGatherAtoms = kGatherThreads / kGatherLanes;     // atoms per pass
constexpr int kGatherStage = 16;                                // halo elements staged per thread
constexpr unsigned kGatherOOB = 0xfffffff0u;                    // byte offset past any grid channel
// gfx9 raw buffer descriptor word 3 (32-bit dwords, range-checked offsets)
constexpr int kBufferWord3 = 0x00020000;


// One channel's halo straight into LDS (buffer loads with the LDS bit: no
// registers, no LDS store instructions).  Wave wv moves elements
// wv 64 + 512 r + lane of the [EX][EY][EZ] region, which land at those
// float offsets of buf; goff holds each element's byte offset in the channel
// (offsets past the channel read as 0).  Completion is tracked by vmcnt.
constexpr int kGatherTileMax = kGatherThreads * kGatherStage;  // floats per tile buffer
__device__ __forceinline__ void gather_dma_halo(const float *grid, int64_t chan, int c, const unsigned (&goff)[kGatherStage],
                                                float *buf, int wv) {
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float *>(grid + int64_t(c) * chan), 0, int(unsigned(chan * 4)), kBufferWord3);
#pragma unroll
  for (int r = 0; r < kGatherStage; ++r)
    __builtin_amdgcn_raw_ptr_buffer_load_lds(
        rs, (__attribute__((address_space(3))) void *)(buf + wv * 64 + kGatherThreads * r), 4, goff[r], 0, 0, 0);
}

template <int P>
__device__ __forceinline__ void gather_body(const Geo &g, const Tables &t, const Work &w, float *__restrict__ fout,
                                            float *__restrict__ pout, int mode, const double *__restrict__ grad, int bx) {
  constexpr int R = (P + kGatherLanes - 1) / kGatherLanes;      // rows per lane
  extern __shared__ float smem[];
  const int Bx = g.B[0], By = g.B[1], Bz = g.B[2];
  const int EX = Bx + P - 1, EY = By + P - 1, EZ = Bz + P - 1;
  const int SZ = EZ;                                            // rows unpadded: the DMA fills linear runs
  const int plane = EY * SZ;
  float *tile0 = smem;                                          // two [EX][EY][EZ] buffers, channels alternate
  float *tile1 = smem + kGatherTileMax;
  float *wcf = smem + 2 * kGatherTileMax;                      // window coefficients, 16-byte aligned
  const int tid = threadIdx.x;
  const int cell = bx;
  const int s = w.cell_start[cell], e = w.cell_start[cell + 1];
  if (s == e) return;
  const int cz = cell % g.nc[2], cy = (cell / g.nc[2]) % g.nc[1], cx = cell / (g.nc[2] * g.nc[1]);
  const int t0[3] = {cx * Bx, cy * By, cz * Bz};
  for (int k = tid; k < kWinSeg * (kWinDeg + 1); k += kGatherThreads) wcf[k] = t.win[k];

  // halo elements this thread moves: elements tid + 512 r of the
  // [EX][EY][EZ] region, the same for every channel.  Byte offsets within a
  // channel of the grid; unused slots get an offset past the buffer range,
  // which a buffer load returns as 0.
  const int nhalo = EX * EY * EZ;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  unsigned goff[kGatherStage];
#pragma unroll
  for (int r = 0; r < kGatherStage; ++r) {
    const int el = tid + kGatherThreads * r;
    const int x = fdiv(el, g.div_geyz), rem = el - x * (EY * EZ), y = fdiv(rem, g.div_gez), z = rem - y * EZ;
    int gx = t0[0] + x, gy = t0[1] + y, gz = t0[2] + z;
    if (gx >= g.M[0]) gx -= g.M[0];
    if (gy >= g.M[1]) gy -= g.M[1];
    if (gz >= g.M[2]) gz -= g.M[2];
    goff[r] = el < nhalo ? unsigned((gx * g.M[1] + gy) * g.M[2] + gz) * 4u : kGatherOOB;
  }
  const int64_t chan = int64_t(g.M[0]) * g.M[1] * g.M[2];
  // channel c is read from buffer c & 1 while channel c + 1 streams into
  // the other one: one barrier per channel
  gather_dma_halo(w.grid, chan, 0, goff, tile0, wv);  // in flight during the set-up
  const int l = tid & (kGatherLanes - 1);
  const float sg = mode == 2 ? -1.0f : 1.0f;
  __syncthreads();  // window coefficients

  for (int p0 = s; p0 < e; p0 += kGatherAtoms) {
    const int na = min(kGatherAtoms, e - p0);
    // four lanes per atom; the lanes of an atom load its record together
    const int slot = tid / kGatherLanes;
    const bool act = slot < na;
    const int a = p0 + min(slot, na - 1);
    const float4 rr = reinterpret_cast<const float4 *>(w.rec_a)[a];
    const int dst_atom = w.perm_a[a];  // used only at the end: loaded early
    float qv = w.q_a[a];               // channel 0; later channels are loaded one ahead
    if (p0 > s) {
      __syncthreads();  // the previous pass has finished with both buffers
      gather_dma_halo(w.grid, chan, 0, goff, tile0, wv);
    }
    const unsigned pk = __float_as_uint(rr.w);
    int o[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      o[ax] = unpack_n0(pk, ax) - t0[ax];
      if (o[ax] < 0) o[ax] += g.M[ax];
    }
    // own offsets l + 4 j: window values and derivatives on the three axes
    float2 vx[R], vy[R], vz[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int off = l + kGatherLanes * j;
      const int oc = min(off, P - 1);
      vx[j] = win_eval_d(wcf, (2.0f * (oc + rr.x)) / P - 1.0f);
      vy[j] = win_eval_d(wcf, (2.0f * (oc + rr.y)) / P - 1.0f);
      vz[j] = win_eval_d(wcf, (2.0f * (oc + rr.z)) / P - 1.0f);
      if (off >= P) vy[j] = make_float2(0.0f, 0.0f);  // rows past the window add nothing
    }
    float wx[P], dwx[P], wz[P], dwz[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int src = i % kGatherLanes, j = i / kGatherLanes;
      wx[i] = __shfl(vx[j].x, src, kGatherLanes);
      dwx[i] = __shfl(vx[j].y, src, kGatherLanes);
      wz[i] = __shfl(vz[j].x, src, kGatherLanes);
      dwz[i] = __shfl(vz[j].y, src, kGatherLanes);
    }
    float wy[R], dwy[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
      wy[j] = vy[j].x;
      dwy[j] = vy[j].y;
    }
    const int base = o[0] * plane + o[1] * SZ + o[2];
    float f0 = 0.f, f1 = 0.f, f2 = 0.f;
    // a wave whose atoms all lie past the end of the tile (the short last
    // pass of a tile with more than kGatherAtoms atoms) only moves halo
    // data and meets the barriers
    const bool wave_busy = (wv * 64) / kGatherLanes < na;

    for (int c = 0; c < g.C; ++c) {
      // this wave's part of channel c has landed; after the barrier all of
      // it has, and every wave is done with channel c - 1
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      const float *tile = (c & 1) ? tile1 : tile0;
      const float qc = qv;
      if (c + 1 < g.C) {
        gather_dma_halo(w.grid, chan, c + 1, goff, (c & 1) ? tile0 : tile1, wv);
        qv = w.q_a[int64_t(c + 1) * g.N + a];
      }
      if (!wave_busy) continue;
      float vphi = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll 1
      for (int j = 0; j < R; ++j) {
        const int yo = min(l + kGatherLanes * j, P - 1);
        const float *b = tile + base + yo * SZ;
        float sp = 0.f, sx = 0.f, szz = 0.f;
        // rows double-buffered in registers: row lx + 1 is read while row
        // lx is contracted
        float gv[2][P];
#pragma unroll
        for (int lz = 0; lz < P; ++lz) gv[0][lz] = b[lz];
#pragma unroll
        for (int lx = 0; lx < P; ++lx) {
          if (lx + 1 < P) {
#pragma unroll
            for (int lz = 0; lz < P; ++lz) gv[(lx + 1) & 1][lz] = b[(lx + 1) * plane + lz];
          }
          float a0 = 0.f, a1 = 0.f;
#pragma unroll
          for (int lz = 0; lz < P; ++lz) {
            a0 = fmaf(wz[lz], gv[lx & 1][lz], a0);
            a1 = fmaf(dwz[lz], gv[lx & 1][lz], a1);
          }
          sp = fmaf(wx[lx], a0, sp);
          sx = fmaf(dwx[lx], a0, sx);
          szz = fmaf(wx[lx], a1, szz);
        }
        const float wyj = j == 0 ? wy[0] : wy[R - 1], dwyj = j == 0 ? dwy[0] : dwy[R - 1];
        vphi = fmaf(wyj, sp, vphi);
        gx = fmaf(wyj, sx, gx);
        gy = fmaf(dwyj, sp, gy);
        gz = fmaf(wyj, szz, gz);
      }
      f0 = fmaf(qc, gx, f0);
      f1 = fmaf(qc, gy, f1);
      f2 = fmaf(qc, gz, f2);
      if (pout) {
#pragma unroll
        for (int off = 1; off < kGatherLanes; off <<= 1) vphi += __shfl_xor(vphi, off, kGatherLanes);
        if (act && l == 0) {
          const double gsc = mode == 2 ? grad[c] : 1.0;
          // potential includes the zero-frequency term dE_0/dq = 2 a Q_net
          const float zero = mode == 3 ? 0.0f : float(2.0 * t.zero_V[c] / g.V * w.qsum[2 * c] * gsc);
          pout[int64_t(c) * g.N + dst_atom] = vphi + zero;
        }
      }
    }
#pragma unroll
    for (int off = 1; off < kGatherLanes; off <<= 1) {
      f0 += __shfl_xor(f0, off, kGatherLanes);
      f1 += __shfl_xor(f1, off, kGatherLanes);
      f2 += __shfl_xor(f2, off, kGatherLanes);
    }
    if (act && l == 0 && fout) {
      // window-argument derivatives on the grid axes -> d/dr: F_b = sum_a gT[a][b] f_a
      const int64_t oo = 3 * int64_t(dst_atom);
      fout[oo] = sg * fmaf(g.gT[0], f0, fmaf(g.gT[3], f1, g.gT[6] * f2));
      fout[oo + 1] = sg * fmaf(g.gT[1], f0, fmaf(g.gT[4], f1, g.gT[7] * f2));
      fout[oo + 2] = sg * fmaf(g.gT[2], f0, fmaf(g.gT[5], f1, g.gT[8] * f2));
    }
  }
}

// Gather tiles go to the XCDs in contiguous ranges (xcd_contiguous) so that
// neighbouring tiles, whose halos overlap, run at the same time behind the
// same L2.

// Order of tiles within an XCD's range: compact groups of up to 4 x 4 x 4
// tiles (the largest of 4, 2, 1 dividing the tile count per axis) instead
// of whole rows, so that the tiles resident at once share most of their
// halo planes in every direction, not only along y and z.
__device__ __forceinline__ int tile_grouped(int i, const int *nc) {
  int gd[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) gd[a] = (nc[a] & 3) == 0 ? 4 : ((nc[a] & 1) == 0 ? 2 : 1);
  const int gsize = gd[0] * gd[1] * gd[2];
  const int gi = i / gsize, wi = i - gi * gsize;
  const int ngy = nc[1] / gd[1], ngz = nc[2] / gd[2];
  const int gz = gi % ngz, gy = (gi / ngz) % ngy, gx = gi / (ngz * ngy);
  const int iz = wi % gd[2], iy = (wi / gd[2]) % gd[1], ix = wi / (gd[2] * gd[1]);
  return ((gx * gd[0] + ix) * nc[1] + gy * gd[1] + iy) * nc[2] + gz * gd[2] + iz;
}

template <int P>
__global__ __launch_bounds__(kGatherThreads, 4) void k_gather(Geo g, Tables t, Work w, float *__restrict__ fout,
                                                            float *__restrict__ pout, int mode,
                                                            const double *__restrict__ grad) {
  gather_body<P>(g, t, w, fout, pout, mode, grad, tile_grouped(xcd_contiguous(blockIdx.x, gridDim.x), g.nc));
}

// Final FP64 reduction: energy [3C + 1] (E_k, E_0, E_self per channel, then
// E_lr = sum_c (E_k + E_0) in channel order) and virial [6].  A non-finite
// input position (status word set by the binning) makes E_lr, every E_k and
// the virial NaN.
template <int THREADS>
__device__ __forceinline__ void finalize_body(const Geo &g, const Tables &t, const Work &w, double *energy, double *virial) {
  // one wave per channel at a time (channels c = wave, wave + THREADS / 64,
  // ...): lane sums over the x-pass blocks, then a fixed-order wave
  // reduction; the channels' energy and virial terms are added in channel
  // order by one thread each.  The result does not depend on THREADS: each
  // lane adds its blocks in the same order whichever wave holds the channel.
  __shared__ double vch[kMaxChannels][7];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool bad = w.status[0] != 0;
  const double nan = __longlong_as_double(0x7ff8000000000000ll);
  for (int c = wave; c < g.C; c += THREADS / 64) {
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    // unrolled so that several blocks' partials are in flight at once; the
    // additions stay in block order
#pragma unroll 4
    for (int b = lane; b < g.nxblk; b += 64)
#pragma unroll
      for (int i = 0; i < 7; ++i) acc[i] += w.epart[(int64_t(c) * g.nxblk + b) * 8 + i];
#pragma unroll
    for (int i = 0; i < 7; ++i)
      for (int off = 32; off > 0; off >>= 1) acc[i] += __shfl_down(acc[i], off, 64);
    if (lane == 0) {
      const double inv2V = 0.5 / g.V;
      const double Ek = bad ? nan : acc[0] * inv2V;
      const double Q = w.qsum[2 * c], Q2 = w.qsum[2 * c + 1];
      const double E0 = t.zero_V[c] / g.V * Q * Q;
      energy[3 * c] = Ek;
      energy[3 * c + 1] = E0;
      energy[3 * c + 2] = t.self_coef[c] * Q2;
      // W_ab = (1/2V) sum |F|^2 D (Phi delta_ab + Phi'/k k_a k_b) + E_0 delta_ab
      vch[c][0] = Ek + E0 + acc[1] * inv2V;
      vch[c][1] = Ek + E0 + acc[2] * inv2V;
      vch[c][2] = Ek + E0 + acc[3] * inv2V;
      vch[c][3] = bad ? nan : acc[4] * inv2V;
      vch[c][4] = bad ? nan : acc[5] * inv2V;
      vch[c][5] = bad ? nan : acc[6] * inv2V;
      vch[c][6] = Ek + E0;
    }
  }
  __syncthreads();
  if (tid < 7 && (virial || tid == 6)) {
    double v = 0.0;
    for (int c = 0; c < g.C; ++c) v += vch[c][tid];
    if (tid < 6) virial[tid] = v;
    else energy[3 * g.C] = g.C > 0 ? v : 0.0;
  }
}

// one wave per channel (up to 16 channels at once)
constexpr int kFinalizeThreads = 1024;
__global__ __launch_bounds__(kFinalizeThreads) void k_finalize(Geo g, Tables t, Work w, double *energy, double *virial) {
  finalize_body<kFinalizeThreads>(g, t, w, energy, virial);
}
// Input validation (plans created with PSWFLR_FLAG_CHECK_INPUTS): bit 0 of
// word[0] is set when a position is not finite, bit 1 when a charge is not.
__global__ __launch_bounds__(PSWF_THREADS) void k_clear_word(int *word) {
  if (threadIdx.x == 0) word[0] = 0;
}

__global__ __launch_bounds__(PSWF_THREADS) void k_check_inputs(const float *__restrict__ pos, const float *__restrict__ q,
                                                               int64_t npos, int64_t nq, int *word) {
  int bits = 0;
  for (int64_t i = int64_t(blockIdx.x) * PSWF_THREADS + threadIdx.x; i < npos + nq;
       i += int64_t(gridDim.x) * PSWF_THREADS) {
    const float v = i < npos ? pos[i] : q[i - npos];
    if (!isfinite(v)) bits |= i < npos ? 1 : 2;
  }
  if (__ballot(bits != 0)) {
    if (bits) atomicOr(word, bits);
  }
}


// ---------------------------------------------------------------------------
// Second derivatives for force-matching training (the derivatives of
// L = sum_i v_i . F_i).  With psi the potential grid of the forward call
// (phi = W^T psi, F_i = -q_i grad_i (W^T psi)) and u the dipole grid
// u(n) = sum_i q_i (v_i . grad_{r_i}) W(n h - r_i):
//   dL/dq_i = -v_i . grad phi(r_i) - (W^T A u)_i
//   dL/dr_i = -q_i (Hess phi(r_i)) v_i - q_i grad_i (W^T A u)
// where A is the forward's convolution (FFT, Phi_p / What^2, inverse FFT).

// dipole charges in cell order: qd[a][c][k] = -q_c(k) v_a(k), so that
// u = sum_a spread(qd[a], derivative factor on axis a)
__global__ __launch_bounds__(PSWF_THREADS) void k_dd_prep(Geo g, Work w, const float *__restrict__ v, float *qd) {
  const int64_t e = int64_t(blockIdx.x) * PSWF_THREADS + threadIdx.x;
  const int64_t cn = int64_t(g.C) * g.N;
  if (e >= cn) return;
  const int64_t k = e % g.N;
  const int i = w.perm_a[k];
  const float qv = w.q_a[e];
  const float vx = v[3 * int64_t(i)], vy = v[3 * int64_t(i) + 1], vz = v[3 * int64_t(i) + 2];
  // v . grad_r = (T v) . grad_u: the dipole in grid units
#pragma unroll
  for (int a = 0; a < 3; ++a)
    qd[a * cn + e] = -qv * fmaf(g.T_hi[3 * a], vx, fmaf(g.T_hi[3 * a + 1], vy, g.T_hi[3 * a + 2] * vz));
}

// one thread per atom: grad phi and the Hessian of phi at the atom from the
// potential grid (separable window, its first and second derivatives);
// writes s1 = v . grad phi per channel and -sum_c q_c (Hess phi_c) v
template <int P>
__global__ __launch_bounds__(PSWF_THREADS) void k_gather_hess(Geo g, Tables t, Work w, const float *__restrict__ v,
                                                             float *__restrict__ s1, float *__restrict__ hv) {
  __shared__ float wcf[kWinSeg * (kWinDeg + 1)];
  for (int e = threadIdx.x; e < kWinSeg * (kWinDeg + 1); e += PSWF_THREADS) wcf[e] = t.win[e];
  __syncthreads();
  const int64_t k = int64_t(blockIdx.x) * PSWF_THREADS + threadIdx.x;
  if (k >= g.N) return;
  const float4 rr = reinterpret_cast<const float4 *>(w.rec_a)[k];
  const unsigned pk = __float_as_uint(rr.w);
  const float dl[3] = {rr.x, rr.y, rr.z};
  float W[3][P], D[3][P], DD[3][P];
  int n[3][P];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int n0 = unpack_n0(pk, a);
#pragma unroll
    for (int l = 0; l < P; ++l) {
      const float3 f = win_eval_dd(wcf, (2.0f * (l + dl[a])) / P - 1.0f);
      W[a][l] = f.x;
      D[a][l] = f.y * (2.0f / P);
      DD[a][l] = f.z * (4.0f / (P * P));
      int m = n0 + l;
      if (m >= g.M[a]) m -= g.M[a];
      n[a][l] = m;
    }
  }
  const int i = w.perm_a[k];
  // derivatives are taken in grid units u = T r: grad_r = T^T grad_u,
  // Hess_r = T^T Hess_u T, so v . grad_r phi = (T v) . grad_u phi and
  // Hess_r v = T^T (Hess_u (T v))
  float vx, vy, vz;
  {
    const float v0 = v[3 * int64_t(i)], v1 = v[3 * int64_t(i) + 1], v2 = v[3 * int64_t(i) + 2];
    vx = fmaf(g.T_hi[0], v0, fmaf(g.T_hi[1], v1, g.T_hi[2] * v2));
    vy = fmaf(g.T_hi[3], v0, fmaf(g.T_hi[4], v1, g.T_hi[5] * v2));
    vz = fmaf(g.T_hi[6], v0, fmaf(g.T_hi[7], v1, g.T_hi[8] * v2));
  }
  const int64_t chan = int64_t(g.M[0]) * g.M[1] * g.M[2];
  float h0 = 0.f, h1 = 0.f, h2 = 0.f;
  for (int c = 0; c < g.C; ++c) {
    const float *psi = w.grid + int64_t(c) * chan;
    float gx = 0.f, gy = 0.f, gz = 0.f, hxx = 0.f, hyy = 0.f, hzz = 0.f, hxy = 0.f, hxz = 0.f, hyz = 0.f;
    for (int lx = 0; lx < P; ++lx) {
      for (int ly = 0; ly < P; ++ly) {
        const float *row = psi + (int64_t(n[0][lx]) * g.M[1] + n[1][ly]) * g.M[2];
        float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
        for (int lz = 0; lz < P; ++lz) {
          const float val = row[n[2][lz]];
          a0 = fmaf(W[2][lz], val, a0);
          a1 = fmaf(D[2][lz], val, a1);
          a2 = fmaf(DD[2][lz], val, a2);
        }
        const float ww = W[0][lx] * W[1][ly], dw = D[0][lx] * W[1][ly], wd = W[0][lx] * D[1][ly];
        // d W / d x_a = -D_a (other factors); d2 W / d x_a d x_b = D_a D_b (...)
        gx -= dw * a0;
        gy -= wd * a0;
        gz -= ww * a1;
        hxx = fmaf(DD[0][lx] * W[1][ly], a0, hxx);
        hyy = fmaf(W[0][lx] * DD[1][ly], a0, hyy);
        hzz = fmaf(ww, a2, hzz);
        hxy = fmaf(D[0][lx] * D[1][ly], a0, hxy);
        hxz = fmaf(dw, a1, hxz);
        hyz = fmaf(wd, a1, hyz);
      }
    }
    s1[int64_t(c) * g.N + i] = vx * gx + vy * gy + vz * gz;
    const float qc = w.q_a[int64_t(c) * g.N + k];
    h0 -= qc * (hxx * vx + hxy * vy + hxz * vz);
    h1 -= qc * (hxy * vx + hyy * vy + hyz * vz);
    h2 -= qc * (hxz * vx + hyz * vy + hzz * vz);
  }
  hv[3 * int64_t(i)] = fmaf(g.T_hi[0], h0, fmaf(g.T_hi[3], h1, g.T_hi[6] * h2));
  hv[3 * int64_t(i) + 1] = fmaf(g.T_hi[1], h0, fmaf(g.T_hi[4], h1, g.T_hi[7] * h2));
  hv[3 * int64_t(i) + 2] = fmaf(g.T_hi[2], h0, fmaf(g.T_hi[5], h1, g.T_hi[8] * h2));
}

// dL/dq = -(s1 + s2), dL/dr = hv + F2 (caller order)
__global__ __launch_bounds__(PSWF_THREADS) void k_dd_combine(int64_t cn, int64_t n3, float *__restrict__ gq,
                                                            const float *__restrict__ s2, float *__restrict__ gp,
                                                            const float *__restrict__ f2) {
  const int64_t e = int64_t(blockIdx.x) * PSWF_THREADS + threadIdx.x;
  if (e < cn) gq[e] = -(gq[e] + s2[e]);
  if (e < n3) gp[e] += f2[e];
}

// dE/dH_ab = -sum_k (H^-1)_ka W_kb at fixed fractional coordinates: with
// H -> H (1 + e)^T, dE = sum (dE/dH)_ab H_ak e_bk must equal -sum W_bk e_bk
__global__ void k_cell_gradient(CellInv hinv, const double *__restrict__ virial, double *__restrict__ grad) {
  const int e = threadIdx.x;
  if (e >= 9) return;
  const int a = e / 3, b = e % 3;
  const int vi[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
  double s = 0.0;
  for (int k = 0; k < 3; ++k) s += hinv.m[3 * k + a] * virial[vi[k][b]];
  grad[e] = -s;
}

// ---------------------------------------------------------------------------
// launchers
static inline unsigned nblocks(int64_t n, int per) { return unsigned((n + per - 1) / per); }

#define LAUNCH_CHECK()                         \
  do {                                         \
    hipError_t e__ = hipGetLastError();        \
    if (e__ != hipSuccess) return e__;         \
  } while (0)

size_t spread_lds_bytes(const Geo &g, int ncg) {
  (void)ncg;
  const int S = spread_pad4(g.B[0]) + spread_pad4(g.B[1]) + spread_pad4(g.B[2]);
  const int cgt = spread_cg_template(ncg);
  return size_t(spread_lds_floats(S, cgt, spread_cap(cgt, g.scap))) * 4;
}
int spread_max_cells() { return kSpreadMaxCells; }
// vector-ALU spread: the larger flush when a launch's tiles all fit on the
// chip at once at its occupancy (two workgroups per CU), else the smaller
int spread_flush_cap(int64_t tiles) { return tiles <= 2 * 256 ? kSpreadCap : kSpreadCapV; }
// candidate cells a tile of edges b has to screen (see spread_body)
int spread_candidate_cells(const int *nc, const int *b, int P) {
  int n = 1;
  for (int a = 0; a < 3; ++a) n *= std::min(std::min(nc[a] - 1, (P - 2) / b[a] + 1) + 1, 8);
  return n;
}
int spread_max_channels() { return kSpreadCGM; }
bool spread_tile_ok(int bx, int by, int bz) {
  const int nbz = spread_nbz(bz);
  if (nbz == 0) return false;
  const int cpw = kSpreadNBW / nbz, nby = spread_pad4(by) / 4, ncol = (spread_pad4(bx) / 4) * nby;
  const int S = spread_pad4(bx) + spread_pad4(by) + spread_pad4(bz);
  return nby % cpw == 0 && ncol <= cpw * (kSpreadThreads / 64) && S <= kSpreadMaxS &&
         bx * by * bz <= spread_stage_floats(S, 2, kSpreadCapV);
}
size_t gather_lds_bytes(const Geo &g, int ncg) {
  (void)ncg;
  const size_t EX = g.B[0] + g.P - 1, EY = g.B[1] + g.P - 1, EZ = g.B[2] + g.P - 1;
  (void)EX;
  (void)EY;
  (void)EZ;
  return (2 * size_t(kGatherTileMax) + kWinSeg * (kWinDeg + 1)) * 4;
}
bool gather_tile_ok(int bx, int by, int bz, int P) {
  Geo g{};
  g.B[0] = bx;
  g.B[1] = by;
  g.B[2] = bz;
  g.P = P;
  const int ex = bx + P - 1, ey = by + P - 1, ez = bz + P - 1;
  return ex * ey * ez <= kGatherThreads * kGatherStage && gather_lds_bytes(g, 1) <= 160 * 1024;
}
size_t zpass_lds_bytes(const Geo &g) {
  if (zreg_ok(g)) return (size_t(32) * kZregLine + 2 * g.Nz + 1) * 8;
  return (size_t(g.Nz) * (g.zlines + 1) + 2 * g.Nz + 1) * 8;
}
size_t ypass_lds_bytes(const Geo &g) {
  const int kb = std::max(g.kb, g.kby);
  return (size_t(g.M[1]) * (kb + 1) + g.M[1]) * 8;
}
bool x_register_path(const Geo &g) { return xreg_ok(g); }
size_t xpass_lds_bytes(const Geo &g) {
  const int kb = std::max(g.kb, g.kbx);
  return (size_t(g.M[0]) * (kb + 1) + g.M[0] + 1) * 8 + 2 * kKerCoef * 4;
}

// Dynamic LDS above 64 KiB needs an opt-in per kernel; request it only when
// a launch needs it, clamped to what the device allows, and clear the
// runtime's error state if the request is refused.
static size_t device_lds_optin() {
  static size_t cached = 0;
  if (cached) return cached;
  int dev = 0, v = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess || v <= 0) {
    (void)hipGetLastError();
    v = 64 * 1024;
  }
  cached = size_t(v);
  return cached;
}

static hipError_t lds_request(const void *fn, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  if (bytes > device_lds_optin()) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
  if (e != hipSuccess) (void)hipGetLastError();
  return e;
}

hipError_t enqueue_sort(const Geo &g, const Work &w, const float *pos, const float *q, hipStream_t st) {
  // cell offsets are produced even for N = 0 (the spread reads them); the
  // charge sums (zero for N = 0) ride in the binning and scatter launches
  const int nq = qsum_blocks(g);
  const int nbin = g.N > 0 ? int(nblocks(g.N, PSWF_THREADS)) : 0;
  hipLaunchKernelGGL(k_zero, dim3(nblocks(g.ncell, PSWF_THREADS)), dim3(PSWF_THREADS), 0, st, g, w);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_bin_qsum, dim3(nbin + nq * g.C), dim3(PSWF_THREADS), 0, st, g, w, pos, q, nbin, nq);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, w, g.ncell, g.N);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_scatter_qreduce, dim3(nbin + 1), dim3(PSWF_THREADS), 0, st, g, w, nbin, nq);
  LAUNCH_CHECK();
  if (g.N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_order, dim3(g.ncell), dim3(PSWF_THREADS), 0, st, g, w);
  LAUNCH_CHECK();
  return hipSuccess;
}

int qsum_blocks(const Geo &g) { return int(std::max<int64_t>(1, (g.N + kQChunk - 1) / kQChunk)); }

bool prep_small(const Geo &g) { return g.N <= kPrepSmallMax; }

hipError_t enqueue_prep_small(const Geo &g, const Work &w, const float *pos, const float *q, hipStream_t st) {
  hipLaunchKernelGGL(k_prep_small, dim3(1), dim3(kPrepThreads), 0, st, g, w, pos, q);
  LAUNCH_CHECK();
  return hipSuccess;
}

template <int P, int NBZ, int CG>
static hipError_t spread_pzc(const Geo &g, const Tables &t, const Work &w, int cg0, int ncg, hipStream_t st,
                             const SpreadSrc &src) {
  hipError_t e = lds_request(reinterpret_cast<const void *>(&k_spread<P, NBZ, CG>), spread_lds_bytes(g, CG));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_spread<P, NBZ, CG>), dim3(g.ncell), dim3(kSpreadThreads), spread_lds_bytes(g, CG), st, g, t,
                     w, cg0, ncg, src);
  LAUNCH_CHECK();
  return hipSuccess;
}

template <int P, int NBZ>
static hipError_t spread_pz(const Geo &g, const Tables &t, const Work &w, int cg0, int ncg, hipStream_t st,
                            const SpreadSrc &src) {
  switch (spread_cg_template(g.CG_spread)) {
    case 2: return spread_pzc<P, NBZ, 2>(g, t, w, cg0, ncg, st, src);
    case 4: return spread_pzc<P, NBZ, 4>(g, t, w, cg0, ncg, st, src);
    default: return spread_pzc<P, NBZ, kSpreadCGM>(g, t, w, cg0, ncg, st, src);
  }
}

template <int P>
static hipError_t spread_p(const Geo &g, const Tables &t, const Work &w, int cg0, int ncg, hipStream_t st,
                           const SpreadSrc &src) {
  switch (spread_nbz(g.B[2])) {
    case 1: return spread_pz<P, 1>(g, t, w, cg0, ncg, st, src);
    case 2: return spread_pz<P, 2>(g, t, w, cg0, ncg, st, src);
    case 4: return spread_pz<P, 4>(g, t, w, cg0, ncg, st, src);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_spread(const Geo &g, const Tables &t, const Work &w, int cg0, int ncg, hipStream_t st,
                         const SpreadSrc &src) {
  switch (g.P) {
    case 2: return spread_p<2>(g, t, w, cg0, ncg, st, src);
    case 3: return spread_p<3>(g, t, w, cg0, ncg, st, src);
    case 4: return spread_p<4>(g, t, w, cg0, ncg, st, src);
    case 5: return spread_p<5>(g, t, w, cg0, ncg, st, src);
    case 6: return spread_p<6>(g, t, w, cg0, ncg, st, src);
    case 7: return spread_p<7>(g, t, w, cg0, ncg, st, src);
    case 8: return spread_p<8>(g, t, w, cg0, ncg, st, src);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_zfwd(const Geo &g, const Tables &t, const FftAxis &az, const Work &w, hipStream_t st) {
  const int64_t lines = int64_t(g.C) * g.M[0] * g.M[1];
  hipLaunchKernelGGL(zreg_ok(g) ? k_zfwd<true> : k_zfwd<false>, dim3(nblocks(lines, g.zlines)), dim3(PSWF_THREADS), zpass_lds_bytes(g), st, g, t,
                     az, w, lines);
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_yfwd(const Geo &g, const Tables &t, const FftAxis &ay, const Work &w, hipStream_t st) {
  const dim3 grid = yreg_ok(g) ? dim3(nblocks(g.KZ, g.kb), g.C * g.M[0])
                               : dim3(nblocks(g.KZ, g.kzq), nblocks(int64_t(g.C) * g.M[0], g.ypl));
  hipLaunchKernelGGL(yreg_ok(g) ? k_yfwd<true> : k_yfwd<false>, grid, dim3(PSWF_THREADS), ypass_lds_bytes(g),
                     st, g, t, ay, w);
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_xmul(const Geo &g, const Tables &t, const FftAxis &ax, const Work &w, int mode,
                       const double *grad, hipStream_t st) {
  if (g.nxblk == 0) return hipSuccess;
  hipLaunchKernelGGL(xreg_ok(g) ? k_xmul<true> : k_xmul<false>, dim3(g.nxblk, g.C), dim3(PSWF_THREADS), xpass_lds_bytes(g), st, g, t, ax, w, mode,
                     grad);
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_yinv(const Geo &g, const Tables &t, const FftAxis &ay, const Work &w, hipStream_t st) {
  const dim3 grid = yreg_ok(g) ? dim3(nblocks(g.KZ, g.kb), g.C * g.M[0])
                               : dim3(nblocks(g.KZ, g.kzq), nblocks(int64_t(g.C) * g.M[0], g.ypl));
  hipLaunchKernelGGL(yreg_ok(g) ? k_yinv<true> : k_yinv<false>, grid, dim3(PSWF_THREADS), ypass_lds_bytes(g),
                     st, g, t, ay, w);
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_zinv(const Geo &g, const Tables &t, const FftAxis &az, const Work &w, hipStream_t st) {
  const int64_t lines = int64_t(g.C) * g.M[0] * g.M[1];
  hipLaunchKernelGGL(zreg_ok(g) ? k_zinv<true> : k_zinv<false>, dim3(nblocks(lines, g.zlines)), dim3(PSWF_THREADS), zpass_lds_bytes(g), st, g, t,
                     az, w, lines);
  LAUNCH_CHECK();
  return hipSuccess;
}

template <int P>
static hipError_t gather_p(const Geo &g, const Tables &t, const Work &w, float *f, float *pot, int mode,
                           const double *grad, hipStream_t st) {
  hipError_t e = lds_request(reinterpret_cast<const void *>(&k_gather<P>), gather_lds_bytes(g, g.CG_gather));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gather<P>, dim3(g.ncell), dim3(kGatherThreads), gather_lds_bytes(g, g.CG_gather), st, g,
                     t, w, f, pot, mode, grad);
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_gather(const Geo &g, const Tables &t, const Work &w, float *forces, float *pot, int mode,
                         const double *grad, hipStream_t st) {
  if (g.N == 0) return hipSuccess;
  switch (g.P) {
    case 2: return gather_p<2>(g, t, w, forces, pot, mode, grad, st);
    case 3: return gather_p<3>(g, t, w, forces, pot, mode, grad, st);
    case 4: return gather_p<4>(g, t, w, forces, pot, mode, grad, st);
    case 5: return gather_p<5>(g, t, w, forces, pot, mode, grad, st);
    case 6: return gather_p<6>(g, t, w, forces, pot, mode, grad, st);
    case 7: return gather_p<7>(g, t, w, forces, pot, mode, grad, st);
    case 8: return gather_p<8>(g, t, w, forces, pot, mode, grad, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_cell_gradient(const CellInv &hinv, const double *virial, double *grad, hipStream_t st) {
  hipLaunchKernelGGL(k_cell_gradient, dim3(1), dim3(64), 0, st, hinv, virial, grad);
  return hipGetLastError();
}

hipError_t launch_check_inputs(const Geo &g, const Work &w, const float *pos, const float *q, hipStream_t st) {
  hipLaunchKernelGGL(k_clear_word, dim3(1), dim3(PSWF_THREADS), 0, st, w.status + 1);
  LAUNCH_CHECK();
  const int64_t n = 3 * g.N + int64_t(g.C) * g.N;
  if (n == 0) return hipSuccess;
  const unsigned nb = unsigned(std::min<int64_t>(2048, (n + PSWF_THREADS - 1) / PSWF_THREADS));
  hipLaunchKernelGGL(k_check_inputs, dim3(nb), dim3(PSWF_THREADS), 0, st, pos, q, 3 * g.N, int64_t(g.C) * g.N,
                     w.status + 1);
  LAUNCH_CHECK();
  return hipSuccess;
}

// Scratch for callers that cannot allocate (pswflr_execute_noalloc): one
// workspace-sized array per device, held until the process ends.  Host code
// never passes the array's name to a kernel (in host code it names a host
// stand-in, not device memory); it uses the device address looked up once
// per device with that device current, kept below.
static __device__ __align__(256) char scratch[kNoallocScratchBytes];

hipError_t noalloc_scratch(void **out) {
  static std::mutex mu;
  static void *addr[kNoallocMaxDevices] = {nullptr};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kNoallocMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *out = addr[dev];
  return hipSuccess;
}

template <int P>
static hipError_t hess_p(const Geo &g, const Tables &t, const Work &w, const float *v, float *s1, float *hv,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_gather_hess<P>, dim3(nblocks(g.N, PSWF_THREADS)), dim3(PSWF_THREADS), 0, st, g, t, w, v, s1, hv);
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_double_backward(const Geo &g, const Tables &t, const FftAxis &az, const FftAxis &ay,
                                  const FftAxis &ax, const Work &w, const float *v, float *qd, float *s2, float *f2,
                                  float *grad_q, float *grad_pos, hipStream_t st) {
  if (g.N == 0) return hipSuccess;
  hipError_t e = hipErrorInvalidValue;
  switch (g.P) {
    case 2: e = hess_p<2>(g, t, w, v, grad_q, grad_pos, st); break;
    case 3: e = hess_p<3>(g, t, w, v, grad_q, grad_pos, st); break;
    case 4: e = hess_p<4>(g, t, w, v, grad_q, grad_pos, st); break;
    case 5: e = hess_p<5>(g, t, w, v, grad_q, grad_pos, st); break;
    case 6: e = hess_p<6>(g, t, w, v, grad_q, grad_pos, st); break;
    case 7: e = hess_p<7>(g, t, w, v, grad_q, grad_pos, st); break;
    case 8: e = hess_p<8>(g, t, w, v, grad_q, grad_pos, st); break;
  }
  if (e != hipSuccess) return e;
  const int64_t cn = int64_t(g.C) * g.N;
  hipLaunchKernelGGL(k_dd_prep, dim3(nblocks(cn, PSWF_THREADS)), dim3(PSWF_THREADS), 0, st, g, w, v, qd);
  LAUNCH_CHECK();
  // the potential grid is no longer needed: the dipole grid takes its place
  for (int a = 0; a < 3; ++a) {
    SpreadSrc src;
    src.q = qd + a * cn;
    src.dax = a;
    src.acc = a > 0;
    for (int cg0 = 0; cg0 < g.C; cg0 += g.CG_spread)
      if ((e = launch_spread(g, t, w, cg0, std::min(g.CG_spread, g.C - cg0), st, src)) != hipSuccess) return e;
  }
  if ((e = launch_zfwd(g, t, az, w, st)) != hipSuccess) return e;
  if ((e = launch_yfwd(g, t, ay, w, st)) != hipSuccess) return e;
  if ((e = launch_xmul(g, t, ax, w, 1, nullptr, st)) != hipSuccess) return e;
  if ((e = launch_yinv(g, t, ay, w, st)) != hipSuccess) return e;
  if ((e = launch_zinv(g, t, az, w, st)) != hipSuccess) return e;
  if ((e = launch_gather(g, t, w, f2, s2, 3, nullptr, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_dd_combine, dim3(nblocks(std::max(cn, 3 * g.N), PSWF_THREADS)), dim3(PSWF_THREADS), 0, st, cn,
                     3 * g.N, grad_q, s2, grad_pos, f2);
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_finalize(const Geo &g, const Tables &t, const Work &w, double *energy, double *virial,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinalizeThreads), 0, st, g, t, w, energy, virial);
  LAUNCH_CHECK();
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Batched launches: one launch per stage covers every structure of a batch.
// prefix[s] is the first virtual block of structure s in this stage
// (prefix[n] = total); a workgroup finds its structure by binary search.
__device__ __forceinline__ int find_item(const int *__restrict__ prefix, int n, int b) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Virtual block b of one stage over the batch.
template <int STAGE>
__device__ __forceinline__ void batch_stage_block(const BatchItem *__restrict__ items, const int *__restrict__ prefix,
                                                  int n, int b) {
  const int s = find_item(prefix, n, b);
  const BatchItem &it = items[s];
  const int vb = b - prefix[s];
  const Geo &g = it.g;
  switch (STAGE) {
    case kBsZero: zero_body(g, it.w, vb); break;
    case kBsBin: bin_body(g, it.w, it.pos, it.q, vb); break;
    case kBsScan: scan_body(it.w, g.ncell, g.N); break;
    case kBsScatter: scatter_body(g, it.w, vb); break;
    case kBsOrder: order_body(g, it.w, vb); break;
    case kBsQsum: qsum_body(g, it.w, it.q, kQChunk, vb % it.qblocks, vb / it.qblocks); break;
    case kBsQreduce: qreduce_body(g, it.w, it.qblocks); break;
    case kBsSpread: break;  // one launch per kernel variant: k_batch_spread
    case kBsZfwd: zfwd_body(g, it.t, it.az, it.w, it.nlines, vb); break;
    case kBsYfwd: {
      const int gx = (g.KZ + g.kzq - 1) / g.kzq;
      yfwd_body(g, it.t, it.ay, it.w, vb % gx, vb / gx);
      break;
    }
    case kBsXmul: xmul_body(g, it.t, it.ax, it.w, it.mode, it.grad, vb % g.nxblk, vb / g.nxblk); break;
    case kBsFinalize: finalize_body<PSWF_THREADS>(g, it.t, it.w, it.energy, it.virial); break;
    case kBsYinv: {
      const int gx = (g.KZ + g.kzq - 1) / g.kzq;
      yinv_body(g, it.t, it.ay, it.w, vb % gx, vb / gx);
      break;
    }
    case kBsZinv: zinv_body(g, it.t, it.az, it.w, it.nlines, vb); break;
    case kBsGather:
      switch (g.P) {
        case 2: gather_body<2>(g, it.t, it.w, it.forces, it.pot, it.mode == 2 ? 2 : 1, it.grad, vb); break;
        case 3: gather_body<3>(g, it.t, it.w, it.forces, it.pot, it.mode == 2 ? 2 : 1, it.grad, vb); break;
        case 4: gather_body<4>(g, it.t, it.w, it.forces, it.pot, it.mode == 2 ? 2 : 1, it.grad, vb); break;
        case 5: gather_body<5>(g, it.t, it.w, it.forces, it.pot, it.mode == 2 ? 2 : 1, it.grad, vb); break;
        case 6: gather_body<6>(g, it.t, it.w, it.forces, it.pot, it.mode == 2 ? 2 : 1, it.grad, vb); break;
        case 7: gather_body<7>(g, it.t, it.w, it.forces, it.pot, it.mode == 2 ? 2 : 1, it.grad, vb); break;
        default: gather_body<8>(g, it.t, it.w, it.forces, it.pot, it.mode == 2 ? 2 : 1, it.grad, vb); break;
      }
      break;
  }
}

template <int STAGE, int THREADS>
__global__ __launch_bounds__(THREADS, ((STAGE == kBsSpread || STAGE == kBsGather) ? 4 : 3)) void k_batch(const BatchItem *__restrict__ items,
                                                    const int *__restrict__ prefix, int n, int mode) {
  (void)mode;
  batch_stage_block<STAGE>(items, prefix, n, blockIdx.x);
}

// Two independent stages of the same workgroup shape in one launch: blocks
// [0, total_a) run stage A, the rest stage B.  Used for stages whose inputs
// an earlier launch has finished (the charge sums beside the binning, their
// reduction beside the scatter), so the batch takes two launches fewer.
template <int STAGE_A, int STAGE_B>
__global__ __launch_bounds__(PSWF_THREADS, 3) void k_batch_pair(const BatchItem *__restrict__ items,
                                                                const int *__restrict__ prefix_a, int total_a,
                                                                const int *__restrict__ prefix_b, int n) {
  const int b = blockIdx.x;
  if (b < total_a)
    batch_stage_block<STAGE_A>(items, prefix_a, n, b);
  else
    batch_stage_block<STAGE_B>(items, prefix_b, n, b - total_a);
}

int batch_stage_threads(int stage) {
  switch (stage) {
    case kBsScan: return 1024;
    case kBsSpread: return kSpreadThreads;
    case kBsGather: return kGatherThreads;
    default: return PSWF_THREADS;
  }
}

// virtual blocks of one structure in one stage (0 when the stage is skipped)
int batch_stage_blocks(const BatchItem &it, int stage, bool adjoint) {
  const Geo &g = it.g;
  const int64_t N = g.N;
  switch (stage) {
    case kBsZero: return int(nblocks(g.ncell, PSWF_THREADS));
    case kBsBin: case kBsScatter: return N > 0 ? int(nblocks(N, PSWF_THREADS)) : 0;
    case kBsScan: case kBsQreduce: case kBsFinalize: return 1;
    case kBsOrder: return N > 0 ? g.ncell : 0;
    case kBsQsum: return it.qblocks * g.C;
    case kBsSpread: return g.ncell;
    case kBsZfwd: return int(nblocks(it.nlines, g.zlines));
    case kBsYfwd: return int(nblocks(g.KZ, g.kzq)) * int(nblocks(int64_t(g.C) * g.M[0], g.ypl));
    case kBsXmul: return g.nxblk * g.C;
    case kBsYinv: return adjoint ? int(nblocks(g.KZ, g.kzq)) * int(nblocks(int64_t(g.C) * g.M[0], g.ypl)) : 0;
    case kBsZinv: return adjoint ? int(nblocks(it.nlines, g.zlines)) : 0;
    case kBsGather: return (adjoint && N > 0) ? g.ncell : 0;
  }
  return 0;
}

size_t batch_stage_lds(const BatchItem &it, int stage) {
  switch (stage) {
    case kBsSpread: return spread_lds_bytes(it.g, it.g.C);
    case kBsZfwd: case kBsZinv: return zpass_lds_bytes(it.g);
    case kBsYfwd: case kBsYinv: return ypass_lds_bytes(it.g);
    case kBsXmul: return xpass_lds_bytes(it.g);
    case kBsGather: return gather_lds_bytes(it.g, it.g.CG_gather);
  }
  return 0;
}

// Spreading of a batch: one launch per kernel variant present in the batch,
// each over every block; a block whose structure has another variant
// returns at once.  The matrix-core variant has a launch per (support, z
// blocks); a vector-ALU variant (NBZ = 0 here) has one per (support,
// channel accumulators) and takes each structure's z-block count inside,
// so structures with different tile depths share one launch and its tail.
// One kernel holding every variant would be large and spill scalar
// registers.
template <int P, int NBZ, int CG>
__global__ __launch_bounds__(kSpreadThreads, NBZ == 0 ? 8 : 4) void k_batch_spread(const BatchItem *__restrict__ items,
                                                                     const int *__restrict__ prefix, int n) {
  const int b = blockIdx.x;
  const int s = find_item(prefix, n, b);
  const BatchItem &it = items[s];
  const Geo &g = it.g;
  if (g.P != P || spread_cg_template(g.C) != CG) return;
  const int vb = b - prefix[s];
  if constexpr (NBZ == 0) {
    switch (spread_nbz(g.B[2])) {
      case 1: spread_body<P, 1, CG>(g, it.t, it.w, 0, g.C, vb, SpreadSrc{}); break;
      case 2: spread_body<P, 2, CG>(g, it.t, it.w, 0, g.C, vb, SpreadSrc{}); break;
      default: spread_body<P, 4, CG>(g, it.t, it.w, 0, g.C, vb, SpreadSrc{}); break;
    }
  } else {
    if (spread_nbz(g.B[2]) != NBZ) return;
    spread_body<P, NBZ, CG>(g, it.t, it.w, 0, g.C, vb, SpreadSrc{});
  }
}

template <int P, int NBZ, int CG>
static hipError_t bspread_launch(const BatchItem *d_items, const int *d_prefix, int n, int total_blocks, size_t lds,
                                 hipStream_t st) {
  hipError_t e = lds_request(reinterpret_cast<const void *>(&k_batch_spread<P, NBZ, CG>), lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_batch_spread<P, NBZ, CG>), dim3(total_blocks), dim3(kSpreadThreads), lds, st, d_items,
                     d_prefix, n);
  LAUNCH_CHECK();
  return hipSuccess;
}

template <int P>
static hipError_t bspread_p(int nbz, int cgt, const BatchItem *d_items, const int *d_prefix, int n,
                            int total_blocks, size_t lds, hipStream_t st) {
  if (cgt == 2) return bspread_launch<P, 0, 2>(d_items, d_prefix, n, total_blocks, lds, st);
  if (cgt == 4) return bspread_launch<P, 0, 4>(d_items, d_prefix, n, total_blocks, lds, st);
  switch (nbz) {
    case 1: return bspread_launch<P, 1, kSpreadCGM>(d_items, d_prefix, n, total_blocks, lds, st);
    case 2: return bspread_launch<P, 2, kSpreadCGM>(d_items, d_prefix, n, total_blocks, lds, st);
    case 4: return bspread_launch<P, 4, kSpreadCGM>(d_items, d_prefix, n, total_blocks, lds, st);
  }
  return hipErrorInvalidValue;
}

// P * 100 + z blocks * 10 (matrix-core variant; 0 for the vector-ALU ones,
// which cover every z-block count) + channel accumulators (0 for 16)
int batch_spread_variant(const Geo &g) {
  const int cgt = spread_cg_template(g.C);
  return cgt == kSpreadCGM ? g.P * 100 + spread_nbz(g.B[2]) * 10 : g.P * 100 + cgt;
}

hipError_t launch_batch_spread(const BatchItem *d_items, const int *d_prefix, int n, int total_blocks, size_t lds,
                               int variant, hipStream_t st) {
  if (total_blocks <= 0) return hipSuccess;
  const int P = variant / 100, nbz = (variant / 10) % 10, cgv = variant % 10;
  const int cgt = cgv == 0 ? kSpreadCGM : cgv;
  switch (P) {
    case 2: return bspread_p<2>(nbz, cgt, d_items, d_prefix, n, total_blocks, lds, st);
    case 3: return bspread_p<3>(nbz, cgt, d_items, d_prefix, n, total_blocks, lds, st);
    case 4: return bspread_p<4>(nbz, cgt, d_items, d_prefix, n, total_blocks, lds, st);
    case 5: return bspread_p<5>(nbz, cgt, d_items, d_prefix, n, total_blocks, lds, st);
    case 6: return bspread_p<6>(nbz, cgt, d_items, d_prefix, n, total_blocks, lds, st);
    case 7: return bspread_p<7>(nbz, cgt, d_items, d_prefix, n, total_blocks, lds, st);
    case 8: return bspread_p<8>(nbz, cgt, d_items, d_prefix, n, total_blocks, lds, st);
  }
  return hipErrorInvalidValue;
}

template <int STAGE>
static hipError_t launch_stage_t(const BatchItem *d_items, const int *d_prefix, int n, int total_blocks, size_t lds,
                                 int mode, hipStream_t st) {
  constexpr int T = (STAGE == kBsScan) ? 1024 : (STAGE == kBsSpread ? kSpreadThreads
                                                                    : (STAGE == kBsGather ? kGatherThreads
                                                                                          : PSWF_THREADS));
  hipError_t e = lds_request(reinterpret_cast<const void *>(&k_batch<STAGE, T>), lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_batch<STAGE, T>), dim3(total_blocks), dim3(T), lds, st, d_items, d_prefix, n, mode);
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_batch_pair(const BatchItem *d_items, const int *d_prefix_a, int total_a, const int *d_prefix_b,
                             int total_b, int n, int stage_a, hipStream_t st) {
  const int total = total_a + total_b;
  if (total <= 0) return hipSuccess;
  if (stage_a == kBsBin)
    hipLaunchKernelGGL((k_batch_pair<kBsBin, kBsQsum>), dim3(total), dim3(PSWF_THREADS), 0, st, d_items, d_prefix_a,
                       total_a, d_prefix_b, n);
  else if (stage_a == kBsScatter)
    hipLaunchKernelGGL((k_batch_pair<kBsScatter, kBsQreduce>), dim3(total), dim3(PSWF_THREADS), 0, st, d_items,
                       d_prefix_a, total_a, d_prefix_b, n);
  else
    return hipErrorInvalidValue;
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_batch_stage(const BatchItem *d_items, const int *d_prefix, int n, int stage, int total_blocks,
                              size_t lds, int mode, hipStream_t st) {
  if (total_blocks <= 0) return hipSuccess;
  switch (stage) {
    case kBsZero: return launch_stage_t<kBsZero>(d_items, d_prefix, n, total_blocks, lds, mode, st);
    case kBsBin: return launch_stage_t<kBsBin>(d_items, d_prefix, n, total_blocks, lds, mode, st);
    case kBsScan: return launch_stage_t<kBsScan>(d_items, d_prefix, n, total_blocks, lds, mode, st);
    case kBsScatter: return launch_stage_t<kBsScatter>(d_items, d_prefix, n, total_blocks, lds, mode, st);
    case kBsOrder: return launch_stage_t<kBsOrder>(d_items, d_prefix, n, total_blocks, lds, mode, st);
    case kBsQsum: return launch_stage_t<kBsQsum>(d_items, d_prefix, n, total_blocks, lds, mode, st);
    case kBsQreduce: return launch_stage_t<kBsQreduce>(d_items, d_prefix, n, total_blocks, lds, mode, st);
    case kBsSpread: return hipErrorInvalidValue;  // launch_batch_spread
    case kBsZfwd: return launch_stage_t<kBsZfwd>(d_items, d_prefix, n, total_blocks, lds, mode, st);
    case kBsYfwd: return launch_stage_t<kBsYfwd>(d_items, d_prefix, n, total_blocks, lds, mode, st);
    case kBsXmul: return launch_stage_t<kBsXmul>(d_items, d_prefix, n, total_blocks, lds, mode, st);
    case kBsFinalize: return launch_stage_t<kBsFinalize>(d_items, d_prefix, n, total_blocks, lds, mode, st);
    case kBsYinv: return launch_stage_t<kBsYinv>(d_items, d_prefix, n, total_blocks, lds, mode, st);
    case kBsZinv: return launch_stage_t<kBsZinv>(d_items, d_prefix, n, total_blocks, lds, mode, st);
    case kBsGather: return launch_stage_t<kBsGather>(d_items, d_prefix, n, total_blocks, lds, mode, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace pswf
