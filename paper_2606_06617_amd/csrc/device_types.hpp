// Plain-data structures passed by value from the planner to the gfx950
// kernels.  No HIP or torch types here so that host-only translation units
// can include it.
#pragma once

#include <cmath>
#include <cstdint>

// functions the kernels share with host-side unit probes (built with g++)
#ifdef __HIPCC__
#define PSWF_HD __host__ __device__
#else
#define PSWF_HD
#endif

namespace pswf {

constexpr int kMaxRadixStages = 8;
constexpr int kMaxChannels = 64;   // channels per plan (the ABI limit)
constexpr int kWinSeg = 8;     // window polynomial: segments on |t| in [0, 1]
constexpr int kWinDeg = 11;    // degree per segment
constexpr int kKerSeg = 16;    // kernel polynomials: segments on kappa in [0, 1]
constexpr int kKerDeg = 11;
constexpr int kKerCoef = kKerSeg * (kKerDeg + 1);

// Division by a loop-invariant divisor d < 2^31 with a multiply-high
// (Granlund-Montgomery): q = (umulhi(n, m) + n) >> s for n < 2^31.
struct FastDiv {
  unsigned m = 0;
  int s = 0;
  int d = 1;
};
inline FastDiv make_fastdiv(int d) {
  FastDiv f;
  f.d = d;
  if (d <= 1) return f;
  int s = 0;
  while ((1u << s) < unsigned(d)) ++s;
  f.s = s;
  f.m = unsigned(((1ull << 32) * ((1ull << s) - unsigned(d))) / unsigned(d) + 1);
  return f;
}

// Window start from a grid coordinate u given as an unevaluated FP32 sum
// p + lo (see grid_coord).  The window covers the P nodes n0 .. n0 + P - 1
// with n0 = ceil(u - P/2); delta = n0 - (u - P/2) is in [0, 1) and n0 is
// returned wrapped into [0, M).  Coordinates a few cells outside keep their
// unwrapped value (only the integer start is wrapped, exactly); beyond 2^22
// grid units the whole multiple of M is removed from p first.
PSWF_HD inline void window_start_dw(float p, float lo, int M, int P, int *n0, float *delta) {
  const float Mf = float(M);
  if (std::fabs(p) >= 4194304.0f) p = std::fma(-std::floor(p / Mf), Mf, p);
  // s = u - P/2 = shi + slo by an error-free two-sum
  const float half = 0.5f * float(P);
  const float shi = p - half;
  const float bv = shi - p;
  const float slo = ((p - (shi - bv)) + (-half - bv)) + lo;
  float nf = std::ceil(shi);
  float d = (nf - shi) - slo;
  if (d < 0.0f) {
    nf += 1.0f;
    d += 1.0f;
  } else if (d >= 1.0f) {
    nf -= 1.0f;
    d -= 1.0f;
  }
  *delta = d < 0.0f ? 0.0f : (d > 0.99999994f ? 0.99999994f : d);
  int n = int(nf) % M;
  if (n < 0) n += M;
  *n0 = n;
}

// Grid coordinate of one axis, u = sum_b T_b r_b (T: one row of
// diag(M) H^-T, H the cell with lattice vectors as rows, so that u / M is the
// fractional coordinate), as an unevaluated FP32 sum hi + lo.  Each T_b is
// carried as two floats th + tl, each product's rounding error is recovered
// by an FMA and the three products are added by error-free two-sums, so u is
// good to ~1e-14 of the largest term (a plain FP32 product would lose ~3e-5
// grid units at M = 256).  Zero entries (an orthorhombic cell) add exact
// zeros.
PSWF_HD inline void grid_coord(const float r[3], const float *th, const float *tl, float *hi, float *lo) {
  float s = 0.0f, e = 0.0f;
  for (int b = 0; b < 3; ++b) {
    const float pr = r[b] * th[b];
    const float pe = std::fma(r[b], th[b], -pr) + r[b] * tl[b];
    const float t = s + pr;
    const float bv = t - s;
    const float err = (s - (t - bv)) + (pr - bv);
    s = t;
    e += err + pe;
  }
  *hi = s;
  *lo = e;
}

// Window start of one component of an orthorhombic position: u = x M / L
// with M / L = sh + sl (FP32 double word).
PSWF_HD inline void window_start(float x, float sh, float sl, int M, int P, int *n0, float *delta) {
  const float p = x * sh;
  const float lo = std::fma(x, sh, -p) + x * sl;
  window_start_dw(p, lo, M, P, n0, delta);
}

// Stockham factorisation of one transform length.
struct FftAxis {
  int n = 1;
  int nst = 0;
  int rad[kMaxRadixStages] = {0};
  FastDiv nsdiv[kMaxRadixStages];   // divisor = product of the radices before stage s
};

// Per-channel constants of the Fourier kernel (see host_math.hpp):
//   Phi     = A kappa^eA f(kappa) + B kappa^eB ln(kappa)
//   Phi'/k  = Cc kappa^eC g(kappa) + D kappa^eD ln(kappa)
struct KChan {
  float A, B, Cc, D;
  int eA, eB, eC, eD;
  int p;
  float zero_over_V;   // E_0 = zero_over_V * Q_net^2 (double on host)
  float pad[2];
};

// One problem geometry in a general (triclinic) cell H, lattice vectors as
// rows (an orthorhombic box is H = diag(L)).  Positions become grid
// coordinates u = T r, T = diag(M) H^-T, in FP32 double-word arithmetic;
// wave vectors are k = 2 pi H^-1 m for the integer frequencies m of the
// grid axes.
struct Geo {
  int C;                  // channels
  int64_t N;              // atoms
  int M[3];               // grid
  int Nz;                 // M_z / 2 (complex length of the z transform)
  int KZ;                 // half-spectrum z columns kept
  int KZP;                // row stride of the z-column arrays (KZ padded for aligned column blocks)
  int NY, FY;             // y frequencies kept: fy in [-FY, FY], NY = 2 FY + 1
  int P;                  // window support
  int B[3];               // tile edge per axis
  int nc[3];              // tiles per axis
  int ncell;
  double L[3];            // lattice vector lengths |a_a| (host side)
  float T_hi[9], T_lo[9]; // T[a][b] = M_a (H^-T)[a][b] = T_hi + T_lo (FP32 double word), row-major
  float gT[9];            // (2 / P) T[a][b]: window-argument derivative -> d/dr_b
  float kmat[9];          // k_b = sum_a kmat[3 b + a] m_a, kmat = 2 pi H^-1
  float kc2;              // k_c^2
  float kinv;             // r_c / c  (kappa = k * kinv)
  float invV;
  double V;
  int CG_spread;          // channels per spread pass
  int scap;               // candidates per flush of the vector-ALU spread (128 or 256)
  int CG_gather;          // channels per gather halo staging (1)
  int nxblk;              // blocks of the fused x pass
  int zlines;             // lines per z-pass block (power of two)
  int kb;                 // columns per y/x-pass block (power of two)
  int kb_log2;
  // generic y passes: blocks of kby columns made of ypl planes (c, x) of
  // kzq k_z columns each (kzq a power of two >= KZ when planes are packed,
  // else kzq = kby and ypl = 1); the 256-point register path uses kb
  int kby, kby_log2, kzq, kzq_log2, ypl;
  // generic fused x pass: blocks of kbx columns, made of whole runs of k_z
  // columns of one k_y row each (several rows per block on small grids)
  int kbx, kbx_log2;
  int srec;               // floats per staged atom record: 4 + C rounded up to 4
  FastDiv div_nz;         // by Nz
  FastDiv div_kz;         // by KZ
  FastDiv div_gez;        // by the gather halo's z extent B_z + P - 1
  FastDiv div_geyz;       // by its y-z plane (B_y + P - 1)(B_z + P - 1)
};

// Device pointers into a plan's table allocation.
struct Tables {
  const float *tw_z;      // [Nz] exp(-2 pi i n / Nz), as float2
  const float *tw_zr;     // [Nz + 1] exp(-2 pi i k / M_z), as float2
  const float *tw_y;      // [M_y] as float2
  const float *tw_x;      // [M_x] as float2
  const float *Dx;        // [M_x] h^2 / What_x^2 by array index
  const float *Dy;        // [NY]  by kept index
  const float *Dz;        // [KZ]
  const float *win;       // [kWinSeg][kWinDeg + 1]
  const float *kf;        // [C][kKerCoef]
  const float *kg;        // [C][kKerCoef]
  const KChan *kch;       // [C]
  const int *xblk;        // runs [nrun][4]: iy, kz0, ncols, first column in the block
  const int *xgrp;        // [nxblk + 1]: first run of each x-pass block
  const int *blim;        // [NY] z columns processed by the x pass per iy
  const double *self_coef;  // [C] E_self = self_coef * sum q^2
  const double *zero_V;     // [C] E_0 = zero_V / V * Q_net^2
};

// Workspace carve-up (device pointers), produced per call.
struct Work {
  float *grid;            // [C][Mx][My][Mz]
  float *s1;              // [C][Mx][My][KZP] complex
  float *s2;              // [C][Mx][NY][KZP] complex
  float *rec_a;           // [N][4] in cell order: delta_x, delta_y, delta_z, packed n0 bits
  float *q_a;             // [C][N] in cell order
  float *q_b;             // the sort's staging: [N][srec] records in caller order
  int *perm_a, *perm_b;   // cell order -> caller order
  int *cell_of, *slot;    // [N]
  int *cell_count;        // [ncell]
  int *cell_start;        // [ncell + 1]
  double *epart;          // [C][nxblk][8]
  double *qpart;          // [nqblk][C][2]
  double *qsum;           // [C][2]: Q_net, Q_self
  int *status;            // [2] input status: [0] bit 0 = a non-finite position met by
                          // the binning; [1] result of the optional input check
};

// Real-space complement of the split (Eq. realLR): the pair kernel
// K_p(r) = (1 - G_p(r / r_c)) / r^p for 0 < r < r_c over all periodic
// images.  Cells are a grid on the fractional coordinates, their widths
// across each lattice plane >= r_c (or the whole cell along an axis whose
// width is shorter than r_c); a cell's neighbours are the offsets -R..R on
// each axis, each offset one periodic image (shift by lattice vectors) of
// the cell it wraps to.
constexpr int kRsSeg = 16;   // complement polynomial: segments on rho in [0, 1]
constexpr int kRsDeg = 11;
constexpr int kRsCoef = kRsSeg * (kRsDeg + 1);
struct RsGeo {
  int C;
  int64_t N;
  int nc[3];              // cells per axis
  int R[3];               // neighbour offsets per axis
  int ncell;
  float A_hi[9], A_lo[9]; // lattice vectors (rows of H) as FP32 double words
  float Binv[9];          // rows of H^-T: fractional coordinate s_a = Binv[a] . r
  float rc, rc2, inv_rc;
  int srec;               // floats per atom record: position + pad, then C charges (multiple of 4)
};
struct RsTables {
  const float *ucoef;     // [C][kRsCoef] 1 - G_p on rho in [0, 1], per channel
  const int *pch;         // [C] exponent of each channel
};
struct RsWork {
  float *rec_b;           // [N][srec] caller order (wrapped positions, charges)
  float *rec_a;           // [N][srec] cell order
  int *perm_b, *perm_a;   // cell order -> caller order (unordered, ordered)
  int *cell_of, *slot;    // [N]
  int *count, *start;     // [ncell], [ncell + 1]
  double *part;           // [ncell][C + 6]: per-cell energy and virial partials
};

// Options of a spreading launch beyond the plain charge grid: another
// charge array (cell order [C][N]; NULL: the sorted charges), the axis whose
// window factor is replaced by its derivative (-1: none), and whether the
// result is added to the grid instead of stored.
struct SpreadSrc {
  const float *q = nullptr;
  int dax = -1;
  int acc = 0;
};

// One structure of a batched call: everything a stage body needs.
struct BatchItem {
  Geo g;
  Tables t;
  Work w;
  FftAxis az, ay, ax;
  const float *pos;
  const float *q;
  double *energy;
  float *forces;
  double *virial;
  float *pot;
  int qblocks;
  int mode;               // x pass: 0 energy only, 1 energy + potential grid, 2 adjoint
  int64_t nlines;
  const double *grad;     // adjoint calls: dL/dE per channel (device), else NULL
};

// Stages of one evaluation, in launch order.
enum BatchStage {
  kBsZero = 0, kBsBin, kBsScan, kBsScatter, kBsOrder, kBsQsum, kBsQreduce, kBsSpread, kBsZfwd, kBsYfwd,
  kBsXmul, kBsFinalize, kBsYinv, kBsZinv, kBsGather, kNumBatchStages
};

}  // namespace pswf
