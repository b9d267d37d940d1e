// Planner and C ABI of the PSWF-LR path (declared in include/pswflr.h).
//
// Plan creation does all FP64 host work once: parameter selection (Methods,
// "Parameter selection"), the PSWF window and kernel polynomial tables, the
// deconvolution tables h^2 / What_a^2, FFT factorisations, the pruned
// x-pass block list and the workspace layout.  Execute calls only enqueue
// kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "device_types.hpp"
#include "host_math.hpp"
#include "kernels.hpp"
#include "pswflr.h"

using namespace pswf;

static_assert(kMaxChannels == PSWFLR_MAX_CHANNELS, "device channel limit follows the ABI");

namespace {

const double kPi = 3.14159265358979323846264338327950288;
thread_local std::string g_last_error;

// Plan tables come from a per-process pool of device blocks: a destroyed
// plan's block is kept for the next plan instead of being freed, because
// hipFree waits for the whole device and would stall every stream in
// flight (a serving loop retires plans while other requests run).  The
// pool holds at most what the peak number of live plans used.
std::mutex g_table_mu;
// A released block carries the event recorded after its plan's last call;
// it is handed out again only once that event has completed (otherwise a
// new block is allocated: no call ever waits here).  Events are one
// per stream, kept for the life of the process and re-recorded by every
// call on that stream: a later record only makes the wait longer, never
// shorter, since work on one stream completes in order.
std::mutex g_event_mu;
std::map<void *, hipEvent_t> g_stream_events;

hipError_t stream_event(hipStream_t st, hipEvent_t *out) {
  std::lock_guard<std::mutex> lock(g_event_mu);
  auto it = g_stream_events.find(static_cast<void *>(st));
  if (it != g_stream_events.end()) {
    *out = it->second;
    return hipSuccess;
  }
  hipEvent_t ev = nullptr;
  hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  if (e != hipSuccess) return e;
  g_stream_events.emplace(static_cast<void *>(st), ev);
  *out = ev;
  return hipSuccess;
}

struct PooledTable {
  int device;
  void *block;
  hipEvent_t done;
};
std::multimap<size_t, PooledTable> g_table_pool;  // capacity -> block

// Plan tables come in power-of-two size classes (at least 4 KiB) carved
// from device arenas of 8 MiB, held until the process ends, so creating a
// plan for a new box costs no hipMalloc once the arenas exist (a serving
// loop builds a plan per request).
struct TableArena {
  int device;
  char *base;
  size_t size, used;
};
std::vector<TableArena> g_table_arenas;
constexpr size_t kTableArenaBytes = size_t(8) << 20;

size_t table_class(size_t bytes) {
  size_t c = 4096;
  while (c < bytes) c <<= 1;
  return c;
}

hipError_t table_alloc(size_t bytes, int device, void **out, size_t *cap) {
  const size_t cls = table_class(bytes);
  std::lock_guard<std::mutex> lock(g_table_mu);
  auto range = g_table_pool.equal_range(cls);
  for (auto it = range.first; it != range.second; ++it) {
    if (it->second.device != device) continue;
    // only a block whose last use has completed: never wait here (the
    // stream's event may stand for newer work queued behind it)
    if (it->second.done && hipEventQuery(it->second.done) != hipSuccess) continue;
    *out = it->second.block;
    *cap = cls;
    g_table_pool.erase(it);
    return hipSuccess;
  }
  for (auto &a : g_table_arenas) {
    if (a.device == device && a.used + cls <= a.size) {
      *out = a.base + a.used;
      a.used += cls;
      *cap = cls;
      return hipSuccess;
    }
  }
  TableArena a{device, nullptr, std::max(kTableArenaBytes, cls), 0};
  hipError_t e = hipMalloc(reinterpret_cast<void **>(&a.base), a.size);
  if (e != hipSuccess) return e;
  *out = a.base;
  a.used = cls;
  *cap = cls;
  g_table_arenas.push_back(a);
  return hipSuccess;
}

void table_release(void *p, size_t cap, int device, hipEvent_t done) {
  if (!p) return;
  std::lock_guard<std::mutex> lock(g_table_mu);
  g_table_pool.emplace(cap, PooledTable{device, p, done});
}

pswflr_status fail(pswflr_status s, const std::string &msg) {
  g_last_error = msg;
  return s;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

FftAxis factorise(int n, bool *ok) {
  FftAxis ax;
  ax.n = n;
  int m = n, a = 0;
  while (m % 2 == 0) { m /= 2; ++a; }
  std::vector<int> r;
  // powers of two as radix 8 and 4 stages (a lone radix-2 stage only for n = 2)
  if (a == 1) {
    r.push_back(2);
    a = 0;
  }
  if (a % 3 == 1) { r.push_back(4); r.push_back(4); a -= 4; }
  if (a % 3 == 2) { r.push_back(4); a -= 2; }
  while (a >= 3) { r.insert(r.begin(), 8); a -= 3; }
  while (m % 3 == 0) { r.push_back(3); m /= 3; }
  while (m % 5 == 0) { r.push_back(5); m /= 5; }
  *ok = (m == 1) && int(r.size()) <= kMaxRadixStages;
  ax.nst = int(r.size());
  int ns = 1;
  for (size_t i = 0; i < r.size() && i < size_t(kMaxRadixStages); ++i) {
    ax.rad[i] = r[i];
    ax.nsdiv[i] = make_fastdiv(ns);
    ns *= r[i];
  }
  return ax;
}

int floor_pow2(int x) {
  int p = 1;
  while (p * 2 <= x) p *= 2;
  return p;
}

// Largest divisor of m in [lo, hi]; 0 if none.
int divisor_in(int m, int lo, int hi) {
  for (int d = std::min(hi, m); d >= std::max(1, lo); --d)
    if (m % d == 0) return d;
  return 0;
}

}  // namespace

struct pswflr_plan_s {
  pswflr_params prm{};
  pswflr_info info{};
  Geo geo{};
  FftAxis az, ay, ax;
  Tables tab{};
  double hinv[9] = {0};   // H^-1 row-major (cell gradient)
  void *dtab = nullptr;
  size_t dtab_bytes = 0;  // capacity of the block dtab points to
  hipEvent_t last_use = nullptr;  // the stream event recorded after its last call (not owned)
  int device = 0;
  // workspace layout for max_atoms
  int64_t max_atoms = 0;
  size_t off_grid = 0, off_s1 = 0, off_s2 = 0, off_rec_a = 0, off_q_a = 0, off_q_b = 0,
         off_perm_a = 0, off_perm_b = 0, off_cell_of = 0, off_slot = 0, off_count = 0, off_start = 0,
         off_epart = 0, off_qpart = 0, off_qsum = 0, off_status = 0, ws_bytes = 0;
  // real-space complement: geometry, tables (in the plan's device block) and
  // workspace regions
  RsGeo rsg{};
  RsTables rst{};
  const int *rs_grp = nullptr, *rs_gch = nullptr;
  int rs_ngrp = 0, rs_cgmax = 0;
  size_t off_rs_rec_b = 0, off_rs_rec_a = 0, off_rs_perm_b = 0, off_rs_perm_a = 0, off_rs_cell_of = 0,
         off_rs_slot = 0, off_rs_count = 0, off_rs_start = 0, off_rs_part = 0;
  size_t off_dd = 0;  // scratch of the second-derivative call: [3 C N + C N + 3 N] floats
  // optional per-stage event timing (measurement only)
  uint32_t prof_mask = 0;  // bit s: launches of stage s are timed
  std::mutex prof_mu;
  std::vector<std::tuple<int, hipEvent_t, hipEvent_t>> prof_ev;
};

namespace {

pswflr_status build_plan(const pswflr_params &in, int64_t max_atoms, pswflr_plan_s &pl) {
  pswflr_params p = in;
  if (p.n_channels < 1 || p.n_channels > PSWFLR_MAX_CHANNELS)
    return fail(PSWFLR_ERR_INVALID_ARG, "n_channels must be in 1..64");
  for (int c = 0; c < p.n_channels; ++c)
    if (p.p[c] < 1 || p.p[c] > 6) return fail(PSWFLR_ERR_INVALID_ARG, "exponent p must be in 1..6");
  // the cell H, lattice vectors as rows (the cell tensor); an all-zero
  // cell means the orthorhombic box diag(box)
  double H[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  bool general = false;
  for (int i = 0; i < 9; ++i) general = general || p.cell[i] != 0.0;
  if (general && p.cell[1] == 0.0 && p.cell[2] == 0.0 && p.cell[3] == 0.0 && p.cell[5] == 0.0 &&
      p.cell[6] == 0.0 && p.cell[7] == 0.0 && p.cell[0] > 0.0 && p.cell[4] > 0.0 && p.cell[8] > 0.0) {
    // a diagonal cell is the orthorhombic box (same plan, same bits)
    general = false;
    p.box[0] = p.cell[0];
    p.box[1] = p.cell[4];
    p.box[2] = p.cell[8];
  }
  if (general) {
    for (int i = 0; i < 9; ++i) {
      if (!std::isfinite(p.cell[i])) return fail(PSWFLR_ERR_INVALID_ARG, "cell entries must be finite");
      H[i / 3][i % 3] = p.cell[i];
    }
  } else {
    for (int a = 0; a < 3; ++a) {
      if (!(p.box[a] > 0.0) || !std::isfinite(p.box[a])) return fail(PSWFLR_ERR_INVALID_ARG, "box edges must be > 0");
      H[a][a] = p.box[a];
    }
  }
  const double det = H[0][0] * (H[1][1] * H[2][2] - H[1][2] * H[2][1]) -
                     H[0][1] * (H[1][0] * H[2][2] - H[1][2] * H[2][0]) +
                     H[0][2] * (H[1][0] * H[2][1] - H[1][1] * H[2][0]);
  double len[3], wid[3], Hinv[3][3];
  for (int a = 0; a < 3; ++a) {
    len[a] = std::sqrt(H[a][0] * H[a][0] + H[a][1] * H[a][1] + H[a][2] * H[a][2]);
    // width of the cell across the plane of the other two lattice vectors
    const int b = (a + 1) % 3, c2 = (a + 2) % 3;
    const double cx = H[b][1] * H[c2][2] - H[b][2] * H[c2][1], cy = H[b][2] * H[c2][0] - H[b][0] * H[c2][2],
                 cz = H[b][0] * H[c2][1] - H[b][1] * H[c2][0];
    wid[a] = std::fabs(det) / std::sqrt(cx * cx + cy * cy + cz * cz);
    // column a of H^-1 is the cross product of rows b and c over det
    Hinv[0][a] = cx / det;
    Hinv[1][a] = cy / det;
    Hinv[2][a] = cz / det;
  }
  if (!(std::fabs(det) > 0.0) || !std::isfinite(det))
    return fail(PSWFLR_ERR_INVALID_ARG, "the cell must have non-zero volume");
  // widths far below the lengths: a degenerate cell (reduce the lattice basis first)
  for (int a = 0; a < 3; ++a)
    if (!(wid[a] > 1e-3 * len[a])) return fail(PSWFLR_ERR_INVALID_ARG, "cell too skewed: reduce its lattice basis");
  if (!(p.r_c > 0.0) || !std::isfinite(p.r_c)) return fail(PSWFLR_ERR_INVALID_ARG, "r_c must be > 0");
  if (max_atoms < 0 || max_atoms > (int64_t(1) << 31) - 1)
    return fail(PSWFLR_ERR_INVALID_ARG, "max_atoms must be in [0, 2^31)");
  const bool need_tol = !(p.c > 0.0) || p.grid[0] <= 0 || p.grid[1] <= 0 || p.grid[2] <= 0 || p.support <= 0;
  if (need_tol && !(p.tol > 0.0 && p.tol <= 0.1))
    return fail(PSWFLR_ERR_INVALID_ARG, "tol must be in (0, 0.1] when c, grid or support are automatic");
  if (p.support != 0 && (p.support < 2 || p.support > 8))
    return fail(PSWFLR_ERR_INVALID_ARG, "support P must be in 2..8");
  if (p.flags & ~uint32_t(PSWFLR_FLAG_CHECK_INPUTS)) return fail(PSWFLR_ERR_INVALID_ARG, "unknown flag bits");

  // bandwidth c ~ log(1/eps_band) with eps_band = tol / 3
  const double c = p.c > 0.0 ? p.c : std::log(3.0 / p.tol);
  const double kc = c / p.r_c;
  int M[3];
  for (int a = 0; a < 3; ++a) {
    if (p.grid[a] > 0) {
      M[a] = p.grid[a];
    } else {
      // h <= eta pi / k_c with eta = 0.6, rounded up to a 2,3,5-smooth size
      const double hmax = 0.6 * kPi / kc;
      M[a] = smooth_size(len[a] / hmax, a == 2);
    }
    if (M[a] > PSWFLR_MAX_GRID) return fail(PSWFLR_ERR_UNSUPPORTED, "grid edge exceeds 1024");
    if (!is_smooth235(M[a])) return fail(PSWFLR_ERR_UNSUPPORTED, "grid edges must factor into 2, 3 and 5");
  }
  if (M[2] % 2) return fail(PSWFLR_ERR_UNSUPPORTED, "M_z must be even (real-to-complex transform)");
  // one channel's grid is addressed with 32-bit byte offsets
  if (int64_t(M[0]) * M[1] * M[2] >= (int64_t(1) << 30))
    return fail(PSWFLR_ERR_UNSUPPORTED, "a channel's grid must hold fewer than 2^30 points");
  double eta = 0.0, h[3];
  for (int a = 0; a < 3; ++a) {
    // the ball's largest frequency along grid axis a is k_c |a_a| / 2 pi
    h[a] = len[a] / M[a];
    eta = std::max(eta, kc * h[a] / kPi);
  }
  if (!(eta < 1.0))
    return fail(PSWFLR_ERR_INVALID_ARG, "grid too coarse: need k_c h / pi < 1 on every axis (Nyquist)");
  int P = p.support;
  double cs = p.c_spread;
  if (P <= 0) {
    // smallest P whose estimated force error (about 25x the aliasing
    // estimate, bounded from above on a cached grid of eta) stays below
    // eps_spread = tol / 3
    P = 8;
    for (int cand = 4; cand <= 8; ++cand) {
      if (25.0 * spread_error_bound(cand, eta, c) <= p.tol / 3.0) {
        P = cand;
        break;
      }
    }
  }
  for (int a = 0; a < 3; ++a)
    if (M[a] < P) return fail(PSWFLR_ERR_INVALID_ARG, "every grid edge must be >= support P");
  if (!(cs > 0.0)) cs = choose_c_spread(P, eta, c);

  const int C = p.n_channels;
  Geo &g = pl.geo;
  g = Geo{};
  g.C = C;
  g.N = 0;
  for (int a = 0; a < 3; ++a) {
    g.M[a] = M[a];
    g.L[a] = len[a];
    for (int b = 0; b < 3; ++b) {
      // T = diag(M) H^-T: u_a = sum_b T[a][b] r_b
      const double T = general ? double(M[a]) * Hinv[b][a] : (a == b ? double(M[a]) / p.box[a] : 0.0);
      g.T_hi[3 * a + b] = float(T);
      g.T_lo[3 * a + b] = float(T - double(g.T_hi[3 * a + b]));
      g.gT[3 * a + b] = float(2.0 / P * T);
      // k = 2 pi H^-1 m: kmat[b][a]
      g.kmat[3 * b + a] = float(2.0 * kPi * (general ? Hinv[b][a] : (a == b ? 1.0 / p.box[a] : 0.0)));
    }
  }
  g.Nz = M[2] / 2;
  g.P = P;
  g.V = std::fabs(det);
  g.invV = float(1.0 / g.V);
  g.kc2 = float(kc * kc);
  g.kinv = float(p.r_c / c);
  // pruned spectrum extents (ball |k| <= k_c strictly inside Nyquist)
  const int kzmax = int(std::floor(kc * len[2] / (2 * kPi)));
  g.KZ = std::min(kzmax + 1, g.Nz);
  g.FY = std::min(int(std::floor(kc * len[1] / (2 * kPi))), (M[1] - 1) / 2);
  g.NY = 2 * g.FY + 1;

  // tiles (binning cells): over all divisor triples, maximise the fraction
  // of useful window work prod B / (B + P - 1) subject to the spreading
  // kernel's register blocks and the gather's LDS halo tile; ties go to the
  // larger tile
  {
    auto divisors = [](int m) {
      std::vector<int> d;
      for (int k = 1; k <= m; ++k)
        if (m % k == 0) d.push_back(k);
      return d;
    };
    double best_eff = -1.0;
    long best_vol = 0;
    int best[3] = {0, 0, 0};
    for (int bx : divisors(M[0]))
      for (int by : divisors(M[1]))
        for (int bz : divisors(M[2])) {
          if (!spread_tile_ok(bx, by, bz) || !gather_tile_ok(bx, by, bz, P)) continue;
          {
            const int b3[3] = {bx, by, bz}, n3[3] = {M[0] / bx, M[1] / by, M[2] / bz};
            if (spread_candidate_cells(n3, b3, P) > spread_max_cells()) continue;
          }
          const double eff = double(bx) / (bx + P - 1) * double(by) / (by + P - 1) * double(bz) / (bz + P - 1);
          const long vol = long(bx) * by * bz;
          if (eff > best_eff + 1e-12 || (std::fabs(eff - best_eff) <= 1e-12 && vol > best_vol)) {
            best_eff = eff;
            best_vol = vol;
            best[0] = bx; best[1] = by; best[2] = bz;
          }
        }
    if (p.tile[0] > 0 || p.tile[1] > 0 || p.tile[2] > 0) {
      for (int a = 0; a < 3; ++a) {
        const int b = p.tile[a] > 0 ? p.tile[a] : best[a];
        if (b <= 0 || M[a] % b != 0) return fail(PSWFLR_ERR_INVALID_ARG, "tile edges must divide the grid");
        best[a] = b;
      }
      {
        const int n3[3] = {M[0] / best[0], M[1] / best[1], M[2] / best[2]};
        if (spread_candidate_cells(n3, best, P) > spread_max_cells())
          return fail(PSWFLR_ERR_UNSUPPORTED, "tile too small for the support: too many candidate cells");
      }
      if (!spread_tile_ok(best[0], best[1], best[2]))
        return fail(PSWFLR_ERR_UNSUPPORTED, "tile exceeds the spreading kernel's 32 4x4x4 blocks");
      if (!gather_tile_ok(best[0], best[1], best[2], P))
        return fail(PSWFLR_ERR_UNSUPPORTED, "tile halo exceeds the gather kernel's LDS staging");
      best_eff = 0.0;
    }
    if (best_eff < 0) return fail(PSWFLR_ERR_UNSUPPORTED, "no tile shape fits this grid");
    for (int a = 0; a < 3; ++a) {
      g.B[a] = best[a];
      g.nc[a] = M[a] / best[a];
    }
  }
  g.ncell = g.nc[0] * g.nc[1] * g.nc[2];
  g.scap = spread_flush_cap(g.ncell);
  // channel groups: the spreading kernel keeps kSpreadCGM channels in
  // registers (groups are balanced); the gather walks all channels, one
  // staged halo tile at a time.
  const size_t kLds = 160 * 1024;
  g.CG_spread = std::min(C, spread_max_channels());
  g.CG_gather = 1;  // the gather stages one channel's halo tile at a time
  if (gather_lds_bytes(g, 1) > kLds) return fail(PSWFLR_ERR_UNSUPPORTED, "gather tile too large for LDS");
  {
    const int ng = (C + g.CG_spread - 1) / g.CG_spread;
    g.CG_spread = (C + ng - 1) / ng;
  }
  if (spread_lds_bytes(g, g.CG_spread) > kLds) return fail(PSWFLR_ERR_UNSUPPORTED, "spread staging exceeds LDS");
  g.kb = std::max(1, std::min(16, floor_pow2(4096 / std::max(M[0], M[1]))));
  g.kb_log2 = 0;
  while ((1 << g.kb_log2) < g.kb) ++g.kb_log2;
  // z-column arrays: rows padded so that each block of kb columns starts on
  // a kb * 8-byte (at least 64-byte) boundary
  {
    const int al = std::max(g.kb, 8);
    g.KZP = (g.KZ + al - 1) / al * al;
  }
  // generic y passes: when a plane has few k_z columns, a block takes
  // several planes so it still holds up to 4096 elements
  g.kby = std::max(1, std::min(64, floor_pow2(4096 / M[1])));
  {
    int q = 1;
    while (q < g.KZ) q <<= 1;
    if (q <= g.kby / 2) {
      g.kzq = q;
      g.ypl = g.kby / q;
    } else {
      g.kby = g.kb;
      g.kzq = g.kb;
      g.ypl = 1;
    }
  }
  g.kby_log2 = 0;
  while ((1 << g.kby_log2) < g.kby) ++g.kby_log2;
  g.kzq_log2 = 0;
  while ((1 << g.kzq_log2) < g.kzq) ++g.kzq_log2;
  g.srec = 4 + (C + 3) / 4 * 4;
  g.zlines = std::max(1, floor_pow2(4096 / g.Nz));
  g.div_nz = make_fastdiv(g.Nz);
  g.div_kz = make_fastdiv(g.KZ);
  g.div_gez = make_fastdiv(g.B[2] + P - 1);
  g.div_geyz = make_fastdiv((g.B[1] + P - 1) * (g.B[2] + P - 1));
  bool ok1, ok2, ok3;
  pl.az = factorise(g.Nz, &ok1);
  pl.ay = factorise(M[1], &ok2);
  pl.ax = factorise(M[0], &ok3);
  if (!(ok1 && ok2 && ok3)) return fail(PSWFLR_ERR_UNSUPPORTED, "transform length not supported");
  if (g.Nz > 4096 || M[0] > 4096 || M[1] > 4096) return fail(PSWFLR_ERR_UNSUPPORTED, "transform too long");

  // x-pass runs: for each kept k_y, the k_z prefix inside the ball in runs
  // of at most one block width; blocks take whole runs (the register path:
  // one run each; the generic path packs short rows of small grids)
  const bool xreg = x_register_path(g);
  g.kbx = xreg ? g.kb : std::max(g.kb, std::min(64, floor_pow2(4096 / M[0])));
  g.kbx_log2 = 0;
  while ((1 << g.kbx_log2) < g.kbx) ++g.kbx_log2;
  const int xstep = xreg ? g.kb : g.kbx;
  std::vector<int> xblk, xgrp, blim(g.NY, 0);
  int fill = g.kbx;  // columns used in the open block
  // |k|^2 = m^T G m with G = (2 pi)^2 H^-T H^-1; minimised over m_x it is
  // the quadratic form S (Schur complement) in (m_y, m_z)
  double G[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double v = 0.0;
      for (int e = 0; e < 3; ++e)
        v += (general ? Hinv[e][a] : (e == a ? 1.0 / p.box[a] : 0.0)) *
             (general ? Hinv[e][b] : (e == b ? 1.0 / p.box[b] : 0.0));
      G[a][b] = 4.0 * kPi * kPi * v;
    }
  const double Syy = G[1][1] - G[1][0] * G[0][1] / G[0][0], Syz = G[1][2] - G[1][0] * G[0][2] / G[0][0],
               Szz = G[2][2] - G[2][0] * G[0][2] / G[0][0];
  for (int iy = 0; iy < g.NY; ++iy) {
    const int fy = iy <= g.FY ? iy : iy - g.NY;
    // k_z columns 0 .. the largest m_z with some m_x inside the ball
    const double disc = Syz * Syz * fy * fy - Szz * (Syy * fy * fy - kc * kc);
    if (disc < 0) continue;
    const double zhi = (-Syz * fy + std::sqrt(disc)) / Szz;
    if (zhi < 0) continue;
    const int kzl = std::min(g.KZ - 1, int(std::floor(zhi)));
    for (int kz0 = 0; kz0 <= kzl; kz0 += xstep) {
      const int ncol = std::min(xstep, g.KZ - kz0);
      if (xreg || fill + ncol > g.kbx) {
        xgrp.push_back(int(xblk.size() / 4));
        fill = 0;
      }
      xblk.insert(xblk.end(), {iy, kz0, ncol, fill});
      fill += ncol;
      blim[iy] = kz0 + ncol;
    }
  }
  g.nxblk = int(xgrp.size());
  xgrp.push_back(int(xblk.size() / 4));

  // ---- tables (host FP64 -> device FP32) ----
  auto wpoly = make_window_poly(cs, kWinSeg, kWinDeg, 1e-9);
  std::vector<ChannelKernel> kers;
  for (int ch = 0; ch < C; ++ch) kers.push_back(make_channel_kernel(p.p[ch], c, p.r_c, 1e-9));

  auto twiddles = [](int n, int denom) {
    std::vector<float> t(2 * size_t(n));
    for (int m = 0; m < n; ++m) {
      t[2 * m] = float(std::cos(-2 * kPi * m / denom));
      t[2 * m + 1] = float(std::sin(-2 * kPi * m / denom));
    }
    return t;
  };
  // h^2 / What_a^2 = (2 / (P window_ft(pi P f / M)))^2, tabulated per
  // (c_s, P, M) and shared by every box with those (host cache)
  const auto dtx = deconvolution_cached(cs, P, M[0]), dty = deconvolution_cached(cs, P, M[1]),
             dtz = deconvolution_cached(cs, P, M[2]);
  std::vector<float> tw_z = twiddles(g.Nz, g.Nz), tw_zr = twiddles(g.Nz + 1, M[2]), tw_y = twiddles(M[1], M[1]),
                     tw_x = twiddles(M[0], M[0]);
  std::vector<float> Dx(M[0]), Dy(g.NY), Dz(g.KZ);
  for (int i = 0; i < M[0]; ++i) Dx[i] = (*dtx)[i <= M[0] / 2 ? i : M[0] - i];
  for (int i = 0; i < g.NY; ++i) Dy[i] = (*dty)[i <= g.FY ? i : g.NY - i];
  for (int i = 0; i < g.KZ; ++i) Dz[i] = (*dtz)[i];
  std::vector<float> win(kWinSeg * (kWinDeg + 1));
  for (size_t i = 0; i < win.size(); ++i) win[i] = float(wpoly.coef[i]);
  std::vector<float> kf(size_t(C) * kKerCoef), kg(size_t(C) * kKerCoef);
  std::vector<KChan> kch(C);
  std::vector<double> selfc(C), zerov(C);
  for (int ch = 0; ch < C; ++ch) {
    const auto &k = kers[ch];
    for (int i = 0; i < kKerCoef; ++i) {
      kf[size_t(ch) * kKerCoef + i] = float(k.f.coef[i]);
      kg[size_t(ch) * kKerCoef + i] = float(k.g.coef[i]);
    }
    KChan kc1{};
    kc1.A = float(k.A); kc1.B = float(k.B); kc1.Cc = float(k.Cc); kc1.D = float(k.D);
    kc1.eA = k.eA; kc1.eB = k.eB; kc1.eC = k.eC; kc1.eD = k.eD;
    kc1.p = k.p;
    kc1.zero_over_V = float(k.zero_coef_V / g.V);
    kch[ch] = kc1;
    selfc[ch] = k.self_coef;
    zerov[ch] = k.zero_coef_V;
  }
  // real-space complement 1 - G_p per distinct exponent, channel groups of
  // one exponent (at most 16 channels each)
  std::vector<int> rs_pdist, rs_grp, rs_gch;
  for (int ch = 0; ch < C; ++ch)
    if (std::find(rs_pdist.begin(), rs_pdist.end(), p.p[ch]) == rs_pdist.end()) rs_pdist.push_back(p.p[ch]);
  std::vector<float> rs_u(rs_pdist.size() * kRsCoef);
  int rs_cgmax = 0;
  for (size_t e = 0; e < rs_pdist.size(); ++e) {
    const PiecewisePoly up = make_complement_poly(rs_pdist[e], c, kRsSeg, kRsDeg, 1e-9);
    for (int i = 0; i < kRsCoef; ++i) rs_u[e * kRsCoef + i] = float(up.coef[i]);
    std::vector<int> chans;
    for (int ch = 0; ch < C; ++ch)
      if (p.p[ch] == rs_pdist[e]) chans.push_back(ch);
    for (size_t b0 = 0; b0 < chans.size(); b0 += 16) {
      const int cnt = int(std::min<size_t>(16, chans.size() - b0));
      rs_grp.insert(rs_grp.end(), {rs_pdist[e], int(rs_gch.size()), cnt, int(e)});
      rs_gch.insert(rs_gch.end(), chans.begin() + b0, chans.begin() + b0 + cnt);
      rs_cgmax = std::max(rs_cgmax, cnt);
    }
  }
  // pack
  std::vector<char> blob;
  auto put = [&](const void *src, size_t bytes) {
    size_t off = align256(blob.size());
    blob.resize(off + bytes);
    if (bytes) std::memcpy(blob.data() + off, src, bytes);
    return off;
  };
  size_t o_twz = put(tw_z.data(), tw_z.size() * 4), o_twzr = put(tw_zr.data(), tw_zr.size() * 4),
         o_twy = put(tw_y.data(), tw_y.size() * 4), o_twx = put(tw_x.data(), tw_x.size() * 4),
         o_dx = put(Dx.data(), Dx.size() * 4), o_dy = put(Dy.data(), Dy.size() * 4),
         o_dz = put(Dz.data(), Dz.size() * 4), o_win = put(win.data(), win.size() * 4),
         o_kf = put(kf.data(), kf.size() * 4), o_kg = put(kg.data(), kg.size() * 4),
         o_kch = put(kch.data(), kch.size() * sizeof(KChan)),
         o_xb = put(xblk.data(), std::max<size_t>(1, xblk.size()) * 4 * (xblk.empty() ? 0 : 1)),
         o_xg = put(xgrp.data(), xgrp.size() * 4),
         o_bl = put(blim.data(), blim.size() * 4), o_self = put(selfc.data(), selfc.size() * 8),
         o_zero = put(zerov.data(), zerov.size() * 8), o_rsu = put(rs_u.data(), rs_u.size() * 4),
         o_rsg = put(rs_grp.data(), rs_grp.size() * 4), o_rsc = put(rs_gch.data(), rs_gch.size() * 4),
         o_rsp = put(p.p, size_t(C) * 4);
  blob.resize(align256(blob.size()) + 256);
  if (hipGetDevice(&pl.device) != hipSuccess) return fail(PSWFLR_ERR_DEVICE, "hipGetDevice failed");
  if (table_alloc(blob.size(), pl.device, &pl.dtab, &pl.dtab_bytes) != hipSuccess) {
    pl.dtab = nullptr;
    return fail(PSWFLR_ERR_OOM, "table allocation failed");
  }
  if (hipMemcpy(pl.dtab, blob.data(), blob.size(), hipMemcpyHostToDevice) != hipSuccess)
    return fail(PSWFLR_ERR_DEVICE, "table upload failed");

  char *b = static_cast<char *>(pl.dtab);
  Tables &t = pl.tab;
  t.tw_z = reinterpret_cast<const float *>(b + o_twz);
  t.tw_zr = reinterpret_cast<const float *>(b + o_twzr);
  t.tw_y = reinterpret_cast<const float *>(b + o_twy);
  t.tw_x = reinterpret_cast<const float *>(b + o_twx);
  t.Dx = reinterpret_cast<const float *>(b + o_dx);
  t.Dy = reinterpret_cast<const float *>(b + o_dy);
  t.Dz = reinterpret_cast<const float *>(b + o_dz);
  t.win = reinterpret_cast<const float *>(b + o_win);
  t.kf = reinterpret_cast<const float *>(b + o_kf);
  t.kg = reinterpret_cast<const float *>(b + o_kg);
  t.kch = reinterpret_cast<const KChan *>(b + o_kch);
  t.xblk = reinterpret_cast<const int *>(b + o_xb);
  t.xgrp = reinterpret_cast<const int *>(b + o_xg);
  t.blim = reinterpret_cast<const int *>(b + o_bl);
  t.self_coef = reinterpret_cast<const double *>(b + o_self);
  t.zero_V = reinterpret_cast<const double *>(b + o_zero);
  pl.rst.ucoef = reinterpret_cast<const float *>(b + o_rsu);
  pl.rst.pch = reinterpret_cast<const int *>(b + o_rsp);
  pl.rs_grp = reinterpret_cast<const int *>(b + o_rsg);
  pl.rs_gch = reinterpret_cast<const int *>(b + o_rsc);
  pl.rs_ngrp = int(rs_grp.size() / 4);
  pl.rs_cgmax = rs_cgmax;
  {
    // cells of edge >= r_c (the whole box along a shorter axis), fewer than
    // max(64, max_atoms) cells in all; neighbour offsets -R..R
    RsGeo &rg = pl.rsg;
    rg = RsGeo{};
    rg.C = C;
    double edge_min = p.r_c;
    for (;;) {
      int64_t tot = 1;
      for (int a = 0; a < 3; ++a) tot *= std::max(1, int(std::floor(wid[a] / edge_min)));
      if (tot <= std::max<int64_t>(64, max_atoms)) break;
      edge_min *= 1.25;
    }
    rg.ncell = 1;
    for (int a = 0; a < 3; ++a) {
      // a vector of length r has fractional component <= r / wid[a] along a
      rg.nc[a] = std::max(1, int(std::floor(wid[a] / edge_min)));
      const double edge = wid[a] / rg.nc[a];
      rg.R[a] = std::max(1, int(std::ceil(p.r_c / edge - 1e-12)));
      for (int b = 0; b < 3; ++b) {
        rg.A_hi[3 * a + b] = float(H[a][b]);
        rg.A_lo[3 * a + b] = float(H[a][b] - double(rg.A_hi[3 * a + b]));
        rg.Binv[3 * a + b] = float(general ? Hinv[b][a] : (a == b ? 1.0 / p.box[a] : 0.0));
      }
      rg.ncell *= rg.nc[a];
    }
    rg.rc = float(p.r_c);
    rg.rc2 = float(p.r_c * p.r_c);
    rg.inv_rc = float(1.0 / p.r_c);
    rg.srec = 4 + (C + 3) / 4 * 4;
  }

  // ---- workspace layout for max_atoms ----
  const int64_t Nm = std::max<int64_t>(max_atoms, 1);
  const size_t grid_b = size_t(C) * M[0] * M[1] * M[2] * 4;
  const size_t s1_b = size_t(C) * M[0] * M[1] * g.KZP * 8;
  const size_t s2_b = size_t(C) * M[0] * g.NY * g.KZP * 8;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t off = o;
    o = align256(o + bytes);
    return off;
  };
  pl.off_grid = take(grid_b);
  pl.off_s1 = take(s1_b);
  pl.off_s2 = s2_b <= grid_b ? pl.off_grid : take(s2_b);  // grid is dead while S2 lives
  pl.off_rec_a = take(size_t(Nm) * 16);
  pl.off_q_a = take(size_t(Nm) * C * 4);
  pl.off_q_b = take(size_t(Nm) * g.srec * 4);
  pl.off_perm_a = take(size_t(Nm) * 4);
  pl.off_perm_b = take(size_t(Nm) * 4);
  pl.off_cell_of = take(size_t(Nm) * 4);
  pl.off_slot = take(size_t(Nm) * 4);
  pl.off_count = take(size_t(g.ncell) * 4);
  pl.off_start = take(size_t(g.ncell + 1) * 4);
  pl.off_epart = take(size_t(C) * std::max(1, g.nxblk) * 8 * 8);
  pl.off_qpart = take(size_t((Nm + kQChunk - 1) / kQChunk + 1) * C * 2 * 8);
  pl.off_qsum = take(size_t(C) * 2 * 8);
  pl.off_status = take(2 * sizeof(int));
  pl.off_rs_rec_b = take(size_t(Nm) * pl.rsg.srec * 4);
  pl.off_rs_rec_a = take(size_t(Nm) * pl.rsg.srec * 4);
  pl.off_rs_perm_b = take(size_t(Nm) * 4);
  pl.off_rs_perm_a = take(size_t(Nm) * 4);
  pl.off_rs_cell_of = take(size_t(Nm) * 4);
  pl.off_rs_slot = take(size_t(Nm) * 4);
  pl.off_rs_count = take(size_t(pl.rsg.ncell) * 4);
  pl.off_rs_start = take(size_t(pl.rsg.ncell + 1) * 4);
  pl.off_rs_part = take(size_t(pl.rsg.ncell) * (C + 6) * 8);
  pl.off_dd = take(size_t(Nm) * (4 * size_t(C) + 3) * 4);
  pl.ws_bytes = o;
  pl.max_atoms = max_atoms;

  // ---- info ----
  pswflr_info &inf = pl.info;
  inf = pswflr_info{};
  inf.c = c; inf.r_c = p.r_c; inf.k_c = kc; inf.c_spread = cs; inf.eta = eta;
  for (int a = 0; a < 3; ++a) { inf.h[a] = h[a]; inf.grid[a] = M[a]; inf.tile[a] = g.B[a]; }
  inf.volume = g.V;
  for (int i = 0; i < 9; ++i) {
    inf.cell[i] = H[i / 3][i % 3];
    pl.hinv[i] = general ? Hinv[i / 3][i % 3] : (i % 4 == 0 ? 1.0 / p.box[i / 3] : 0.0);
  }
  inf.support = P;
  inf.n_channels = C;
  inf.kz_keep = g.KZ;
  inf.ny_keep = g.NY;
  inf.cg_spread = g.CG_spread;
  inf.cg_gather = g.CG_gather;
  inf.xcols = 0;
  for (size_t i = 2; i < xblk.size(); i += 4) inf.xcols += xblk[i];
  inf.max_atoms = max_atoms;
  inf.workspace_bytes = pl.ws_bytes;
  inf.grid_offset = pl.off_grid;
  for (int ch = 0; ch < C; ++ch) {
    inf.self_coef[ch] = selfc[ch];
    inf.zero_coef[ch] = zerov[ch] / g.V;
  }
  pl.prm = p;
  pl.prm.c = c;
  pl.prm.support = P;
  pl.prm.c_spread = cs;
  for (int a = 0; a < 3; ++a) pl.prm.grid[a] = M[a];
  return PSWFLR_OK;
}

Work carve(const pswflr_plan_s &pl, void *ws, int64_t N) {
  char *b = static_cast<char *>(ws);
  Work w{};
  w.grid = reinterpret_cast<float *>(b + pl.off_grid);
  w.s1 = reinterpret_cast<float *>(b + pl.off_s1);
  w.s2 = reinterpret_cast<float *>(b + pl.off_s2);
  w.rec_a = reinterpret_cast<float *>(b + pl.off_rec_a);
  w.q_a = reinterpret_cast<float *>(b + pl.off_q_a);
  w.q_b = reinterpret_cast<float *>(b + pl.off_q_b);
  w.perm_a = reinterpret_cast<int *>(b + pl.off_perm_a);
  w.perm_b = reinterpret_cast<int *>(b + pl.off_perm_b);
  w.cell_of = reinterpret_cast<int *>(b + pl.off_cell_of);
  w.slot = reinterpret_cast<int *>(b + pl.off_slot);
  w.cell_count = reinterpret_cast<int *>(b + pl.off_count);
  w.cell_start = reinterpret_cast<int *>(b + pl.off_start);
  w.epart = reinterpret_cast<double *>(b + pl.off_epart);
  w.qpart = reinterpret_cast<double *>(b + pl.off_qpart);
  w.qsum = reinterpret_cast<double *>(b + pl.off_qsum);
  w.status = reinterpret_cast<int *>(b + pl.off_status);
  (void)N;
  return w;
}

pswflr_status check_call(pswflr_plan pl, void *ws, size_t ws_bytes, int64_t n, const float *pos,
                         const float *q) {
  if (!pl) return fail(PSWFLR_ERR_INVALID_ARG, "plan is NULL");
  if (n < 0 || n > pl->max_atoms) return fail(PSWFLR_ERR_INVALID_ARG, "n_atoms must be in [0, max_atoms]");
  if (!ws || ws_bytes < pl->ws_bytes) return fail(PSWFLR_ERR_WORKSPACE, "workspace missing or too small");
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(PSWFLR_ERR_WORKSPACE, "workspace not 256-byte aligned");
  if (n > 0 && (!pos || !q)) return fail(PSWFLR_ERR_INVALID_ARG, "pos and q must be non-NULL");
  return PSWFLR_OK;
}

// Optional input validation (PSWFLR_FLAG_CHECK_INPUTS): a check kernel,
// then the result word is read back, which waits for the stream.
pswflr_status check_inputs(const pswflr_plan_s &pl, hipStream_t st, const Geo &g, const Work &w, const float *pos,
                           const float *q) {
  if (!(pl.prm.flags & PSWFLR_FLAG_CHECK_INPUTS)) return PSWFLR_OK;
  hipError_t e = launch_check_inputs(g, w, pos, q, st);
  int word = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&word, w.status + 1, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(PSWFLR_ERR_DEVICE, std::string("input check failed: ") + hipGetErrorString(e));
  if (word & 1) return fail(PSWFLR_ERR_INVALID_ARG, "a position is not finite");
  if (word & 2) return fail(PSWFLR_ERR_INVALID_ARG, "a charge is not finite");
  return PSWFLR_OK;
}

#define HIPCHK(expr)                                                                      \
  do {                                                                                    \
    hipError_t e__ = (expr);                                                              \
    if (e__ != hipSuccess) return fail(PSWFLR_ERR_DEVICE, std::string(#expr) + ": " +     \
                                                              hipGetErrorString(e__));    \
  } while (0)

}  // namespace

extern "C" {

pswflr_status pswflr_plan_create(const pswflr_params *params, int64_t max_atoms, pswflr_plan *out) {
  if (!params || !out) return fail(PSWFLR_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  pswflr_plan_s *pl = nullptr;
  try {
    pl = new pswflr_plan_s();
    pswflr_status s = build_plan(*params, max_atoms, *pl);
    if (s != PSWFLR_OK) {
      table_release(pl->dtab, pl->dtab_bytes, pl->device, pl->last_use);
      delete pl;
      return s;
    }
  } catch (const std::exception &e) {
    if (pl) table_release(pl->dtab, pl->dtab_bytes, pl->device, pl->last_use);
    delete pl;
    return fail(PSWFLR_ERR_INTERNAL, e.what());
  }
  *out = pl;
  return PSWFLR_OK;
}

pswflr_status pswflr_plan_info(pswflr_plan plan, pswflr_info *out) {
  if (!plan || !out) return fail(PSWFLR_ERR_INVALID_ARG, "NULL argument");
  *out = plan->info;
  return PSWFLR_OK;
}

pswflr_status pswflr_plan_destroy(pswflr_plan plan) {
  if (!plan) return PSWFLR_OK;
  table_release(plan->dtab, plan->dtab_bytes, plan->device, plan->last_use);
  delete plan;
  return PSWFLR_OK;
}

}  // extern "C"

namespace {

// Runs one stage (one kernel launch, or the small sort/charge-sum groups)
// and, while its stage is timed, brackets it with events on the same stream.
struct StageRunner {
  pswflr_plan_s *pl;
  hipStream_t st;
  bool timing = true;  // false: never create timing events (allocation-free calls)
  template <class F>
  hipError_t operator()(int stage, F &&f) {
    if (!timing || stage < 0 || stage >= 32 || !((pl->prof_mask >> stage) & 1u)) return f();
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return hipErrorOutOfMemory;
    (void)hipEventRecord(a, st);
    hipError_t e = f();
    (void)hipEventRecord(b, st);
    std::lock_guard<std::mutex> lock(pl->prof_mu);
    pl->prof_ev.emplace_back(stage, a, b);
    return e;
  }
};

hipError_t run_forward(pswflr_plan_s *pl, hipStream_t st, const Geo &g, const Work &w, const float *pos,
                       const float *q, int xmode, double *energy, double *virial, bool timing = true) {
  StageRunner run{pl, st, timing};
  const Tables &t = pl->tab;
  hipError_t e;
  if (prep_small(g)) {
    if ((e = run(PSWFLR_STAGE_SORT, [&] { return enqueue_prep_small(g, w, pos, q, st); })) != hipSuccess) return e;
  } else {
    // the charge sums ride in the sort's launches (timed as the sort)
    if ((e = run(PSWFLR_STAGE_SORT, [&] { return enqueue_sort(g, w, pos, q, st); })) != hipSuccess) return e;
  }
  for (int cg0 = 0; cg0 < g.C; cg0 += g.CG_spread) {
    const int ncg = std::min(g.CG_spread, g.C - cg0);
    if ((e = run(PSWFLR_STAGE_SPREAD, [&] { return launch_spread(g, t, w, cg0, ncg, st); })) != hipSuccess)
      return e;
  }
  if ((e = run(PSWFLR_STAGE_FFT_Z, [&] { return launch_zfwd(g, t, pl->az, w, st); })) != hipSuccess) return e;
  if ((e = run(PSWFLR_STAGE_FFT_Y, [&] { return launch_yfwd(g, t, pl->ay, w, st); })) != hipSuccess) return e;
  if ((e = run(PSWFLR_STAGE_FFT_X_SCALE, [&] { return launch_xmul(g, t, pl->ax, w, xmode, nullptr, st); })) !=
      hipSuccess)
    return e;
  return run(PSWFLR_STAGE_REDUCE, [&] { return launch_finalize(g, t, w, energy, virial, st); });
}

hipError_t run_adjoint(pswflr_plan_s *pl, hipStream_t st, const Geo &g, const Work &w, float *forces,
                       float *pot, int mode, const double *grad, bool timing = true) {
  StageRunner run{pl, st, timing};
  const Tables &t = pl->tab;
  hipError_t e;
  if (mode == 2) {
    if ((e = run(PSWFLR_STAGE_FFT_X_SCALE, [&] { return launch_xmul(g, t, pl->ax, w, 2, grad, st); })) !=
        hipSuccess)
      return e;
  }
  if ((e = run(PSWFLR_STAGE_IFFT_Y, [&] { return launch_yinv(g, t, pl->ay, w, st); })) != hipSuccess) return e;
  if ((e = run(PSWFLR_STAGE_IFFT_Z, [&] { return launch_zinv(g, t, pl->az, w, st); })) != hipSuccess) return e;
  return run(PSWFLR_STAGE_GATHER, [&] { return launch_gather(g, t, w, forces, pot, mode, grad, st); });
}

}  // namespace

namespace {
// record the end of a call on `st` for the plans it used
hipError_t mark_use(hipStream_t st, const pswflr_plan *plans, int n) {
  hipEvent_t ev = nullptr;
  hipError_t e = stream_event(st, &ev);
  if (e == hipSuccess) e = hipEventRecord(ev, st);
  if (e != hipSuccess) return e;
  for (int i = 0; i < n; ++i) plans[i]->last_use = ev;
  return hipSuccess;
}
}  // namespace

extern "C" {

pswflr_status pswflr_execute(pswflr_plan plan, pswflr_stream stream, void *workspace, size_t ws_bytes,
                             int64_t n_atoms, const float *pos, const float *q, double *energy, float *forces,
                             double *virial, float *potential) {
  pswflr_status s = check_call(plan, workspace, ws_bytes, n_atoms, pos, q);
  if (s != PSWFLR_OK) return s;
  if (!energy) return fail(PSWFLR_ERR_INVALID_ARG, "energy output is required");
  hipStream_t st = static_cast<hipStream_t>(stream);
  Geo g = plan->geo;
  g.N = n_atoms;
  Work w = carve(*plan, workspace, n_atoms);
  if ((s = check_inputs(*plan, st, g, w, pos, q)) != PSWFLR_OK) return s;
  const bool adjoint = forces || potential;
  hipError_t e = run_forward(plan, st, g, w, pos, q, adjoint ? 1 : 0, energy, virial);
  if (e == hipSuccess && adjoint) e = run_adjoint(plan, st, g, w, forces, potential, 1, nullptr);
  if (e == hipSuccess) e = mark_use(st, &plan, 1);
  if (e != hipSuccess) return fail(PSWFLR_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return PSWFLR_OK;
}

pswflr_status pswflr_execute_noalloc(pswflr_plan plan, pswflr_stream stream, int64_t n_atoms, const float *pos,
                                     const float *q, double *energy, float *forces, double *virial,
                                     float *potential) {
  if (!plan) return fail(PSWFLR_ERR_INVALID_ARG, "plan is NULL");
  if (plan->ws_bytes > kNoallocScratchBytes)
    return fail(PSWFLR_ERR_WORKSPACE, "the plan's workspace (" + std::to_string(plan->ws_bytes) +
                                          " B for its max_atoms) exceeds the no-allocation scratch of " +
                                          std::to_string(kNoallocScratchBytes) + " B");
  if (plan->prm.flags & PSWFLR_FLAG_CHECK_INPUTS)
    return fail(PSWFLR_ERR_INVALID_ARG, "the input check waits on the host; use pswflr_execute");
  void *scratch = nullptr;
  hipError_t e = noalloc_scratch(&scratch);
  if (e != hipSuccess) return fail(PSWFLR_ERR_DEVICE, std::string("scratch lookup failed: ") + hipGetErrorString(e));
  pswflr_status s = check_call(plan, scratch, kNoallocScratchBytes, n_atoms, pos, q);
  if (s != PSWFLR_OK) return s;
  if (!energy) return fail(PSWFLR_ERR_INVALID_ARG, "energy output is required");
  hipStream_t st = static_cast<hipStream_t>(stream);
  Geo g = plan->geo;
  g.N = n_atoms;
  Work w = carve(*plan, scratch, n_atoms);
  const bool adjoint = forces || potential;
  e = run_forward(plan, st, g, w, pos, q, adjoint ? 1 : 0, energy, virial, false);
  if (e == hipSuccess && adjoint) e = run_adjoint(plan, st, g, w, forces, potential, 1, nullptr, false);
  if (e != hipSuccess) return fail(PSWFLR_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return PSWFLR_OK;
}

pswflr_status pswflr_realspace(pswflr_plan plan, pswflr_stream stream, void *workspace, size_t ws_bytes,
                               int64_t n_atoms, const float *pos, const float *q, double *energy, float *forces,
                               double *virial, float *potential) {
  pswflr_status s = check_call(plan, workspace, ws_bytes, n_atoms, pos, q);
  if (s != PSWFLR_OK) return s;
  if (!energy) return fail(PSWFLR_ERR_INVALID_ARG, "energy output is required");
  hipStream_t st = static_cast<hipStream_t>(stream);
  {
    Geo g = plan->geo;
    g.N = n_atoms;
    Work w = carve(*plan, workspace, n_atoms);
    if ((s = check_inputs(*plan, st, g, w, pos, q)) != PSWFLR_OK) return s;
  }
  RsGeo rg = plan->rsg;
  rg.N = n_atoms;
  char *b = static_cast<char *>(workspace);
  RsWork rw{};
  rw.rec_b = reinterpret_cast<float *>(b + plan->off_rs_rec_b);
  rw.rec_a = reinterpret_cast<float *>(b + plan->off_rs_rec_a);
  rw.perm_b = reinterpret_cast<int *>(b + plan->off_rs_perm_b);
  rw.perm_a = reinterpret_cast<int *>(b + plan->off_rs_perm_a);
  rw.cell_of = reinterpret_cast<int *>(b + plan->off_rs_cell_of);
  rw.slot = reinterpret_cast<int *>(b + plan->off_rs_slot);
  rw.count = reinterpret_cast<int *>(b + plan->off_rs_count);
  rw.start = reinterpret_cast<int *>(b + plan->off_rs_start);
  rw.part = reinterpret_cast<double *>(b + plan->off_rs_part);
  hipError_t e = launch_realspace(rg, plan->rst, rw, plan->rs_grp, plan->rs_gch, plan->rs_ngrp, plan->rs_cgmax, pos,
                                  q, energy, forces, virial, potential, st);
  if (e == hipSuccess) e = mark_use(st, &plan, 1);
  if (e != hipSuccess) return fail(PSWFLR_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return PSWFLR_OK;
}

pswflr_status pswflr_cell_gradient(pswflr_plan plan, pswflr_stream stream, const double *virial,
                                   double *grad_cell) {
  if (!plan || !virial || !grad_cell) return fail(PSWFLR_ERR_INVALID_ARG, "plan, virial and grad_cell are required");
  CellInv hi{};
  for (int i = 0; i < 9; ++i) hi.m[i] = plan->hinv[i];
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = launch_cell_gradient(hi, virial, grad_cell, st);
  if (e == hipSuccess) e = mark_use(st, &plan, 1);
  if (e != hipSuccess) return fail(PSWFLR_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return PSWFLR_OK;
}

pswflr_status pswflr_force_vjp(pswflr_plan plan, pswflr_stream stream, void *workspace, size_t ws_bytes,
                                int64_t n_atoms, const float *pos, const float *q, const float *v, float *grad_q,
                                float *grad_pos) {
  pswflr_status s = check_call(plan, workspace, ws_bytes, n_atoms, pos, q);
  if (s != PSWFLR_OK) return s;
  if (n_atoms > 0 && (!v || !grad_q || !grad_pos))
    return fail(PSWFLR_ERR_INVALID_ARG, "v, grad_q and grad_pos are required");
  hipStream_t st = static_cast<hipStream_t>(stream);
  Geo g = plan->geo;
  g.N = n_atoms;
  Work w = carve(*plan, workspace, n_atoms);
  char *b = static_cast<char *>(workspace) + plan->off_dd;
  const size_t cn = size_t(g.C) * size_t(n_atoms);
  float *qd = reinterpret_cast<float *>(b);
  float *s2 = qd + 3 * cn;
  float *f2 = s2 + cn;
  hipError_t e = launch_double_backward(g, plan->tab, plan->az, plan->ay, plan->ax, w, v, qd, s2, f2, grad_q,
                                        grad_pos, st);
  if (e == hipSuccess) e = mark_use(st, &plan, 1);
  if (e != hipSuccess) return fail(PSWFLR_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return PSWFLR_OK;
}

pswflr_status pswflr_backward(pswflr_plan plan, pswflr_stream stream, void *workspace, size_t ws_bytes,
                              int64_t n_atoms, const float *pos, const float *q, const double *grad_energy,
                              float *grad_q, float *grad_pos) {
  pswflr_status s = check_call(plan, workspace, ws_bytes, n_atoms, pos, q);
  if (s != PSWFLR_OK) return s;
  if (!grad_energy) return fail(PSWFLR_ERR_INVALID_ARG, "grad_energy is required");
  if (!grad_q && !grad_pos) return PSWFLR_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  Geo g = plan->geo;
  g.N = n_atoms;
  Work w = carve(*plan, workspace, n_atoms);
  hipError_t e = run_adjoint(plan, st, g, w, grad_pos, grad_q, 2, grad_energy);
  if (e == hipSuccess) e = mark_use(st, &plan, 1);
  if (e != hipSuccess) return fail(PSWFLR_ERR_DEVICE, std::string("launch failed: ") + hipGetErrorString(e));
  return PSWFLR_OK;
}

pswflr_status pswflr_profile_enable(pswflr_plan plan, int enable) {
  return pswflr_profile_stages(plan, enable != 0 ? (1u << PSWFLR_NUM_STAGES) - 1u : 0u);
}

pswflr_status pswflr_profile_stages(pswflr_plan plan, uint32_t stage_mask) {
  if (!plan) return fail(PSWFLR_ERR_INVALID_ARG, "plan is NULL");
  if (stage_mask >> PSWFLR_NUM_STAGES) return fail(PSWFLR_ERR_INVALID_ARG, "stage mask names no stage");
  plan->prof_mask = stage_mask;
  return PSWFLR_OK;
}

pswflr_status pswflr_profile_read(pswflr_plan plan, double *ms_total, int64_t *launches) {
  if (!plan || !ms_total || !launches) return fail(PSWFLR_ERR_INVALID_ARG, "NULL argument");
  for (int i = 0; i < PSWFLR_NUM_STAGES; ++i) {
    ms_total[i] = 0.0;
    launches[i] = 0;
  }
  std::lock_guard<std::mutex> lock(plan->prof_mu);
  pswflr_status s = PSWFLR_OK;
  for (auto &ev : plan->prof_ev) {
    hipEvent_t a = std::get<1>(ev), b = std::get<2>(ev);
    float ms = 0.f;
    if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess)
      s = fail(PSWFLR_ERR_DEVICE, "event timing failed");
    ms_total[std::get<0>(ev)] += ms;
    launches[std::get<0>(ev)] += 1;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
  plan->prof_ev.clear();
  return s;
}

}  // extern "C"

namespace {

size_t batch_header_bytes(int n) {
  return align256(size_t(n) * sizeof(BatchItem)) + align256(size_t(kNumBatchStages) * (n + 1) * sizeof(int));
}

int stage_profile_id(int bs) {
  switch (bs) {
    case kBsZero: case kBsBin: case kBsScan: case kBsScatter: case kBsOrder: return PSWFLR_STAGE_SORT;
    case kBsQsum: case kBsQreduce: return PSWFLR_STAGE_QSUM;
    case kBsSpread: return PSWFLR_STAGE_SPREAD;
    case kBsZfwd: return PSWFLR_STAGE_FFT_Z;
    case kBsYfwd: return PSWFLR_STAGE_FFT_Y;
    case kBsXmul: return PSWFLR_STAGE_FFT_X_SCALE;
    case kBsFinalize: return PSWFLR_STAGE_REDUCE;
    case kBsYinv: return PSWFLR_STAGE_IFFT_Y;
    case kBsZinv: return PSWFLR_STAGE_IFFT_Z;
    default: return PSWFLR_STAGE_GATHER;
  }
}

// Pinned staging for batch headers, one per host thread and reused across
// calls: the upload is then a plain DMA with no host callback on the stream.
// An event recorded after each upload keeps the next call from overwriting
// the buffer before the copy has run.  Kept for the life of the process.
struct HeaderStage {
  char *buf = nullptr;
  size_t cap = 0;
  hipEvent_t ev = nullptr;
  int device = -1;
};
thread_local HeaderStage g_header;

hipError_t header_buffer(size_t bytes, char **out) {
  HeaderStage &h = g_header;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (h.ev) {
    e = hipEventSynchronize(h.ev);  // the previous upload from this buffer has run
    if (e != hipSuccess) return e;
  }
  if (h.device != dev) {
    h.ev = nullptr;  // an event of another device is left as is
    e = hipEventCreateWithFlags(&h.ev, hipEventDisableTiming);
    if (e != hipSuccess) return e;
    h.device = dev;
  }
  if (h.cap < bytes) {
    // hipHostFree synchronizes with the device, so growth is kept rare: at
    // least 1 MiB (a few hundred structures) and at least double the last
    // size, instead of a new buffer each time a batch has more structures
    // than any before.
    const size_t want = std::max(bytes, std::max(2 * h.cap, size_t(1) << 20));
    if (h.buf) (void)hipHostFree(h.buf);
    h.buf = nullptr;
    h.cap = 0;
    e = hipHostMalloc(reinterpret_cast<void **>(&h.buf), want, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    h.cap = want;
  }
  *out = h.buf;
  return hipSuccess;
}

}  // namespace

extern "C" {

pswflr_status pswflr_batch_workspace(int32_t n, const pswflr_plan *plans, const int64_t *n_atoms, size_t *bytes) {
  if (n < 0 || (n > 0 && (!plans || !n_atoms)) || !bytes) return fail(PSWFLR_ERR_INVALID_ARG, "bad batch arguments");
  size_t tot = batch_header_bytes(n);
  for (int i = 0; i < n; ++i) {
    if (!plans[i]) return fail(PSWFLR_ERR_INVALID_ARG, "NULL plan in batch");
    if (n_atoms[i] < 0 || n_atoms[i] > plans[i]->max_atoms)
      return fail(PSWFLR_ERR_INVALID_ARG, "batch entry exceeds its plan's max_atoms");
    tot += align256(plans[i]->ws_bytes);
  }
  *bytes = tot;
  return PSWFLR_OK;
}

}  // extern "C"

namespace {

// One structure of a batched call, forward or adjoint.
struct BatchEntry {
  int64_t n_atoms;
  const float *pos, *q;
  double *energy;
  float *forces;      // forward: forces; adjoint: dL/dr
  double *virial;
  float *potential;   // forward: potentials; adjoint: dL/dq
  const double *grad; // adjoint: dL/dE per channel
};

// Batched forward (every stage, one launch per stage over all structures)
// or adjoint (scaled inverse transforms and the gather of an energy-only
// batched forward on the same workspace).
pswflr_status batch_impl(int32_t n, const pswflr_plan *plans, const BatchEntry *io, pswflr_stream stream,
                         void *workspace, size_t ws_bytes, bool adjoint_call) {
  if (n == 0) return PSWFLR_OK;
  if (n < 0 || !plans || !io) return fail(PSWFLR_ERR_INVALID_ARG, "bad batch arguments");
  std::vector<int64_t> na(n);
  for (int i = 0; i < n; ++i) na[i] = io[i].n_atoms;
  size_t need = 0;
  pswflr_status s = pswflr_batch_workspace(n, plans, na.data(), &need);
  if (s != PSWFLR_OK) return s;
  if (!workspace || ws_bytes < need) return fail(PSWFLR_ERR_WORKSPACE, "batch workspace missing or too small");
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
    return fail(PSWFLR_ERR_WORKSPACE, "workspace not 256-byte aligned");
  for (int i = 0; i < n; ++i) {
    if (!adjoint_call && !io[i].energy) return fail(PSWFLR_ERR_INVALID_ARG, "energy output is required");
    if (adjoint_call && !io[i].grad) return fail(PSWFLR_ERR_INVALID_ARG, "grad_energy is required");
    if (io[i].n_atoms > 0 && (!io[i].pos || !io[i].q)) return fail(PSWFLR_ERR_INVALID_ARG, "pos and q required");
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  char *ws = static_cast<char *>(workspace);
  const size_t hdr = batch_header_bytes(n);
  if (!adjoint_call) {
    size_t off = hdr;
    for (int i = 0; i < n; ++i) {
      Geo gi = plans[i]->geo;
      gi.N = io[i].n_atoms;
      if ((s = check_inputs(*plans[i], st, gi, carve(*plans[i], ws + off, io[i].n_atoms), io[i].pos, io[i].q)) !=
          PSWFLR_OK)
        return s;
      off += align256(plans[i]->ws_bytes);
    }
  }
  bool fused = true;
  for (int i = 0; i < n; ++i) fused = fused && plans[i]->geo.C <= spread_max_channels();
  if (!fused) {  // channel groups beyond one spreading launch: one call per structure
    size_t off = hdr;
    for (int i = 0; i < n; ++i) {
      s = adjoint_call ? pswflr_backward(plans[i], stream, ws + off, plans[i]->ws_bytes, io[i].n_atoms, io[i].pos,
                                         io[i].q, io[i].grad, io[i].potential, io[i].forces)
                       : pswflr_execute(plans[i], stream, ws + off, plans[i]->ws_bytes, io[i].n_atoms, io[i].pos,
                                        io[i].q, io[i].energy, io[i].forces, io[i].virial, io[i].potential);
      if (s != PSWFLR_OK) return s;
      off += align256(plans[i]->ws_bytes);
    }
    return PSWFLR_OK;
  }
  // host image of the header: items, then per-stage prefixes
  char *blob = nullptr;
  if (header_buffer(hdr, &blob) != hipSuccess) return fail(PSWFLR_ERR_DEVICE, "batch header staging failed");
  std::memset(blob, 0, hdr);
  BatchItem *items = reinterpret_cast<BatchItem *>(blob);
  int *prefix = reinterpret_cast<int *>(blob + align256(size_t(n) * sizeof(BatchItem)));
  std::vector<bool> adj(n);
  size_t off = hdr;
  // the vector-ALU spread's flush size follows the tiles of the whole batch
  int64_t batch_tiles = 0;
  for (int i = 0; i < n; ++i) batch_tiles += plans[i]->geo.ncell;
  const int scap = spread_flush_cap(batch_tiles);
  for (int i = 0; i < n; ++i) {
    const pswflr_plan_s &pl = *plans[i];
    BatchItem &it = items[i];
    it.g = pl.geo;
    it.g.N = io[i].n_atoms;
    it.g.scap = scap;
    it.t = pl.tab;
    it.w = carve(pl, ws + off, io[i].n_atoms);
    it.az = pl.az;
    it.ay = pl.ay;
    it.ax = pl.ax;
    it.pos = io[i].pos;
    it.q = io[i].q;
    it.energy = io[i].energy;
    it.forces = io[i].forces;
    it.virial = io[i].virial;
    it.pot = io[i].potential;
    it.qblocks = qsum_blocks(it.g);
    it.nlines = int64_t(it.g.C) * it.g.M[0] * it.g.M[1];
    it.grad = adjoint_call ? io[i].grad : nullptr;
    adj[i] = adjoint_call || io[i].forces || io[i].potential;
    // energy-only structures keep their spectrum for a later adjoint call
    it.mode = adjoint_call ? 2 : (adj[i] ? 1 : 0);
    off += align256(pl.ws_bytes);
  }
  std::vector<int> total(kNumBatchStages);
  std::vector<size_t> lds(kNumBatchStages, 0);
  for (int stg = 0; stg < kNumBatchStages; ++stg) {
    int acc = 0;
    for (int i = 0; i < n; ++i) {
      prefix[stg * (n + 1) + i] = acc;
      acc += batch_stage_blocks(items[i], stg, adj[i]);
      lds[stg] = std::max(lds[stg], batch_stage_lds(items[i], stg));
    }
    prefix[stg * (n + 1) + n] = acc;
    total[stg] = acc;
  }
  // kernel variants of the spreading stage present in the batch, each with
  // the largest LDS footprint among its own structures
  std::vector<int> spread_variants;
  std::vector<size_t> spread_lds;
  for (int i = 0; i < n; ++i) {
    const int v = batch_spread_variant(items[i].g);
    const size_t l = batch_stage_lds(items[i], kBsSpread);
    const auto it = std::find(spread_variants.begin(), spread_variants.end(), v);
    if (it == spread_variants.end()) {
      spread_variants.push_back(v);
      spread_lds.push_back(l);
    } else {
      size_t &m = spread_lds[size_t(it - spread_variants.begin())];
      m = std::max(m, l);
    }
  }
  hipError_t e = hipMemcpyAsync(ws, blob, hdr, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipEventRecord(g_header.ev, st);
  if (e != hipSuccess)
    return fail(PSWFLR_ERR_DEVICE, std::string("batch header upload failed: ") + hipGetErrorString(e));
  const BatchItem *d_items = reinterpret_cast<const BatchItem *>(ws);
  const int *d_prefix = reinterpret_cast<const int *>(ws + align256(size_t(n) * sizeof(BatchItem)));
  StageRunner run{plans[0], st};
  for (int stg = 0; stg < kNumBatchStages; ++stg) {
    // the adjoint runs the scaled x pass and what follows it, minus the
    // energy reduction
    if (adjoint_call && (stg < kBsXmul || stg == kBsFinalize)) continue;
    // the charge sums ride in the binning launch, their reduction in the
    // scatter launch
    if (stg == kBsQsum || stg == kBsQreduce) continue;
    e = run(stage_profile_id(stg), [&] {
      if (stg == kBsBin || stg == kBsScatter) {
        const int pb = stg == kBsBin ? kBsQsum : kBsQreduce;
        return launch_batch_pair(d_items, d_prefix + stg * (n + 1), total[stg], d_prefix + pb * (n + 1), total[pb], n,
                                 stg, st);
      }
      if (stg != kBsSpread)
        return launch_batch_stage(d_items, d_prefix + stg * (n + 1), n, stg, total[stg], lds[stg], 1, st);
      hipError_t r = hipSuccess;
      for (size_t k = 0; k < spread_variants.size(); ++k)
        if (r == hipSuccess)
          r = launch_batch_spread(d_items, d_prefix + stg * (n + 1), n, total[stg], spread_lds[k], spread_variants[k], st);
      return r;
    });
    if (e != hipSuccess) return fail(PSWFLR_ERR_DEVICE, std::string("batch launch failed: ") + hipGetErrorString(e));
  }
  if ((e = mark_use(st, plans, n)) != hipSuccess)
    return fail(PSWFLR_ERR_DEVICE, std::string("event record failed: ") + hipGetErrorString(e));
  return PSWFLR_OK;
}

// Per-structure pointers into flat arrays: atoms, charges and outputs of
// consecutive structures follow each other.
std::vector<BatchEntry> flat_entries(int32_t n, const pswflr_plan *plans, const int64_t *n_atoms, const float *pos,
                                     const float *q, double *energy, float *forces, double *virial,
                                     float *potential, const double *grad, bool adjoint_call) {
  std::vector<BatchEntry> io(std::max(0, n));
  int64_t a0 = 0, q0 = 0, e0 = 0, c0 = 0;
  for (int i = 0; i < n; ++i) {
    const int64_t N = n_atoms[i], C = plans[i]->geo.C;
    BatchEntry &b = io[i];
    b.n_atoms = N;
    b.pos = pos ? pos + 3 * a0 : nullptr;
    b.q = q ? q + q0 : nullptr;
    b.energy = energy ? energy + e0 : nullptr;
    b.forces = forces ? forces + 3 * a0 : nullptr;
    b.virial = virial ? virial + 6 * i : nullptr;
    b.potential = potential ? potential + q0 : nullptr;
    b.grad = grad ? grad + c0 : nullptr;
    a0 += N;
    q0 += C * N;
    e0 += 3 * C + 1;
    c0 += C;
  }
  (void)adjoint_call;
  return io;
}

}  // namespace

extern "C" {

pswflr_status pswflr_execute_batch(int32_t n, const pswflr_plan *plans, const pswflr_io *io,
                                   pswflr_stream stream, void *workspace, size_t ws_bytes) {
  if (n > 0 && (!plans || !io)) return fail(PSWFLR_ERR_INVALID_ARG, "bad batch arguments");
  std::vector<BatchEntry> e(std::max(0, n));
  for (int i = 0; i < n; ++i)
    e[i] = BatchEntry{io[i].n_atoms, io[i].pos, io[i].q, io[i].energy, io[i].forces, io[i].virial, io[i].potential,
                      nullptr};
  return batch_impl(n, plans, e.data(), stream, workspace, ws_bytes, false);
}

pswflr_status pswflr_execute_batch_flat(int32_t n, const pswflr_plan *plans, const int64_t *n_atoms,
                                        const float *pos, const float *q, double *energy, float *forces,
                                        double *virial, float *potential, pswflr_stream stream, void *workspace,
                                        size_t ws_bytes) {
  if (n == 0) return PSWFLR_OK;
  if (n < 0 || !plans || !n_atoms) return fail(PSWFLR_ERR_INVALID_ARG, "bad batch arguments");
  for (int i = 0; i < n; ++i)
    if (!plans[i]) return fail(PSWFLR_ERR_INVALID_ARG, "NULL plan in batch");
  auto e = flat_entries(n, plans, n_atoms, pos, q, energy, forces, virial, potential, nullptr, false);
  return batch_impl(n, plans, e.data(), stream, workspace, ws_bytes, false);
}

pswflr_status pswflr_backward_batch_flat(int32_t n, const pswflr_plan *plans, const int64_t *n_atoms,
                                         const float *pos, const float *q, const double *grad_energy,
                                         float *grad_q, float *grad_pos, pswflr_stream stream, void *workspace,
                                         size_t ws_bytes) {
  if (n == 0) return PSWFLR_OK;
  if (n < 0 || !plans || !n_atoms || !grad_energy) return fail(PSWFLR_ERR_INVALID_ARG, "bad batch arguments");
  if (!grad_q && !grad_pos) return PSWFLR_OK;
  for (int i = 0; i < n; ++i)
    if (!plans[i]) return fail(PSWFLR_ERR_INVALID_ARG, "NULL plan in batch");
  auto e = flat_entries(n, plans, n_atoms, pos, q, nullptr, grad_pos, nullptr, grad_q, grad_energy, true);
  return batch_impl(n, plans, e.data(), stream, workspace, ws_bytes, true);
}

const char *pswflr_status_string(pswflr_status status) {
  switch (status) {
    case PSWFLR_OK: return "ok";
    case PSWFLR_ERR_INVALID_ARG: return "invalid argument";
    case PSWFLR_ERR_UNSUPPORTED: return "unsupported";
    case PSWFLR_ERR_WORKSPACE: return "workspace missing or too small";
    case PSWFLR_ERR_DEVICE: return "device error";
    case PSWFLR_ERR_OOM: return "out of memory";
    case PSWFLR_ERR_INTERNAL: return "internal error";
  }
  return "unknown status";
}

void pswflr_last_error(char *buf, size_t len) {
  if (!buf || len == 0) return;
  std::snprintf(buf, len, "%s", g_last_error.c_str());
}

}  // extern "C"
