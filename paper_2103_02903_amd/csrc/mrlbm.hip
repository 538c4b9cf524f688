// C-ABI of the MR-LBM hot path (declared in include/mrlbm.h): context set-up in a
// caller-owned workspace for a batch of instances, the flattened transport
// weights, and the per-step launch sequence of Algorithm 1 of arXiv 2103.02903.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <utility>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "mr_adjoint.h"
#include "mr_kernels.h"
#include "mr_kernels3d.h"
#include "mrlbm.h"

using namespace mrlbm;

namespace {

int scheme_dim(int s) { return s == MRLBM_D3Q6 ? 3 : s == MRLBM_D2Q9 || s == MRLBM_D2Q4_EULER ? 2 : 1; }
int scheme_q(int s) {
  return s == MRLBM_D1Q2 ? 2 : s == MRLBM_D1Q3 ? 3 : s == MRLBM_D2Q9 ? 9 : s == MRLBM_D3Q6 ? 6 : 16;
}
void scheme_eta(int s, int h, int &ex, int &ey) {
  static const int d1q2[2] = {1, -1};
  static const int d1q3[3] = {0, 1, -1};
  static const int d2q9x[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  static const int d2q9y[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  static const int d2q4x[4] = {1, 0, -1, 0};
  static const int d2q4y[4] = {0, 1, 0, -1};
  if (s == MRLBM_D1Q2) { ex = d1q2[h]; ey = 0; }
  else if (s == MRLBM_D1Q3) { ex = d1q3[h]; ey = 0; }
  else if (s == MRLBM_D2Q9) { ex = d2q9x[h]; ey = d2q9y[h]; }
  else { ex = d2q4x[h & 3]; ey = d2q4y[h & 3]; }
}
bool conserved(int s, int i) {
  return s == MRLBM_D2Q9 ? i < 3 : s == MRLBM_D2Q4_EULER ? (i & 3) == 0 : i == 0;
}

int validate_one(const mrlbm_params *p) {
  if (!p) return MRLBM_ERR_INVALID;
  if (p->scheme < MRLBM_D1Q2 || p->scheme > MRLBM_D3Q6) return MRLBM_ERR_INVALID;
  if (p->scheme == MRLBM_D2Q4_EULER && !(p->eq_param > 1.0)) return MRLBM_ERR_INVALID;  // gamma_gas
  const int dim = scheme_dim(p->scheme);
  const int maxj = dim == 3 ? 8 : dim == 2 ? 13 : 25;  // 3D: cells of level 8 fill the 26 bits of a list entry
  if (dim == 3) {  // periodic, gamma = 1, finite velocity
    for (int k = 0; k < 4; ++k)
      if (p->bc[k] != MRLBM_PERIODIC) return MRLBM_ERR_INVALID;
    if (p->gamma > 1) return MRLBM_ERR_INVALID;
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(p->velocity[a])) return MRLBM_ERR_INVALID;
  }
  if (p->jmin < 1 || p->jmax < p->jmin || p->jmax > maxj) return MRLBM_ERR_INVALID;
  if (p->precision != 4 && p->precision != 8) return MRLBM_ERR_INVALID;
  if (!(p->lambda > 0.0) || !std::isfinite(p->lambda)) return MRLBM_ERR_INVALID;
  if (!(p->eps >= 0.0)) return MRLBM_ERR_INVALID;
  const int g = p->gamma == 0 ? 1 : p->gamma;
  if (g < 1 || g > 3 || (p->metric != MRLBM_METRIC_MAX && p->metric != MRLBM_METRIC_L2)) return MRLBM_ERR_INVALID;
  if (!(p->mu_bar >= 0.0 && p->mu_bar <= 2 * g + 1)) return MRLBM_ERR_INVALID;
  for (int i = 0; i < scheme_q(p->scheme); ++i) {
    if (!std::isfinite(p->s[i])) return MRLBM_ERR_INVALID;
    if (conserved(p->scheme, i) && p->s[i] != 0.0) return MRLBM_ERR_INVALID;
  }
  for (int k = 0; k < 4; ++k)
    if (p->bc[k] < MRLBM_PERIODIC || p->bc[k] > MRLBM_ANTI_BOUNCE_BACK) return MRLBM_ERR_INVALID;
  for (int a = 0; a < 2; ++a)  // an axis is periodic on both sides or walled on both
    if ((p->bc[2 * a] == MRLBM_PERIODIC) != (p->bc[2 * a + 1] == MRLBM_PERIODIC)) return MRLBM_ERR_INVALID;
  if (dim == 1 && (p->bc[2] != MRLBM_PERIODIC || p->bc[3] != MRLBM_PERIODIC)) return MRLBM_ERR_INVALID;
  // one reflection at a wall covers the widest read (2 gamma cells) of the coarsest level
  if (p->bc[0] != MRLBM_PERIODIC || p->bc[2] != MRLBM_PERIODIC)
    if ((1 << p->jmin) < 2 * g) return MRLBM_ERR_INVALID;
  return MRLBM_OK;
}
int walls_of(const mrlbm_params *p) { return (p->bc[0] ? 1 : 0) | (p->bc[2] ? 2 : 0); }
int gamma_of(const mrlbm_params *p) { return p->gamma == 0 ? 1 : p->gamma; }

int validate(const mrlbm_params *p, int batch) {
  if (!p || batch < 1 || batch > MAXB) return MRLBM_ERR_INVALID;
  long long cells = 0;
  for (int i = 0; i < batch; ++i) {
    const int rc = validate_one(&p[i]);
    if (rc) return rc;
    if (p[i].scheme != p[0].scheme || p[i].precision != p[0].precision || p[i].jmin != p[0].jmin ||
        gamma_of(&p[i]) != gamma_of(&p[0]))
      return MRLBM_ERR_INVALID;
    for (int l = p[i].jmin; l <= p[i].jmax; ++l) cells += 1ll << (scheme_dim(p[i].scheme) * l);
  }
  if (cells >= (1ll << 31)) return MRLBM_ERR_INVALID;  // list positions are 32-bit
  return MRLBM_OK;
}

// ---------------------------------------------------------------- transport weights
// Coefficients c_1 .. c_gamma of the prediction of half-width gamma (Table 1).
double table1_coef(int g, int a) {
  static const double c[4][3] = {{0, 0, 0}, {-0.125, 0, 0}, {-22.0 / 128, 3.0 / 128, 0},
                                 {-201.0 / 1024, 11.0 / 256, -5.0 / 1024}};
  return c[g][a - 1];
}

// Value at finest index i of the reconstruction, m levels down, of a unit
// impulse on cell a of a coarse level, by repeated 1D prediction of half-width
// g: each level is computed on the window of cells that the levels below read.
long long floor_half(long long j) { return j >= 0 ? j / 2 : -((1 - j) / 2); }
double impulse_value(int g, int m, int a, long long i) {
  std::vector<long long> lo(m + 1), hi(m + 1);
  lo[m] = hi[m] = i;
  for (int k = m; k > 0; --k) {
    lo[k - 1] = floor_half(lo[k]) - g;
    hi[k - 1] = floor_half(hi[k]) + g;
  }
  std::vector<double> v((size_t)(hi[0] - lo[0] + 1));
  for (long long k = lo[0]; k <= hi[0]; ++k) v[(size_t)(k - lo[0])] = k == a ? 1.0 : 0.0;
  for (int k = 1; k <= m; ++k) {
    std::vector<double> w((size_t)(hi[k] - lo[k] + 1));
    const long long pl = lo[k - 1];
    auto at = [&](long long t) { return v[(size_t)(t - pl)]; };
    for (long long j = lo[k]; j <= hi[k]; ++j) {
      const long long p = floor_half(j);
      double q = table1_coef(g, 1) * (at(p + 1) - at(p - 1));
      for (int b = 2; b <= g; ++b) q = q + table1_coef(g, b) * (at(p + b) - at(p - b));
      w[(size_t)(j - lo[k])] = (j & 1) ? at(p) - q : at(p) + q;
    }
    v.swap(w);
  }
  return v[0];
}

// Sums of the reconstruction of a unit impulse at cell `a` of level J - m over
// ranges of finest cells. The prediction keeps the sum of each pair of children
// equal to twice their parent, so a whole block of 2^m finest cells under a
// coarse cell k sums to 2^m [k == a]; a range that differs from whole blocks by
// a cell at either end adds or takes that cell's value.
struct ImpulseSums {
  int g;
  explicit ImpulseSums(int gamma) : g(gamma) {}
  // Sum over the finest cells [-e, 2^n - e) (the leaf's finest cells shifted by
  // -e, |e| <= 1; the leaf covers [0, 2^n) finest cells, n >= m). A leaf
  // touching a wall (wall = 1: the lower one, at finest cell 0; 2: the upper
  // one, at 2^n) sums only the cells on its side of it.
  double sum(int n, int m, int e, int a, int wall = 0) {
    const long long N = 1ll << n;
    long long b0 = -e, b1 = N - e;
    if (wall == 1) b0 = std::max(b0, 0ll);
    if (wall == 2) b1 = std::min(b1, N);
    double s = (a >= 0 && a < (1ll << (n - m))) ? std::ldexp(1.0, m) : 0.0;
    for (long long i = b0; i < 0; ++i) s += impulse_value(g, m, a, i);
    for (long long i = 0; i < b0; ++i) s -= impulse_value(g, m, a, i);
    for (long long i = N; i < b1; ++i) s += impulse_value(g, m, a, i);
    for (long long i = b1; i < N; ++i) s -= impulse_value(g, m, a, i);
    return s;
  }
};

// W[h][(2R+1)^2] and C[h][(2R+2)^2], R = 2 gamma, of a leaf n >= 1 levels
// above the finest (see header; a 1D scheme uses the middle rows). With a wall
// case (per axis 0 none, 1 the leaf touches the lower wall, 2 the upper one)
// the sums over E leave out the finest cells beyond the walls (E minus those
// cells is still a box: (B - eta) clipped to the domain), and N[h][2] receives
// how many of those cells lie beyond the x wall and, with x inside, beyond the
// y wall.
void transport_tables(int scheme, int n, double *W, double *C, int wx = 0, int wy = 0, double *N = nullptr,
                      int g = 1, ImpulseSums *cache = nullptr) {
  const int q = scheme_q(scheme), dim = scheme_dim(scheme), R = 2 * g, WW = 2 * R + 1, CW = 2 * R + 2;
  ImpulseSums own(g);
  ImpulseSums &is = cache ? *cache : own;
  for (int h = 0; h < q; ++h) {
    int ex, ey;
    scheme_eta(scheme, h, ex, ey);
    double Sx[13], Sy[13], Tx[14], Ty[14];
    for (int a = -R; a <= R; ++a) {
      Sx[a + R] = is.sum(n, n, ex, a, wx);
      Sy[a + R] = dim == 2 ? is.sum(n, n, ey, a, wy) : (a == 0 ? 1.0 : 0.0);
    }
    // detail impulses live one level below the leaf, on cells 2k + y, y in
    // [-R, R+1]; the leaf's range is then [0, 2) cells of that level = [0, 2^n)
    // finest cells
    for (int y = -R; y <= R + 1; ++y) {
      Tx[y + R] = is.sum(n, n - 1, ex, y, wx);
      Ty[y + R] = dim == 2 ? is.sum(n, n - 1, ey, y, wy) : (y == 0 ? 1.0 : 0.0);
    }
    if (N) {  // positions of [-e, 2^n - e) beyond the touched wall, per axis
      const double w = std::ldexp(1.0, n);
      const double ox = (wx == 1 && ex > 0) || (wx == 2 && ex < 0) ? 1.0 : 0.0;
      const double oy = dim == 2 && ((wy == 1 && ey > 0) || (wy == 2 && ey < 0)) ? 1.0 : 0.0;
      N[2 * h] = ox * (dim == 2 ? w : 1.0);
      N[2 * h + 1] = (w - ox) * oy;
      if (ex == 0 && ey == 0) N[2 * h] = N[2 * h + 1] = 0.0;
    }
    const double full = std::ldexp(1.0, dim * n);
    const bool rest = ex == 0 && ey == 0;
    for (int b = -R; b <= R; ++b)
      for (int a = -R; a <= R; ++a) {
        double w = Sx[a + R] * Sy[b + R];
        if (a == 0 && b == 0) w -= rest ? w : full;  // E - A form; rest velocity: 0
        W[h * WW * WW + (b + R) * WW + (a + R)] = w;
      }
    for (int y2 = -R; y2 <= R + 1; ++y2)
      for (int y1 = -R; y1 <= R + 1; ++y1)
        C[h * CW * CW + (y2 + R) * CW + (y1 + R)] = rest ? 0.0 : Tx[y1 + R] * Ty[y2 + R];
  }
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
// Entries per population of the general path's tables: (4 gamma + 1)^d and (4 gamma + 2)^d.
int wide_ws(int dim, int g) { return dim == 2 ? (4 * g + 1) * (4 * g + 1) : 4 * g + 1; }
int wide_cs(int dim, int g) { return dim == 2 ? (4 * g + 2) * (4 * g + 2) : 4 * g + 2; }

// Dense per-level passes: cells per block, and the levels they cover
// (jmin <= L <= jmax - margin): ghost classification with 4 cells per thread
// (0) or 16 (3), grading (1, level l-1 of l; one cell per thread of the fused
// block of q populations) and ancestor closure (2, level l-2 of l) with one.
constexpr int NDENSE = 4;
long long dense_cells(int off, int q) {
  return off == 0 ? (long long)GCHUNK : off == 3 ? (long long)CCHUNK : off == 1 ? (long long)std::max(64 * q, BLK)
                                                                                  : (long long)BLK;
}
int dense_margin(int off) { return off == 1 ? 1 : off == 2 ? 2 : 0; }

// Static description of a batch: instance descriptors (double-precision
// thresholds; converted to the working precision on upload), block tables, and
// the workspace layout.
struct Plan {
  int B, dim, q, jmin, maxJ, nmax, nblocks;
  int gamma;       // prediction half-width, shared by the batch (the transport tables depend on it)
  int metric_mode; // sibling metric of every instance (0 max, 1 l2), or 2 if they differ
  bool any_walls;  // some instance has walls: the launches take the kernel variants that handle them
  size_t rs;
  long long ctotal;
  std::vector<Inst<double>> inst;
  std::vector<long long> cb;   // [B + 1] first cell of each instance
  std::vector<int> cbp;        // [B + 1] first compaction block of each instance
  std::vector<int> dtab;       // [NDENSE][LVL_STRIDE][B + 1] dense-level block prefixes
  std::vector<uint32_t> binfo; // [nblocks] instance | level << 8 | chunk << 13 of all-level passes
  std::vector<uint32_t> dinfo; // dense per-level passes: instance | chunk << 8, rows at dstart
  std::vector<uint32_t> wband; // wall bands of the transport (gamma = 1 with walls): instance | level << 8 | chunk << 13
  std::vector<uint32_t> gtile; // gamma > 1: tiles of the ghost classification, instance | tile << 8, by level
  std::vector<long long> gtile_start;  // [LVL_STRIDE + 1] first tile of each level in gtile
  std::vector<long long> dstart;  // [NDENSE][LVL_STRIDE] first entry of each (off, L) row in dinfo
  bool ghost16[LVL_STRIDE];       // level L's codes (and L+1's) are 16-byte aligned in every instance
  size_t off_F[2], off_code[2], off_lists[2], off_lvl[2], off_keep, off_refg, off_tnew, off_mark, off_act, off_sync, off_ne[2], off_bcnt, off_boff, off_W,
      off_C, off_Wb, off_Cb, off_Nb, off_red, off_bad, off_cnt, off_inst, off_cb, off_cbp, off_dtab, off_binfo, off_dinfo, off_wband, off_gtile, bytes;
  int dtab_total(int off, int L) const { return dtab[((size_t)off * LVL_STRIDE + L) * (B + 1) + B]; }
  const uint32_t *dinfo_row(const uint32_t *dev, int off, int L) const {
    return dev + dstart[(size_t)off * LVL_STRIDE + L];
  }
};

void make_plan(const mrlbm_params *p, int B, Plan &P) {
  P.B = B;
  P.dim = scheme_dim(p[0].scheme);
  P.q = scheme_q(p[0].scheme);
  P.jmin = p[0].jmin;
  P.maxJ = 0;
  P.rs = p[0].precision == 8 ? 8 : 4;
  P.gamma = gamma_of(&p[0]);
  P.metric_mode = p[0].metric;
  for (int i = 1; i < B; ++i)
    if (p[i].metric != p[0].metric) P.metric_mode = 2;
  P.inst.assign(B, Inst<double>());
  P.any_walls = false;
  P.cb.assign(B + 1, 0);
  P.cbp.assign(B + 1, 0);
  long long cells = 0;
  int blocks = 0;
  for (int i = 0; i < B; ++i) {
    Inst<double> &I = P.inst[i];
    std::memset(&I, 0, sizeof I);
    I.jmin = p[i].jmin;
    I.jmax = p[i].jmax;
    P.maxJ = std::max(P.maxJ, I.jmax);
    I.cbase = cells;
    P.cb[i] = cells;
    P.cbp[i] = blocks;
    long long off = cells;
    for (int l = 0; l < LVL_STRIDE; ++l) {
      I.loff[l] = off;
      I.bstart[l] = blocks;
      if (l >= I.jmin && l <= I.jmax) {
        const long long n = 1ll << (P.dim * l);
        off += n;
        blocks += (int)((n + CCHUNK - 1) / CCHUNK);
      }
    }
    I.total = off - cells;
    cells = off;
    for (int l = 0; l < LVL_STRIDE; ++l) {
      I.eps_l[l] = std::ldexp(p[i].eps, P.dim * (l - p[i].jmax));
      I.ref_l[l] = std::ldexp(I.eps_l[l], P.dim) * std::exp2(p[i].mu_bar);
      if (p[i].metric == MRLBM_METRIC_L2) {  // the l2 metric is kept squared: squared thresholds
        I.eps_l[l] *= I.eps_l[l];
        I.ref_l[l] *= I.ref_l[l];
      }
    }
    I.gamma = P.gamma;
    I.metric = p[i].metric;
    I.sc.lam = p[i].lambda;
    I.sc.inv_lam = 1.0 / p[i].lambda;
    I.sc.eq = p[i].eq_param;
    for (int k = 0; k < 16; ++k) I.sc.s[k] = p[i].s[k];
    for (int k = 0; k < 3; ++k) I.sc.vel[k] = p[i].velocity[k];
    I.walls = walls_of(&p[i]);
    if (I.walls) P.any_walls = true;
    for (int k = 0; k < 4; ++k) I.bck[k] = p[i].bc[k];
  }
  P.cb[B] = cells;
  P.cbp[B] = blocks;
  P.binfo.clear();
  for (int i = 0; i < B; ++i)
    for (int l = P.inst[i].jmin; l <= P.inst[i].jmax; ++l) {
      const int nb = P.inst[i].bstart[l + 1] - P.inst[i].bstart[l];
      for (int k = 0; k < nb; ++k) P.binfo.push_back((uint32_t)i | ((uint32_t)l << 8) | ((uint32_t)k << 13));
    }
  P.ctotal = cells;
  P.nblocks = blocks;
  P.nmax = P.maxJ - P.jmin;
  // dense passes over level L of every instance where jmin <= L <= jmax - off
  P.dtab.assign((size_t)NDENSE * LVL_STRIDE * (B + 1), 0);
  for (int off = 0; off < NDENSE; ++off)
    for (int L = 0; L < LVL_STRIDE; ++L) {
      int *row = &P.dtab[((size_t)off * LVL_STRIDE + L) * (B + 1)];
      int acc = 0;
      for (int i = 0; i < B; ++i) {
        row[i] = acc;
        if (L >= P.jmin && L <= P.inst[i].jmax - dense_margin(off))
          acc += (int)(((1ll << (P.dim * L)) + dense_cells(off, P.q) - 1) / dense_cells(off, P.q));
      }
      row[B] = acc;
    }
  P.dinfo.clear();
  P.dstart.assign((size_t)NDENSE * LVL_STRIDE, 0);
  for (int off = 0; off < NDENSE; ++off)
    for (int L = 0; L < LVL_STRIDE; ++L) {
      P.dstart[(size_t)off * LVL_STRIDE + L] = (long long)P.dinfo.size();
      for (int i = 0; i < B; ++i)
        if (L >= P.jmin && L <= P.inst[i].jmax - dense_margin(off)) {
          const int nb = (int)(((1ll << (P.dim * L)) + dense_cells(off, P.q) - 1) / dense_cells(off, P.q));
          for (int k = 0; k < nb; ++k) P.dinfo.push_back((uint32_t)i | ((uint32_t)k << 8));
        }
    }
  // cells within R = 2 gamma of a wall, per instance with walls and level: the
  // rows of the y band, then the columns of the x band in the other rows
  P.wband.clear();
  for (int i = 0; i < B && P.gamma == 1; ++i) {
    const int walls = P.inst[i].walls, R = 2 * P.gamma;
    if (!walls) continue;
    for (int l = P.inst[i].jmin; l <= P.inst[i].jmax; ++l) {
      const long long N = 1ll << l;
      const long long rows = (P.dim == 2 && (walls & 2)) ? std::min<long long>(2 * R, N) : 0;
      const long long cols = (walls & 1) ? std::min<long long>(2 * R, N) : 0;
      const long long n = rows * N + (P.dim == 2 ? N - rows : 1) * cols;
      for (long long k = 0; k < (n + WBAND_CHUNK - 1) / WBAND_CHUNK; ++k)
        P.wband.push_back((uint32_t)i | ((uint32_t)l << 8) | ((uint32_t)k << 13));
    }
  }
  // gamma > 1: tiles of GT_X x GT_Y cells (1D: GT_X * GT_Y) of every level above jmin
  P.gtile.clear();
  P.gtile_start.assign(LVL_STRIDE + 1, 0);
  for (int l = 0; l < LVL_STRIDE; ++l) {
    P.gtile_start[l] = (long long)P.gtile.size();
    if (P.gamma == 1 || l <= P.jmin) continue;
    const long long N = 1ll << l, tx = P.dim == 2 ? GT_X : GT_X * GT_Y, ty = P.dim == 2 ? GT_Y : 1;
    const long long nt = ((N + tx - 1) / tx) * (P.dim == 2 ? (N + ty - 1) / ty : 1);
    for (int i = 0; i < B; ++i)
      if (l <= P.inst[i].jmax)
        for (long long t = 0; t < nt; ++t) P.gtile.push_back((uint32_t)i | ((uint32_t)t << 8));
  }
  P.gtile_start[LVL_STRIDE] = (long long)P.gtile.size();
  for (int L = 0; L < LVL_STRIDE; ++L) {
    bool ok = L >= 4;
    for (int i = 0; i < B && ok; ++i)
      if (L >= P.inst[i].jmin && L <= P.inst[i].jmax)
        ok = P.inst[i].loff[L] % 16 == 0 && (L == P.inst[i].jmax || P.inst[i].loff[L + 1] % 16 == 0);
    P.ghost16[L] = ok;
  }
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
  for (int k = 0; k < 2; ++k) P.off_F[k] = take(P.rs * P.q * P.ctotal);
  for (int k = 0; k < 2; ++k) P.off_code[k] = take(P.ctotal);
  for (int k = 0; k < 2; ++k) P.off_lists[k] = take(sizeof(uint32_t) * NCAT * P.ctotal);
  for (int k = 0; k < 2; ++k) P.off_lvl[k] = take(sizeof(int) * B * NCAT * LVL_STRIDE);
  P.off_keep = take(P.ctotal);
  P.off_refg = take(P.ctotal);
  P.off_tnew = take(P.ctotal);
  P.off_mark = take(P.ctotal);
  P.off_act = take(sizeof(int) * ACT * B);
  P.off_sync = take(sizeof(unsigned) * 4);
  for (int k = 0; k < 2; ++k) P.off_ne[k] = take(sizeof(int) * NCAT * LVL_STRIDE);
  P.off_bcnt = take(sizeof(int) * NCAT * P.nblocks);
  P.off_boff = take(sizeof(int) * NCAT * P.nblocks);
  const int ws = P.dim == 2 ? 25 : 5, cs = P.dim == 2 ? 36 : 6;
  P.off_W = take(P.rs * std::max(1, P.nmax) * P.q * ws);
  P.off_C = take(P.rs * std::max(1, P.nmax) * P.q * cs);
  // tables of the general path (walls, gamma > 1): [n - 1][wall case 0..8][h][.]
  P.off_Wb = take(P.rs * std::max(1, P.nmax) * 9 * P.q * wide_ws(P.dim, P.gamma));
  P.off_Cb = take(P.rs * std::max(1, P.nmax) * 9 * P.q * wide_cs(P.dim, P.gamma));
  P.off_Nb = take(P.rs * std::max(1, P.nmax) * 9 * P.q * 2);
  P.off_red = take(sizeof(double) * 2 * RED_BLOCKS * B);
  P.off_bad = take(sizeof(int) * std::max(4, B));  // non-finite flag per instance
  P.off_cnt = take(sizeof(unsigned long long) * 4);
  P.off_inst = take(std::max(sizeof(Inst<double>), sizeof(Inst<float>)) * B);
  P.off_cb = take(sizeof(long long) * (B + 1));
  P.off_cbp = take(sizeof(int) * (B + 1));
  P.off_dtab = take(sizeof(int) * P.dtab.size());
  P.off_binfo = take(sizeof(uint32_t) * P.binfo.size());
  P.off_dinfo = take(sizeof(uint32_t) * std::max<size_t>(1, P.dinfo.size()));
  P.off_wband = take(sizeof(uint32_t) * std::max<size_t>(1, P.wband.size()));
  P.off_gtile = take(sizeof(uint32_t) * std::max<size_t>(1, P.gtile.size()));
  P.bytes = o + 256;  // slack for aligning the base pointer
}

// Moment matrix M of a scheme (rows scaled by powers of lambda) and its inverse
// (Gauss-Jordan with partial pivoting), for the adjoint of the collision.
void moment_mats(int scheme, double lam, double *M, double *Minv) {
  const int q = scheme_q(scheme);
  const double L = lam, L2 = L * L, L3 = L2 * L, L4 = L2 * L2;
  std::memset(M, 0, sizeof(double) * 81);
  if (scheme == MRLBM_D1Q2) {
    const double m[4] = {1, 1, L, -L};
    std::memcpy(M, m, sizeof m);
  } else if (scheme == MRLBM_D1Q3) {
    const double m[9] = {1, 1, 1, 0, L, -L, 0, L2, L2};
    std::memcpy(M, m, sizeof m);
  } else {
    const double m[81] = {1, 1, 1, 1, 1, 1, 1, 1, 1,
                          0, L, 0, -L, 0, L, -L, -L, L,
                          0, 0, L, 0, -L, L, L, -L, -L,
                          -4 * L2, -L2, -L2, -L2, -L2, 2 * L2, 2 * L2, 2 * L2, 2 * L2,
                          0, -2 * L3, 0, 2 * L3, 0, L3, -L3, -L3, L3,
                          0, 0, -2 * L3, 0, 2 * L3, L3, L3, -L3, -L3,
                          4 * L4, -2 * L4, -2 * L4, -2 * L4, -2 * L4, L4, L4, L4, L4,
                          0, L2, -L2, L2, -L2, 0, 0, 0, 0,
                          0, 0, 0, 0, 0, L2, -L2, L2, -L2};
    std::memcpy(M, m, sizeof m);
  }
  double A[9][18];
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < 2 * q; ++j) A[i][j] = j < q ? M[i * q + j] : (j - q == i ? 1.0 : 0.0);
  for (int col = 0; col < q; ++col) {
    int piv = col;
    for (int r = col + 1; r < q; ++r)
      if (std::fabs(A[r][col]) > std::fabs(A[piv][col])) piv = r;
    for (int j = 0; j < 2 * q; ++j) std::swap(A[col][j], A[piv][j]);
    const double dd = A[col][col];
    for (int j = 0; j < 2 * q; ++j) A[col][j] /= dd;
    for (int r = 0; r < q; ++r) {
      if (r == col) continue;
      const double f = A[r][col];
      for (int j = 0; j < 2 * q; ++j) A[r][j] -= f * A[col][j];
    }
  }
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < q; ++j) Minv[i * q + j] = A[i][q + j];
}

// Layout of the adjoint workspace: one checkpoint (codes and populations) every
// K steps; for two segments of K steps (the one being swept backwards and the
// one being recomputed; one when a single segment covers the run) the tape
// (each step's new mesh and pre-collision populations) and the mesh the
// segment starts from; four adjoint buffers.
struct AdjLayout {
  int nck;
  size_t code_b, F_b, lists_b, lvl_b;
  size_t ck_code, ck_F, tape_code, tape_lists, tape_lvl, tape_h, st_code, st_lists, st_lvl, A, Hb, Gs, Go, spart, rec_lvl,
      bytes;
};
constexpr int ADJ_GRID = 512;

AdjLayout adj_layout(const Plan &P, int nsteps, int K) {
  AdjLayout L;
  L.nck = (nsteps + K - 1) / K;
  L.code_b = align256(P.ctotal);
  L.F_b = align256(P.rs * P.q * P.ctotal);
  L.lists_b = align256(sizeof(uint32_t) * NCAT * P.ctotal);
  L.lvl_b = align256(sizeof(int) * P.B * NCAT * LVL_STRIDE);
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += align256(bytes); return r; };
  L.ck_code = take(L.code_b * std::max(1, L.nck));
  L.ck_F = take(L.F_b * std::max(1, L.nck));
  const size_t nt = L.nck > 1 ? 2 : 1, Kt = std::min(K, nsteps);  // tape b of a field starts at b times its size
  L.tape_code = take(L.code_b * Kt * nt);
  L.tape_lists = take(L.lists_b * Kt * nt);
  L.tape_lvl = take(L.lvl_b * Kt * nt);
  L.tape_h = take(L.F_b * Kt * nt);
  L.st_code = take(L.code_b * nt);
  L.st_lists = take(L.lists_b * nt);
  L.st_lvl = take(L.lvl_b * nt);
  L.A = take(L.F_b);
  L.Hb = take(L.F_b);
  L.Gs = take(L.F_b);
  L.Go = take(L.F_b);
  L.spart = take(sizeof(double) * 9 * ADJ_GRID);
  L.rec_lvl = take(L.lvl_b * ((size_t)nsteps + 1));  // list bounds of every mesh of the recorded run
  L.bytes = o + 256;
  return L;
}

unsigned grid_cap(long long n, unsigned cap) {
  if (n < 1) n = 1;
  return (unsigned)(n > cap ? cap : n);
}
// Grid of a list kernel: a multiple of the 8 XCDs (see chunk_sched).
unsigned list_grid(long long chunks, unsigned cap) { return (grid_cap(chunks, cap) + NXCD - 1) / NXCD * NXCD; }

}  // namespace

struct mrlbm_ctx {
  std::vector<mrlbm_params> p;
  Plan P;
  Batch bt;
  hipStream_t stream;
  void *F[2];
  uint8_t *code[2];
  uint32_t *lists[2];
  int *lvl[2];
  uint8_t *keep, *refg, *tnew;
  uint8_t *mark;      // change marks of the reconstruction after an adaptation
  int *act;           // mesh activity per instance (see active_top)
  unsigned *sync;     // paired links: counter, leave count, spin budget, sticky timeout flag
  int *ne[2];         // per mesh: lists with items at [category][level] (0/1)
  bool recon_reuse;   // the next reconstruction follows an adaptation
  int *bcnt, *boff;
  void *W, *C;
  void *Wb, *Cb, *Nb;  // transport tables of the leaves touching a wall
  double *red;
  int *bad;
  unsigned long long *cnt;  // device counters: leaf updates, transport launches
  void *inst;               // Inst<T>[B]
  long long *cb;
  int *cbp, *dtab;
  uint32_t *binfo, *dinfo, *wband, *gtile;
  int cur;   // F[cur] holds the state
  int mcur;  // code/lists/lvl[mcur] describe the current mesh
  std::vector<char> has_state;
  int transport_variant;  // 0: by size, 1: one thread per leaf, 2: one wavefront per population
  bool pair_links;        // the finest two links of the level chains share a launch (tuning pair_links)
  unsigned grid_all, grid_level;  // block caps of the all-level and per-level list kernels
  // adjoint: checkpoints and tape of a recorded run (workspace owned by the caller)
  char *adj_ws;
  int adj_nsteps, adj_K;
  bool adj_taped;  // the recorded forward wrote the tape (a single segment)
  // HIP graphs of one step, captured on a private stream: [plain (0) or with
  // event-record nodes around the transport kernel (1)][2 * cur + mcur]. The
  // timed graphs keep their source graph and event nodes, whose events are
  // pointed at fresh pool events before each launch.
  bool use_graph;
  int static_dev;  // device whose static workspace the context uses, or -1 (caller's workspace)
  hipStream_t cap_stream;
  hipGraphExec_t graph[2][4];
  hipGraph_t timed_src[4];
  hipGraphNode_t timed_ev[4][2];
  hipEvent_t ev_placeholder;
  bool profiling;
  unsigned long long timing_period;  // graph steps per event-timed transport launch (1 or 8)
  unsigned long long graph_steps;    // graph-replayed steps since profiling was switched on
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used;
  std::vector<std::pair<int, size_t>> ev_marks;  // (phase, index of the first of two events)
  bool all_ready() const {
    for (char h : has_state)
      if (!h) return false;
    return true;
  }
};

namespace {

// Every level active until the compaction has built two meshes (after the
// mesh or the buffers were set from outside the step sequence).
void activity_reset(mrlbm_ctx *c) {
  k_fill_u32<<<1, BLK, 0, c->stream>>>((uint32_t *)c->act, (long long)ACT * c->P.B, (uint32_t)ACT_ALL);
}

#define HIPCHK(x)                                \
  do {                                           \
    if ((x) != hipSuccess) return MRLBM_ERR_HIP; \
  } while (0)

enum { PH_TRANSPORT = 0, PH_RECON = 1, PH_ADAPT = 2 };

// Timing events: no system-scope fence when they are recorded (no cache
// writeback and invalidation around the timed kernel, which would slow it
// down); they are read only after the stream has been synchronised.
hipError_t timing_event(hipEvent_t *e) { return hipEventCreateWithFlags(e, hipEventDisableSystemFence); }

// Start (begin = true) or end a timed phase: two events on the context stream.
void phase_mark(mrlbm_ctx *c, int phase, bool begin) {
  if (!c->profiling) return;
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e;
    if (timing_event(&e) != hipSuccess) return;
    c->ev_pool.push_back(e);
  }
  if (begin) c->ev_marks.push_back({phase, c->ev_used});
  (void)hipEventRecord(c->ev_pool[c->ev_used++], c->stream);
}

constexpr unsigned LIST_GRID_LEVEL = 1024, LIST_GRID_ALL = 4096, DENSE_GRID = 4096;
constexpr unsigned PAIR_WAIT_BUDGET = 1u << 20;  // spins of a paired-link wait (about 50 ms)

// Sticky device-side failure of the context: a paired-link wait that gave up
// (sync[3]). Synchronises the context stream.
int sync_status(mrlbm_ctx *c) {
  unsigned flag = 0;
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(&flag, c->sync + 3, sizeof flag, hipMemcpyDeviceToHost));
  return flag ? MRLBM_ERR_SYNC : MRLBM_OK;
}

// Invalidate the captured step graphs (after a change of the launch schedule).
void drop_graphs(mrlbm_ctx *c) {
  for (auto &row : c->graph)
    for (auto &g : row)
      if (g) {
        (void)hipGraphExecDestroy(g);
        g = nullptr;
      }
  for (auto &g : c->timed_src)
    if (g) {
      (void)hipGraphDestroy(g);
      g = nullptr;
    }
}

// Event-record nodes e0 -> (the last `count` kernel nodes) -> e1 in a captured
// linear graph whose last nodes are the transport kernels; returns the two nodes.
hipError_t bracket_last_kernels(hipGraph_t g, hipEvent_t ev, hipGraphNode_t *n0, hipGraphNode_t *n1, int count) {
  size_t n = 0;
  hipError_t e = hipGraphGetNodes(g, nullptr, &n);
  if (e != hipSuccess) return e;
  if (n == 0) return hipErrorInvalidValue;
  std::vector<hipGraphNode_t> nodes(n);
  if ((e = hipGraphGetNodes(g, nodes.data(), &n)) != hipSuccess) return e;
  hipGraphNode_t sink = nullptr;
  for (hipGraphNode_t nd : nodes) {
    size_t k = 0;
    if ((e = hipGraphNodeGetDependentNodes(nd, nullptr, &k)) != hipSuccess) return e;
    if (k == 0) {
      if (sink) return hipErrorInvalidValue;  // not a chain
      sink = nd;
    }
  }
  hipGraphNodeType type;
  if (!sink || (e = hipGraphNodeGetType(sink, &type)) != hipSuccess) return sink ? e : hipErrorInvalidValue;
  if (type != hipGraphNodeTypeKernel) return hipErrorInvalidValue;
  // walk back to the first of the last `count` kernel nodes (a chain: one dependency each)
  hipGraphNode_t first = sink;
  for (int k = 1; k < count; ++k) {
    size_t np = 0;
    if ((e = hipGraphNodeGetDependencies(first, nullptr, &np)) != hipSuccess) return e;
    if (np != 1) return hipErrorInvalidValue;
    hipGraphNode_t prev = nullptr;
    if ((e = hipGraphNodeGetDependencies(first, &prev, &np)) != hipSuccess) return e;
    first = prev;
    if ((e = hipGraphNodeGetType(first, &type)) != hipSuccess) return e;
    if (type != hipGraphNodeTypeKernel) return hipErrorInvalidValue;
  }
  size_t nd = 0;
  if ((e = hipGraphNodeGetDependencies(first, nullptr, &nd)) != hipSuccess) return e;
  std::vector<hipGraphNode_t> deps(nd);
  if (nd && (e = hipGraphNodeGetDependencies(first, deps.data(), &nd)) != hipSuccess) return e;
  for (hipGraphNode_t d : deps)
    if ((e = hipGraphRemoveDependencies(g, &d, &first, 1)) != hipSuccess) return e;
  if ((e = hipGraphAddEventRecordNode(n0, g, deps.data(), nd, ev)) != hipSuccess) return e;
  if ((e = hipGraphAddDependencies(g, n0, &first, 1)) != hipSuccess) return e;
  return hipGraphAddEventRecordNode(n1, g, &sink, 1, ev);
}
// Above this many cells (all instances and levels) the transport and the
// details run one thread per item; below, one wavefront per population (more
// parallelism for small sets). Both variants compute bit-identical results.
constexpr long long LEAF_KERNEL_CELLS = 1ll << 23;
constexpr unsigned long long TIMING_PERIOD = 8;  // graph steps per timed transport launch (profile mode 1)

// Step replay and dry-step timing, shared by the engines (E: the engine, with
// its adaptation, reconstruction and transport).
//
// One full step replayed from a HIP graph, one graph per assignment of the
// double buffers (a step swaps the mesh buffers and, in the transport, F). With
// profiling on, every TIMING_PERIOD-th step replays a graph in which
// event-record nodes bracket the transport kernel; before each such launch
// they are pointed at two fresh events. (Each event record drains the queue,
// some microseconds, so timing every step would slow the steps it measures.)
template <class E>
int step_graph_impl(mrlbm_ctx *c) {
  const int timed = c->profiling && (c->graph_steps++ % c->timing_period == 0) ? 1 : 0;
  const int par = c->mcur, key = 2 * c->cur + par;
  hipGraphExec_t &g = c->graph[timed][key];
  if (!g) {
    const int cur0 = c->cur;
    hipStream_t user = c->stream;
    const bool prof = c->profiling;
    c->stream = c->cap_stream;
    c->profiling = false;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed);
    int rc = e == hipSuccess ? E::adapt(c) : MRLBM_ERR_HIP;
    if (rc == MRLBM_OK) E::reconstruct(c, (typename E::Real *)c->F[c->cur], c->mcur);
    if (rc == MRLBM_OK) rc = E::transport_kernel(c);
    if (e == hipSuccess) e = hipStreamEndCapture(c->cap_stream, &graph);
    c->stream = user;
    c->profiling = prof;
    c->mcur = par;
    c->cur = cur0;
    if (rc == MRLBM_OK && e == hipSuccess && timed)
      e = bracket_last_kernels(graph, c->ev_placeholder, &c->timed_ev[key][0], &c->timed_ev[key][1],
                               E::transport_kernels(c));
    if (rc == MRLBM_OK && e == hipSuccess) e = hipGraphInstantiate(&g, graph, nullptr, nullptr, 0);
    if (rc == MRLBM_OK && e == hipSuccess && timed) {
      c->timed_src[key] = graph;  // the event nodes belong to it
      graph = nullptr;
    }
    if (graph) (void)hipGraphDestroy(graph);
    if (rc != MRLBM_OK) return rc;
    if (e != hipSuccess) { g = nullptr; return MRLBM_ERR_HIP; }
  }
  if (timed) {
    for (int k = 0; k < 2; ++k) {
      if (c->ev_used + k == c->ev_pool.size()) {
        hipEvent_t ev;
        if (timing_event(&ev) != hipSuccess) return MRLBM_ERR_HIP;
        c->ev_pool.push_back(ev);
      }
      if (hipGraphExecEventRecordNodeSetEvent(g, c->timed_ev[key][k], c->ev_pool[c->ev_used + k]) != hipSuccess)
        return MRLBM_ERR_HIP;
    }
    c->ev_marks.push_back({PH_TRANSPORT, c->ev_used});
    c->ev_used += 2;
  }
  if (hipGraphLaunch(g, c->stream) != hipSuccess) return MRLBM_ERR_HIP;
  c->mcur = 1 - par;    // the adaptation's swap
  c->cur = 1 - c->cur;  // the transport's swap
  return MRLBM_OK;
}

// A step that leaves the state as it was: the adaptation writes the next mesh
// buffers and, in the current value buffer, recomputes the values already
// there (its reconstruction) or writes cells outside the current mesh (its
// transfer); the transport then runs on the current mesh into the other value
// buffer. Captured once per schedule and replayed `reps` times between HIP
// events.
template <class E>
int time_dry_steps_impl(mrlbm_ctx *c, int reps, float *ms) {
  const int cur0 = c->cur, m0 = c->mcur;
  hipStream_t user = c->stream;
  const bool prof = c->profiling;
  c->stream = c->cap_stream;
  c->profiling = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed);
  // each replay repeats the same adaptation: every level active, as the
  // activity history would not match the replayed meshes
  if (e == hipSuccess) activity_reset(c);
  int rc = e == hipSuccess ? E::adapt(c) : MRLBM_ERR_HIP;
  c->mcur = m0;
  if (rc == MRLBM_OK) rc = E::transport(c);
  c->cur = cur0;
  if (e == hipSuccess) e = hipStreamEndCapture(c->cap_stream, &graph);
  c->stream = user;
  c->profiling = prof;
  if (rc == MRLBM_OK && e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  if (rc != MRLBM_OK) return rc;
  if (e != hipSuccess) return MRLBM_ERR_HIP;
  hipEvent_t a = nullptr, b = nullptr;
  e = timing_event(&a);
  if (e == hipSuccess) e = timing_event(&b);
  if (e == hipSuccess) e = hipGraphLaunch(exec, c->stream);  // warm-up
  if (e == hipSuccess) e = hipEventRecord(a, c->stream);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = hipGraphLaunch(exec, c->stream);
  if (e == hipSuccess) e = hipEventRecord(b, c->stream);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hipGraphExecDestroy(exec);
  activity_reset(c);  // the replays left the history of their own meshes
  if (e != hipSuccess) return MRLBM_ERR_HIP;
  *ms /= (float)reps;
  return MRLBM_OK;
}

// GAM = 1: a batch with gamma = 1 (the kernels that predict take it as a
// constant); GAM = 0: gamma > 1, read per instance.
template <int DIM, int SCHEME, typename T, int GAM>
struct Engine {
  using Real = T;
  static constexpr int Q = Vel<SCHEME>::Q;
  static constexpr unsigned QB = 64 * Q;
  static constexpr unsigned FB = fused_block<Q>();

  static const Inst<T> *I(mrlbm_ctx *c) { return (const Inst<T> *)c->inst; }
  static WallTabs<T> wall_tabs(mrlbm_ctx *c) { return WallTabs<T>{(const T *)c->Wb, (const T *)c->Cb, (const T *)c->Nb}; }
  static long long level_chunks(mrlbm_ctx *c, int l) {  // capacity of the per-level lists in chunks
    long long n = 0;
    for (int i = 0; i < c->P.B; ++i)
      if (l >= c->P.jmin && l <= c->P.inst[i].jmax) n += ((1ll << (DIM * l)) + CHUNK - 1) / CHUNK;
    return n;
  }
  static unsigned chunks_level(mrlbm_ctx *c, int l) { return list_grid(level_chunks(c, l), c->grid_level); }
  static unsigned chunks_all(mrlbm_ctx *c) { return list_grid((c->P.ctotal + CHUNK - 1) / CHUNK, c->grid_all); }
  // Finest level that the one-block-per-instance kernels walk: levels of at
  // most 4096 cells when the batch has 32 instances or more (one block each),
  // else of at most 1024 (with few blocks a larger level is better spread over
  // one launch of many blocks).
  static int coarse_cap(const mrlbm_ctx *c) {
    const long long cells = c->P.B >= 32 ? 4096 : 1024;
    int lc = 0;
    while ((1ll << (DIM * (lc + 1))) <= cells) ++lc;
    return lc;
  }
  // One thread per item and all populations in it (large sets), or one
  // wavefront per population (small sets: nine times the threads): for the
  // transport and the details.
  // Kernel launches of the transport: one, and the wall-band kernel for gamma = 1 with walls.
  static int transport_kernels(const mrlbm_ctx *c) {
    return (c->P.gamma == 1 && c->P.any_walls && !c->P.wband.empty()) ? 2 : 1;
  }
  static bool per_leaf(const mrlbm_ctx *c) {
    return c->transport_variant == 1 || (c->transport_variant == 0 && c->P.ctotal >= LEAF_KERNEL_CELLS);
  }

  // Lists of mesh m. With F, also the transfer from the mesh in code_old into
  // the new leaves of mesh m, in place in F (the adaptation).
  static void compact(mrlbm_ctx *c, int m, const uint8_t *code_old = nullptr, T *F = nullptr) {
    const Plan &P = c->P;
    k_compact_count<DIM, T><<<P.nblocks, BLK, 0, c->stream>>>(c->bt, I(c), c->binfo, c->code[m], c->bcnt, P.nblocks,
                                                               c->act, c->ne[m]);
    k_compact_scan<T><<<P.B, 1024, 0, c->stream>>>(c->bt, I(c), c->cbp, c->bcnt, c->boff, c->lvl[m], P.nblocks,
                                                   c->act, c->ne[m]);
    k_compact_scatter<DIM, Q, T, GAM><<<P.nblocks, BLK, 0, c->stream>>>(c->bt, I(c), c->binfo, c->code[m], c->boff,
                                                                   c->lists[m], P.nblocks, code_old, F, c->mark,
                                                                   c->act);
  }

  // Codes (leaf / internal / ghost) of the membership array tnew into code[m],
  // then its lists (and, with F, the transfer from the mesh in code_old).
  static void classify(mrlbm_ctx *c, int m, const uint8_t *code_old = nullptr, T *F = nullptr) {
    const Plan &P = c->P;
    k_classify_tree<DIM, T><<<P.nblocks, BLK, 0, c->stream>>>(c->bt, I(c), c->binfo, c->tnew, c->code[m], c->keep,
                                                              c->refg, c->act);
    const int lc = coarse_cap(c);
    if (P.gamma > 1) {  // wider stencils: one tiled pass per level, finest first
      for (int l = P.maxJ; l > P.jmin; --l) {
        const long long nb = P.gtile_start[l + 1] - P.gtile_start[l];
        if (nb)
          k_classify_ghost_tile<DIM, T><<<(unsigned)nb, BLK, 0, c->stream>>>(c->bt, I(c), c->code[m],
                                                                          c->gtile + P.gtile_start[l], l, c->act);
      }
      compact(c, m, code_old, F);
      return;
    }
    for (int l = P.maxJ; l > std::max(P.jmin, lc); --l) {
      if (P.ghost16[l]) {
        const int nb = P.dtab_total(3, l);
        if (nb)
          k_classify_ghost16<DIM, T><<<nb, BLK, 0, c->stream>>>(c->bt, I(c), c->code[m], P.dinfo_row(c->dinfo, 3, l), l,
                                                                c->act);
      } else {
        const int nb = P.dtab_total(0, l);
        if (nb)
          k_classify_ghost<DIM, T><<<nb, BLK, 0, c->stream>>>(c->bt, I(c), c->code[m], P.dinfo_row(c->dinfo, 0, l), l,
                                                              c->act);
      }
    }
    if (lc > P.jmin) {
      unsigned long long v16 = 0;
      for (int l = 0; l <= lc; ++l)
        if (P.ghost16[l]) v16 |= 1ull << l;
      k_classify_ghost_coarse<DIM, T><<<P.B, CBLK, 0, c->stream>>>(I(c), c->code[m], lc, v16);
    }

    compact(c, m, code_old, F);
  }

  // Projections of the internal cells of a mesh: levels above the coarse cap
  // one launch each (fine to coarse), then the coarse levels in one launch,
  // followed there by the coarse ghost predictions when lg is given. With
  // mark, only the cells whose subtree changed (k_project_marked).
  static void project_all(mrlbm_ctx *c, int m, T *F, const uint32_t *li, const int *lvl,
                          const uint32_t *lg = nullptr, uint8_t *mark = nullptr) {
    const Plan &P = c->P;
    const int lc = coarse_cap(c);
    int l = P.maxJ - 1;
    if (c->pair_links && l - 1 > std::max(P.jmin - 1, lc)) {  // the two finest levels share a launch
      if (mark) {
        const unsigned g0 = list_grid((level_chunks(c, l) + Q - 1) / Q, c->grid_level);
        const unsigned g1 = list_grid((level_chunks(c, l - 1) + Q - 1) / Q, c->grid_level);
        k_pair<DIM, Q, T, 2, GAM><<<g0 + g1, QB, 0, c->stream>>>(c->bt, I(c), F, li, lvl, l, l - 1, (int)g0, (int)g1,
                                                           c->sync, mark, c->ne[m]);
      } else {
        const unsigned g0 = chunks_level(c, l), g1 = chunks_level(c, l - 1);
        k_pair<DIM, Q, T, 0, GAM><<<g0 + g1, QB, 0, c->stream>>>(c->bt, I(c), F, li, lvl, l, l - 1, (int)g0, (int)g1,
                                                           c->sync, nullptr, c->ne[m]);
      }
      l -= 2;
    }
    for (; l > std::max(P.jmin - 1, lc); --l) {
      if (mark)
        k_project_marked<DIM, Q, T><<<list_grid((level_chunks(c, l) + BLK / 64 - 1) / (BLK / 64), c->grid_level), BLK,
                                      0, c->stream>>>(c->bt, I(c), F, li, lvl, l, mark);
      else
        k_project<DIM, Q, T><<<chunks_level(c, l), QB, 0, c->stream>>>(c->bt, I(c), F, li, lvl, l);
    }
    if (lc >= P.jmin)
      k_project_coarse<DIM, Q, T, GAM><<<P.B, CBLK, 0, c->stream>>>(I(c), F, li, lvl, lc, lc > P.jmin ? lg : nullptr,
                                                               mark);
  }

  // Reconstruction on mesh m inside F: projections upward, ghost predictions
  // downward. Right after an adaptation, only the projections that changed.
  static void reconstruct(mrlbm_ctx *c, T *F, int m) {
    const Plan &P = c->P;
    const uint32_t *li = c->lists[m] + (size_t)CAT_INTERNAL * P.ctotal;
    const uint32_t *lg = c->lists[m] + (size_t)CAT_GHOST * P.ctotal;
    const int lc = coarse_cap(c);
    project_all(c, m, F, li, c->lvl[m], lg, c->recon_reuse ? c->mark : nullptr);
    c->recon_reuse = false;
    const int l0 = std::max(P.jmin, lc) + 1;
    const int last = c->pair_links && P.maxJ - 1 >= l0 ? P.maxJ - 1 : P.maxJ + 1;  // first of the shared pair
    for (int l = l0; l <= P.maxJ && l < last; ++l)
      k_ghost<DIM, Q, T, GAM><<<chunks_level(c, l), QB, 0, c->stream>>>(c->bt, I(c), F, lg, c->lvl[m], l);
    if (last <= P.maxJ) {  // the two finest levels share a launch
      const unsigned g0 = chunks_level(c, last), g1 = chunks_level(c, last + 1);
      k_pair<DIM, Q, T, 1, GAM><<<g0 + g1, QB, 0, c->stream>>>(c->bt, I(c), F, lg, c->lvl[m], last, last + 1, (int)g0,
                                                         (int)g1, c->sync, nullptr, c->ne[m]);
    }
  }

  static int adapt(mrlbm_ctx *c) {
    const Plan &P = c->P;
    const int mo = c->mcur, mn = 1 - c->mcur;
    T *Fc = (T *)c->F[c->cur];
    const uint32_t *li = c->lists[mo] + (size_t)CAT_INTERNAL * P.ctotal;
    const uint32_t *lg = c->lists[mo] + (size_t)CAT_GHOST * P.ctotal;
    phase_mark(c, PH_ADAPT, true);
    // Projections of the old mesh (the details read tree cells only). The keep
    // and refine flags are zero here: the tree classification of the previous
    // adaptation, or the creation, cleared them.
    project_all(c, mo, Fc, li, c->lvl[mo]);
    // the sibling metric as a constant when the batch shares it
    if (per_leaf(c)) {
      auto kern = P.metric_mode == 0   ? k_details_leaf<DIM, Q, T, GAM, 0>
                  : P.metric_mode == 1 ? k_details_leaf<DIM, Q, T, GAM, 1>
                                       : k_details_leaf<DIM, Q, T, GAM, 2>;
      kern<<<list_grid((P.ctotal + BLK - 1) / BLK, c->grid_all), BLK, 0, c->stream>>>(
          c->bt, I(c), Fc, c->lists[mo] + (size_t)CAT_INTERNAL * P.ctotal, c->lvl[mo], c->keep, c->refg, c->act);
    } else {
      auto kern = P.metric_mode == 0   ? k_details<DIM, Q, T, GAM, 0>
                  : P.metric_mode == 1 ? k_details<DIM, Q, T, GAM, 1>
                                       : k_details<DIM, Q, T, GAM, 2>;
      kern<<<chunks_all(c), QB, 0, c->stream>>>(
          c->bt, I(c), Fc, c->lists[mo] + (size_t)CAT_INTERNAL * P.ctotal, c->lvl[mo], c->keep, c->refg, c->act);
    }
    const int lc = coarse_cap(c);
    int la = P.maxJ;
    const int la_end = std::max(P.jmin + 2, lc + 3);
    if (c->pair_links && la - 1 >= la_end && P.dtab_total(2, la - 2) && P.dtab_total(2, la - 3)) {
      // the two finest links in one launch, ordered when the finest has kept
      // cells (children of internal cells one level up in the old mesh)
      const int nb0 = P.dtab_total(2, la - 2), nb1 = P.dtab_total(2, la - 3);
      k_ancestor_pair<DIM, T><<<nb0 + nb1, BLK, 0, c->stream>>>(
          c->bt, I(c), c->keep, P.dinfo_row(c->dinfo, 2, la - 2), P.dinfo_row(c->dinfo, 2, la - 3), la, la - 1, nb0,
          nb1, c->act, c->ne[mo] + CAT_INTERNAL * LVL_STRIDE + (la - 1), c->sync);
      la -= 2;
    }
    for (int l = la; l >= la_end; --l) {
      const int nb = P.dtab_total(2, l - 2);
      if (nb)
        k_ancestor<DIM, T><<<nb, BLK, 0, c->stream>>>(c->bt, I(c), c->keep, P.dinfo_row(c->dinfo, 2, l - 2), l, c->act);
    }
    // the coarse ancestor closure; beside it the coarse link of the old mesh's
    // ghost predictions (which only the transfer reads), whose finer links
    // ride in the grading launches below
    if (lc > P.jmin)
      k_ancestor_ghost_coarse<DIM, Q, T, GAM><<<2 * P.B, CBLK, 0, c->stream>>>(I(c), c->keep, lc, P.B, Fc, lg,
                                                                         c->lvl[mo]);
    else if (lc + 2 >= P.jmin + 2)
      k_ancestor_coarse<DIM, T><<<P.B, CBLK, 0, c->stream>>>(I(c), c->keep, lc);

    auto enlarge = P.any_walls ? k_enlarge<DIM, SCHEME, T, true> : k_enlarge<DIM, SCHEME, T, false>;
    enlarge<<<P.nblocks, BLK, 0, c->stream>>>(c->bt, I(c), c->binfo, c->keep, c->refg, c->tnew,
                                                                c->act);
    // Grading (levels maxJ .. jmin+1) beside the finer links of the old mesh's
    // ghost predictions (levels above the coarse cap, coarse to fine): one link
    // of each chain per launch. The coarse levels of the grading are one link
    // (one block per instance); 0 marks a launch without that chain.
    {
      const int lc = coarse_cap(c);
      std::vector<int> gl, hl;  // levels, or -1 for the coarse link
      for (int l = P.maxJ; l >= std::max(P.jmin + 1, lc + 1); --l) gl.push_back(l);
      if (lc > P.jmin) gl.push_back(-1);
      for (int l = std::max(P.jmin, lc) + 1; l <= P.maxJ; ++l) hl.push_back(l);
      for (size_t k = 0; k < std::max(gl.size(), hl.size()); ++k) {
        const int g = k < gl.size() ? gl[k] : 0, h = k < hl.size() ? hl[k] : 0;
        const unsigned nb = g == 0 ? 0u : g < 0 ? (unsigned)P.B : (unsigned)P.dtab_total(1, g - 1);
        const unsigned G = h == 0 ? 0u : h < 0 ? (unsigned)P.B : chunks_level(c, h);
        const uint32_t *gi = g > 0 ? P.dinfo_row(c->dinfo, 1, g - 1) : c->dinfo;
        if (G + nb == 0) continue;
        const bool w = P.any_walls;
        auto kern = g < 0 && h < 0 ? (w ? k_grade_ghost<DIM, Q, T, true, true, true, GAM> : k_grade_ghost<DIM, Q, T, true, true, false, GAM>)
                    : g < 0        ? (w ? k_grade_ghost<DIM, Q, T, true, false, true, GAM> : k_grade_ghost<DIM, Q, T, true, false, false, GAM>)
                    : h < 0        ? (w ? k_grade_ghost<DIM, Q, T, false, true, true, GAM> : k_grade_ghost<DIM, Q, T, false, true, false, GAM>)
                                   : (w ? k_grade_ghost<DIM, Q, T, false, false, true, GAM> : k_grade_ghost<DIM, Q, T, false, false, false, GAM>);
        kern<<<G + nb, FB, 0, c->stream>>>(c->bt, I(c), c->tnew, gi, g, Fc, lg, c->lvl[mo], h, (int)G, lc, c->act);
      }
    }

    // new codes and lists, with the transfer in place: a new leaf's value is
    // the old reconstruction's value at that cell, which F already holds for
    // old leaves, merged cells (their projection) and old ghosts (their
    // prediction); only cells outside the old mesh are predicted from level
    // l-1, whose parent stencils lie in the old mesh (the old tree is graded
    // and refines by one level), so nothing read there is written there.
    classify(c, mn, c->code[mo], Fc);
    phase_mark(c, PH_ADAPT, false);
    c->mcur = mn;
    if (hipPeekAtLastError() != hipSuccess) return MRLBM_ERR_HIP;
    // F holds the old mesh's projections and the transfer: the next
    // reconstruction recomputes only what the marks name.
    c->recon_reuse = true;
    return MRLBM_OK;
  }

  static int transport(mrlbm_ctx *c, T *tape = nullptr) {
    phase_mark(c, PH_RECON, true);
    reconstruct(c, (T *)c->F[c->cur], c->mcur);
    phase_mark(c, PH_RECON, false);
    return transport_kernel(c, tape);
  }

  // The transport + collision kernel alone (the current mesh's reconstruction
  // must be in F[cur]).
  static int transport_kernel(mrlbm_ctx *c, T *tape = nullptr) {
    const Plan &P = c->P;
    const int m = c->mcur;
    T *Fc = (T *)c->F[c->cur];
    T *Fn = (T *)c->F[1 - c->cur];
    phase_mark(c, PH_TRANSPORT, true);
    const uint32_t *lf = c->lists[m] + (size_t)CAT_LEAF * P.ctotal;
    // kernel variant: 0 periodic with gamma = 1, 1 walls with gamma = 1 (the
    // wall band in a kernel of its own), gamma > 1: the variant of that gamma
    // (the general path near walls)
    const int mode = P.gamma > 1 ? P.gamma : (P.any_walls ? 1 : 0);
    if (per_leaf(c)) {
      auto kern = mode == 3   ? k_transport_collide_leaf<DIM, SCHEME, T, 3>
                  : mode == 2 ? k_transport_collide_leaf<DIM, SCHEME, T, 2>
                  : mode == 1 ? k_transport_collide_leaf<DIM, SCHEME, T, 1>
                              : k_transport_collide_leaf<DIM, SCHEME, T, 0>;
      kern<<<list_grid((P.ctotal + BLK - 1) / BLK, c->grid_all), BLK, 0, c->stream>>>(
          c->bt, I(c), Fc, Fn, c->code[m], lf, c->lvl[m], (const T *)c->W, (const T *)c->C, wall_tabs(c), c->cnt, tape);
    } else {
      auto kern = mode == 3   ? k_transport_collide_pop<DIM, SCHEME, T, 3>
                  : mode == 2 ? k_transport_collide_pop<DIM, SCHEME, T, 2>
                  : mode == 1 ? k_transport_collide_pop<DIM, SCHEME, T, 1>
                              : k_transport_collide_pop<DIM, SCHEME, T, 0>;
      kern<<<chunks_all(c), QB, 0, c->stream>>>(
          c->bt, I(c), Fc, Fn, c->code[m], lf, c->lvl[m], (const T *)c->W, (const T *)c->C, wall_tabs(c), c->cnt, tape);
    }
    if (mode == 1 && !P.wband.empty())  // the leaves near a wall, which the kernel above left out
      k_transport_wall_band<DIM, SCHEME, T><<<(unsigned)P.wband.size(), QB, 0, c->stream>>>(
          I(c), Fc, Fn, c->code[m], c->wband, wall_tabs(c), tape);
    phase_mark(c, PH_TRANSPORT, false);
    c->cur = 1 - c->cur;
    return hipPeekAtLastError() == hipSuccess ? MRLBM_OK : MRLBM_ERR_HIP;
  }

  static int step_graph(mrlbm_ctx *c) { return step_graph_impl<Engine>(c); }

  static int init(mrlbm_ctx *c, int i, const void *mom) {
    const Plan &P = c->P;
    T *F = (T *)c->F[c->cur];
    const long long nf = 1ll << (DIM * P.inst[i].jmax);
    k_init_equilibrium<DIM, SCHEME, T><<<grid_cap((nf + BLK - 1) / BLK, DENSE_GRID), BLK, 0, c->stream>>>(
        I(c), i, F, (const T *)mom);
    k_full_tree<T><<<grid_cap((P.inst[i].total + BLK - 1) / BLK, DENSE_GRID), BLK, 0, c->stream>>>(I(c), i,
                                                                                                  c->code[c->mcur]);
    activity_reset(c);
    compact(c, c->mcur);
    c->has_state[i] = 1;
    c->recon_reuse = false;
    return hipPeekAtLastError() == hipSuccess ? MRLBM_OK : MRLBM_ERR_HIP;
  }

  static int mass(mrlbm_ctx *c) {
    k_mass_partial<DIM, Q, T><<<dim3(RED_BLOCKS, c->P.B), BLK, 0, c->stream>>>(
        c->bt, I(c), (const T *)c->F[c->cur], c->lists[c->mcur] + (size_t)CAT_LEAF * c->P.ctotal, c->lvl[c->mcur],
        c->red, c->bad);
    return MRLBM_OK;
  }

  static int exportl(mrlbm_ctx *c, int i, uint32_t *cells, void *vals) {
    k_export<DIM, Q, T><<<grid_cap((c->P.inst[i].total + BLK - 1) / BLK, DENSE_GRID), BLK, 0, c->stream>>>(
        I(c), i, (const T *)c->F[c->cur], c->lists[c->mcur] + (size_t)CAT_LEAF * c->P.ctotal, c->lvl[c->mcur], cells,
        (T *)vals);
    return MRLBM_OK;
  }

  // Leaf table, populations or moments of instance i (device outputs, either
  // of cells / vals may be null for the first two).
  static int leaf_fields(mrlbm_ctx *c, int i, int what, void *out) {
    const long long n = c->P.inst[i].total;
    const unsigned g = grid_cap((n + BLK - 1) / BLK, DENSE_GRID);
    const uint32_t *lf = c->lists[c->mcur] + (size_t)CAT_LEAF * c->P.ctotal;
    if (what == MRLBM_FIELD_MOMENTS)
      k_moments<DIM, SCHEME, T><<<g, BLK, 0, c->stream>>>(I(c), i, (const T *)c->F[c->cur], lf, c->lvl[c->mcur],
                                                           (T *)out);
    else
      k_export<DIM, Q, T><<<g, BLK, 0, c->stream>>>(I(c), i, (const T *)c->F[c->cur], lf, c->lvl[c->mcur],
                                                    what == MRLBM_FIELD_LEAF_TABLE ? (uint32_t *)out : nullptr,
                                                    what == MRLBM_FIELD_POPULATIONS ? (T *)out : nullptr);
    return hipPeekAtLastError() == hipSuccess ? MRLBM_OK : MRLBM_ERR_HIP;
  }

  // The double-hat reconstruction of instance i on its finest level, [h][N_J^d]
  // into out: the reconstruction of the current mesh (projections, ghost
  // predictions), then the predictions of every other cell outside the tree,
  // level by level down to J, in F (cells outside the tree hold scratch).
  static int finest(mrlbm_ctx *c, int i, void *out) {
    const Inst<double> &In = c->P.inst[i];
    T *F = (T *)c->F[c->cur];
    reconstruct(c, F, c->mcur);
    for (int l = In.jmin + 1; l <= In.jmax; ++l)
      k_predict_outside<DIM, Q, T, GAM><<<grid_cap(((1ll << (DIM * l)) + BLK - 1) / BLK, DENSE_GRID), BLK, 0,
                                     c->stream>>>(I(c), i, F, c->code[c->mcur], l);
    const size_t bytes = sizeof(T) * Q * ((size_t)1 << (DIM * In.jmax));
    HIPCHK(hipMemcpyAsync(out, F + (size_t)Q * In.loff[In.jmax], bytes, hipMemcpyDeviceToDevice, c->stream));
    return hipPeekAtLastError() == hipSuccess ? MRLBM_OK : MRLBM_ERR_HIP;
  }

  // One step on given new trees (membership bytes of every instance, host):
  // the adaptation is replaced by the given mesh; the transfer, transport and
  // collision are those of a normal step.
  static int frozen(mrlbm_ctx *c, const uint8_t *trees) {
    const Plan &P = c->P;
    const int mo = c->mcur, mn = 1 - mo;
    T *Fc = (T *)c->F[c->cur];
    reconstruct(c, Fc, mo);  // the old mesh's projections and ghosts feed the transfer
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(c->tnew, trees, P.ctotal, hipMemcpyHostToDevice));
    activity_reset(c);
    classify(c, mn, c->code[mo], Fc);
    c->mcur = mn;
    c->recon_reuse = false;
    return transport(c);
  }

  // ---------------------------------------------------------------- adjoint
  struct Mesh {
    const uint8_t *code;
    const uint32_t *lists;
    const int *lvl;
  };

  static void copy_mesh_out(mrlbm_ctx *c, int m, uint8_t *code, uint32_t *lists, int *lvl) {
    const Plan &P = c->P;
    (void)hipMemcpyAsync(code, c->code[m], P.ctotal, hipMemcpyDeviceToDevice, c->stream);
    (void)hipMemcpyAsync(lists, c->lists[m], sizeof(uint32_t) * NCAT * P.ctotal, hipMemcpyDeviceToDevice, c->stream);
    (void)hipMemcpyAsync(lvl, c->lvl[m], sizeof(int) * P.B * NCAT * LVL_STRIDE, hipMemcpyDeviceToDevice, c->stream);
  }

  static void zero(mrlbm_ctx *c, void *p, size_t bytes) { zero(p, bytes, c->stream); }
  static void zero(void *p, size_t bytes, hipStream_t st) {
    const long long n4 = (long long)(bytes / 4);
    k_fill_u32<<<grid_cap((n4 + BLK - 1) / BLK, DENSE_GRID), BLK, 0, st>>>((uint32_t *)p, n4, 0u);
  }

  // From the current state (a restored checkpoint, or the recorded run's
  // start): rebuild the lists and run `steps` steps into tape b of the adjoint
  // workspace, taping each step's new mesh and pre-collision values.
  static int tape_segment(mrlbm_ctx *c, const AdjLayout &L, int K, int b, int steps) {
    char *w = c->adj_ws;
    activity_reset(c);  // the other code buffer and tnew hold later meshes
    compact(c, c->mcur);
    copy_mesh_out(c, c->mcur, (uint8_t *)(w + L.st_code + b * L.code_b), (uint32_t *)(w + L.st_lists + b * L.lists_b),
                  (int *)(w + L.st_lvl + b * L.lvl_b));
    for (int j = 0; j < steps; ++j) {
      const size_t k = (size_t)b * K + j;
      int rc = adapt(c);
      if (!rc) rc = transport(c, (T *)(w + L.tape_h + k * L.F_b));
      if (rc) return rc;
      copy_mesh_out(c, c->mcur, (uint8_t *)(w + L.tape_code + k * L.code_b),
                    (uint32_t *)(w + L.tape_lists + k * L.lists_b), (int *)(w + L.tape_lvl + k * L.lvl_b));
    }
    return MRLBM_OK;
  }

  static int record(mrlbm_ctx *c, int nsteps, int K) {
    const AdjLayout L = adj_layout(c->P, nsteps, K);
    char *w = c->adj_ws;
    if (L.nck == 1) {  // one segment: the run is taped now and the adjoint recomputes nothing
      (void)hipMemcpyAsync(w + L.ck_code, c->code[c->mcur], c->P.ctotal, hipMemcpyDeviceToDevice, c->stream);
      (void)hipMemcpyAsync(w + L.ck_F, c->F[c->cur], c->P.rs * c->P.q * c->P.ctotal, hipMemcpyDeviceToDevice,
                           c->stream);
      const int rc = tape_segment(c, L, K, 0, nsteps);
      if (rc) return rc;
      (void)hipMemcpyAsync(w + L.rec_lvl, w + L.st_lvl, L.lvl_b, hipMemcpyDeviceToDevice, c->stream);
      (void)hipMemcpyAsync(w + L.rec_lvl + L.lvl_b, w + L.tape_lvl, L.lvl_b * nsteps, hipMemcpyDeviceToDevice,
                           c->stream);
      c->adj_taped = true;
      return hipPeekAtLastError() == hipSuccess ? MRLBM_OK : MRLBM_ERR_HIP;
    }
    const size_t lvl_bytes = sizeof(int) * c->P.B * NCAT * LVL_STRIDE;
    (void)hipMemcpyAsync(w + L.rec_lvl, c->lvl[c->mcur], lvl_bytes, hipMemcpyDeviceToDevice, c->stream);
    for (int n = 0; n < nsteps; ++n) {
      if (n % K == 0) {
        const int k = n / K;
        (void)hipMemcpyAsync(w + L.ck_code + k * L.code_b, c->code[c->mcur], c->P.ctotal, hipMemcpyDeviceToDevice,
                             c->stream);
        (void)hipMemcpyAsync(w + L.ck_F + k * L.F_b, c->F[c->cur], c->P.rs * c->P.q * c->P.ctotal,
                             hipMemcpyDeviceToDevice, c->stream);
      }
      int rc;
      if (c->use_graph) {
        rc = step_graph(c);
      } else {
        rc = adapt(c);
        if (!rc) rc = transport(c);
      }
      if (rc) return rc;
      (void)hipMemcpyAsync(w + L.rec_lvl + (n + 1) * L.lvl_b, c->lvl[c->mcur], lvl_bytes, hipMemcpyDeviceToDevice,
                           c->stream);
    }
    return hipPeekAtLastError() == hipSuccess ? MRLBM_OK : MRLBM_ERR_HIP;
  }

  // Reconstruction transpose on mesh `ms` in the dense adjoint G: ghost
  // predictions pushed up from the finest level, then projections pushed down.
  // Levels up to the coarse cap in one launch (k_adj_coarse), finer levels a
  // launch each.
  // Levels whose ghost (internal) list is empty in every mesh of the run
  // (bits of gm, im clear) get no launch: it would do nothing.
  static void reconstruct_T(mrlbm_ctx *c, T *G, const Mesh &ms, hipStream_t st, uint64_t gm, uint64_t im) {
    const Plan &P = c->P;
    const int lc = std::max(P.jmin, coarse_cap(c));
    const uint32_t *lg = ms.lists + (size_t)CAT_GHOST * P.ctotal, *li = ms.lists + (size_t)CAT_INTERNAL * P.ctotal;
    for (int l = P.maxJ; l > lc; --l)
      if ((gm >> l) & 1u) k_adj_ghost<DIM, Q, T><<<ADJ_GRID, BLK, 0, st>>>(c->bt, I(c), G, lg, ms.lvl, l);
    k_adj_coarse<DIM, Q, T><<<P.B, CBLK, 0, st>>>(I(c), G, lg, li, ms.lvl, lc);
    for (int l = lc; l <= P.maxJ - 1; ++l)
      if ((im >> l) & 1u) k_adj_project<DIM, Q, T><<<ADJ_GRID, BLK, 0, st>>>(c->bt, I(c), G, li, ms.lvl, l);
  }

  // A second stream and its events for the adjoint sweep, and the graphs of
  // the segment recomputations (one per tape), released on scope exit.
  struct SweepStream {
    hipStream_t s = nullptr;
    hipEvent_t rec[2] = {nullptr, nullptr}, rev[2] = {nullptr, nullptr}, start = nullptr;
    hipGraphExec_t seg[2] = {nullptr, nullptr};
    hipGraphExec_t sw[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [tape][adjoint buffer in A]
    hipError_t init() {
      hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
      for (int b = 0; b < 2 && e == hipSuccess; ++b) {
        e = hipEventCreateWithFlags(&rec[b], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&rev[b], hipEventDisableTiming);
      }
      if (e == hipSuccess) e = hipEventCreateWithFlags(&start, hipEventDisableTiming);
      return e;
    }
    ~SweepStream() {
      if (s) (void)hipStreamSynchronize(s);
      for (int b = 0; b < 2; ++b) {
        if (rec[b]) (void)hipEventDestroy(rec[b]);
        if (rev[b]) (void)hipEventDestroy(rev[b]);
      }
      if (start) (void)hipEventDestroy(start);
      for (int b = 0; b < 2; ++b) {
        if (seg[b]) (void)hipGraphExecDestroy(seg[b]);
        for (int a = 0; a < 2; ++a)
          if (sw[b][a]) (void)hipGraphExecDestroy(sw[b][a]);
      }
      if (s) (void)hipStreamDestroy(s);
    }
  };

  static int adjoint(mrlbm_ctx *c, const void *abar_final, void *mbar0, double *sbar) {
    const Plan &P = c->P;
    const int nsteps = c->adj_nsteps, K = c->adj_K;
    const AdjLayout L = adj_layout(P, nsteps, K);
    char *w = c->adj_ws;
    T *A = (T *)(w + L.A), *Hb = (T *)(w + L.Hb), *Gs = (T *)(w + L.Gs), *Go = (T *)(w + L.Go);
    double *spart = (double *)(w + L.spart);
    MomentMats<T> mm;
    {
      double M[81], Minv[81];
      moment_mats(c->p[0].scheme, c->p[0].lambda, M, Minv);
      for (int k = 0; k < 81; ++k) {
        mm.M[k] = (T)M[k];
        mm.Minv[k] = (T)Minv[k];
      }
    }
    // the levels whose ghost or internal list is non-empty in some mesh of the
    // recorded run (the list bounds the recorded forward kept)
    uint64_t gmask = 0, imask = 0;
    {
      std::vector<int> bounds((size_t)(nsteps + 1) * (L.lvl_b / sizeof(int)));
      HIPCHK(hipStreamSynchronize(c->stream));
      HIPCHK(hipMemcpy(bounds.data(), w + L.rec_lvl, L.lvl_b * ((size_t)nsteps + 1), hipMemcpyDeviceToHost));
      const int jmin = P.inst[0].jmin, jmax = P.inst[0].jmax;
      for (int n = 0; n <= nsteps; ++n) {
        const int *Lv = bounds.data() + (size_t)n * (L.lvl_b / sizeof(int));
        const int *Lg = Lv + CAT_GHOST * LVL_STRIDE, *Li = Lv + CAT_INTERNAL * LVL_STRIDE;
        for (int l = jmin; l <= jmax; ++l) {
          if (Lg[l + 1] > Lg[l]) gmask |= 1ull << l;
          if (Li[l + 1] > Li[l]) imask |= 1ull << l;
        }
      }
    }
    // The segments' recomputations run on the context stream and their reverse
    // sweeps on a second one, through two tapes: segment k-1 is recomputed
    // (tape (k-1) & 1) while segment k is swept (tape k & 1). Both are chains
    // of small launches on one instance, so they overlap on the GPU.
    SweepStream ss;
    HIPCHK(ss.init());
    const hipStream_t rs = ss.s;
    HIPCHK(hipEventRecord(ss.start, c->stream));  // the caller's work before this call
    HIPCHK(hipStreamWaitEvent(rs, ss.start, 0));
    zero(spart, sizeof(double) * 9 * ADJ_GRID, rs);
    (void)hipMemcpyAsync(A, abar_final, L.F_b <= P.rs * P.q * P.ctotal ? L.F_b : P.rs * P.q * P.ctotal,
                         hipMemcpyDeviceToDevice, rs);
    const size_t fbytes = P.rs * P.q * P.ctotal;
    auto tape_mesh = [&](int b, int j) {  // step j of tape b; j = -1: the segment's starting mesh
      if (j < 0)
        return Mesh{(const uint8_t *)(w + L.st_code + b * L.code_b), (const uint32_t *)(w + L.st_lists + b * L.lists_b),
                    (const int *)(w + L.st_lvl + b * L.lvl_b)};
      const size_t k = (size_t)b * K + j;
      return Mesh{(const uint8_t *)(w + L.tape_code + k * L.code_b),
                  (const uint32_t *)(w + L.tape_lists + k * L.lists_b), (const int *)(w + L.tape_lvl + k * L.lvl_b)};
    };
    auto tape_h = [&](int b, int j) { return (T *)(w + L.tape_h + ((size_t)b * K + j) * L.F_b); };
    auto seg_steps = [&](int seg) { return std::min(seg * K + K, nsteps) - seg * K; };
    auto segment_body = [&](int b, int steps) { return tape_segment(c, L, K, b, steps); };
    // A full segment (K steps) runs as a graph captured at its first use, one
    // per tape, when there are four full segments or more (each graph is then
    // replayed); the checkpoint is restored into the buffers of parity 0 first,
    // so every replay starts from the same buffers. Context stream.
    const bool graphs = c->use_graph && nsteps / K >= 4;
    int mK = 0, cK = 0;  // the buffer parities after a full segment
    auto recompute = [&](int seg) -> int {
      const int b = seg & 1, steps = seg_steps(seg);
      c->mcur = 0;
      c->cur = 0;
      (void)hipMemcpyAsync(c->code[0], w + L.ck_code + seg * L.code_b, P.ctotal, hipMemcpyDeviceToDevice, c->stream);
      (void)hipMemcpyAsync(c->F[0], w + L.ck_F + seg * L.F_b, fbytes, hipMemcpyDeviceToDevice, c->stream);
      int rc = MRLBM_OK;
      if (steps < K || !graphs) {
        rc = segment_body(b, steps);
      } else {
        if (!ss.seg[b]) {
          hipStream_t user = c->stream;
          const bool prof = c->profiling;
          c->stream = c->cap_stream;
          c->profiling = false;
          hipGraph_t graph = nullptr;
          hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed);
          rc = e == hipSuccess ? segment_body(b, steps) : MRLBM_ERR_HIP;
          if (e == hipSuccess) e = hipStreamEndCapture(c->cap_stream, &graph);
          c->stream = user;
          c->profiling = prof;
          if (rc == MRLBM_OK && e == hipSuccess) e = hipGraphInstantiate(&ss.seg[b], graph, nullptr, nullptr, 0);
          if (graph) (void)hipGraphDestroy(graph);
          if (rc == MRLBM_OK && e != hipSuccess) {
            ss.seg[b] = nullptr;
            rc = MRLBM_ERR_HIP;
          }
          mK = c->mcur;
          cK = c->cur;
        }
        if (rc == MRLBM_OK && hipGraphLaunch(ss.seg[b], c->stream) != hipSuccess) rc = MRLBM_ERR_HIP;
        c->mcur = mK;
        c->cur = cK;
      }
      if (rc) return rc;
      return hipEventRecord(ss.rec[b], c->stream) == hipSuccess ? MRLBM_OK : MRLBM_ERR_HIP;
    };
    // the reverse sweep over tape b (its last `steps` steps first)
    auto sweep_body = [&](int b, int steps, hipStream_t st) {
      for (int j = steps - 1; j >= 0; --j) {
        const Mesh mn = tape_mesh(b, j), mo = tape_mesh(b, j - 1);
        const uint32_t *leaves_n = mn.lists + (size_t)CAT_LEAF * P.ctotal;
        zero(Gs, fbytes, st);
        zero(Go, fbytes, st);
        k_adj_collide<DIM, SCHEME, T><<<ADJ_GRID, BLK, 0, st>>>(c->bt, I(c), mm, tape_h(b, j), A, Hb, leaves_n, mn.lvl,
                                                                spart);
        k_adj_transport_gather<DIM, SCHEME, T><<<dim3(ADJ_GATHER_GRID, NCAT, Q), BLK, 0, st>>>(
            c->bt, I(c), Hb, Gs, mn.code, mn.lists, mn.lvl, (const T *)c->W, P.nmax);
        k_adj_transport<DIM, SCHEME, T><<<ADJ_GRID, BLK, 0, st>>>(c->bt, I(c), Hb, Gs, mn.code, leaves_n, mn.lvl,
                                                                  (const T *)c->C);
        reconstruct_T(c, Gs, mn, st, gmask, imask);
        k_adj_transfer<DIM, Q, T><<<ADJ_GRID, BLK, 0, st>>>(c->bt, I(c), Gs, Go, mo.code, leaves_n, mn.lvl);
        reconstruct_T(c, Go, mo, st, gmask, imask);
        std::swap(A, Go);
      }
    };
    // The sweep of a recomputed segment on the second stream; a full segment
    // as a graph captured at its first use per tape and per buffer then in A
    // (the two buffers A and Go trade places every step).
    T *const A0 = A;
    auto sweep = [&](int seg) -> int {
      const int b = seg & 1, steps = seg_steps(seg);
      if (hipStreamWaitEvent(rs, ss.rec[b], 0) != hipSuccess) return MRLBM_ERR_HIP;
      if (steps < K || !graphs) {
        sweep_body(b, steps, rs);
      } else {
        hipGraphExec_t &g = ss.sw[b][A == A0 ? 0 : 1];
        if (!g) {  // capturing swaps A and Go as the steps do
          hipGraph_t graph = nullptr;
          hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed);
          if (e == hipSuccess) {
            sweep_body(b, steps, c->cap_stream);
            e = hipStreamEndCapture(c->cap_stream, &graph);
          }
          if (e == hipSuccess) e = hipGraphInstantiate(&g, graph, nullptr, nullptr, 0);
          if (graph) (void)hipGraphDestroy(graph);
          if (e != hipSuccess) {
            g = nullptr;
            return MRLBM_ERR_HIP;
          }
        } else if (steps & 1) {
          std::swap(A, Go);
        }
        if (hipGraphLaunch(g, rs) != hipSuccess) return MRLBM_ERR_HIP;
      }
      return hipEventRecord(ss.rev[b], rs) == hipSuccess ? MRLBM_OK : MRLBM_ERR_HIP;
    };
    // a run of one segment was taped by the recorded forward itself
    int rc = c->adj_taped ? (hipEventRecord(ss.rec[0], c->stream) == hipSuccess ? MRLBM_OK : MRLBM_ERR_HIP)
                          : recompute(L.nck - 1);
    for (int seg = L.nck - 1; seg >= 0 && !rc; --seg) {
      rc = sweep(seg);
      if (rc || seg == 0) break;
      // segment seg-1 overwrites the tape that the sweep of segment seg+1 read
      if (seg + 1 < L.nck && hipStreamWaitEvent(c->stream, ss.rev[(seg + 1) & 1], 0) != hipSuccess) rc = MRLBM_ERR_HIP;
      if (!rc) rc = recompute(seg - 1);
    }
    if (rc) return rc;
    // the recorded run started from the full finest mesh of checkpoint 0
    const long long nf = 1ll << (DIM * P.inst[0].jmax);
    k_adj_init<DIM, SCHEME, T><<<grid_cap((nf + BLK - 1) / BLK, DENSE_GRID), BLK, 0, rs>>>(
        I(c), mm, (const T *)(w + L.ck_F), A, (T *)mbar0);
    HIPCHK(hipStreamSynchronize(rs));
    std::vector<double> part(9 * ADJ_GRID);
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(part.data(), spart, sizeof(double) * part.size(), hipMemcpyDeviceToHost));
    for (int k = 0; k < 9; ++k) {
      double acc = 0.0;
      for (int b = 0; b < ADJ_GRID; ++b) acc += part[b * 9 + k];
      sbar[k] = acc;
    }
    return hipPeekAtLastError() == hipSuccess ? MRLBM_OK : MRLBM_ERR_HIP;
  }

  // ------------------------------------------------------------- autotuning
  static int time_dry_steps(mrlbm_ctx *c, int reps, float *ms) { return time_dry_steps_impl<Engine>(c, reps, ms); }

  static int upload_inst(mrlbm_ctx *c) {
    std::vector<Inst<T>> v(c->P.B);
    for (int i = 0; i < c->P.B; ++i) {
      const Inst<double> &s = c->P.inst[i];
      Inst<T> &d = v[i];
      std::memset(&d, 0, sizeof d);
      d.jmin = s.jmin;
      d.jmax = s.jmax;
      d.cbase = s.cbase;
      d.total = s.total;
      for (int l = 0; l < LVL_STRIDE; ++l) {
        d.loff[l] = s.loff[l];
        d.bstart[l] = s.bstart[l];
        d.eps_l[l] = (T)s.eps_l[l];
        d.ref_l[l] = (T)s.ref_l[l];
      }
      d.sc.lam = (T)s.sc.lam;
      d.sc.inv_lam = (T)s.sc.inv_lam;
      d.sc.eq = (T)s.sc.eq;
      for (int k = 0; k < 16; ++k) d.sc.s[k] = (T)s.sc.s[k];
      for (int k = 0; k < 3; ++k) d.sc.vel[k] = (T)s.sc.vel[k];
      d.walls = s.walls;
      for (int k = 0; k < 4; ++k) d.bck[k] = s.bck[k];
      d.gamma = s.gamma;
      d.metric = s.metric;
    }
    HIPCHK(hipMemcpy(c->inst, v.data(), sizeof(Inst<T>) * v.size(), hipMemcpyHostToDevice));
    return MRLBM_OK;
  }
};

// The three-dimensional engine (D3Q6, gamma = 1, periodic): the same step of
// Algorithm 1 with the kernels of mr_kernels3d.h. Per step: the old mesh's
// projections (fine to coarse) and ghost predictions (coarse to fine), the
// details and their flags, thresholding, ancestor closure, neighbour addition
// and refinement, grading, the new codes and ghost marks, the lists, the
// transfer into the cells outside the old mesh, the new mesh's reconstruction,
// then transport + collision into the other value buffer.
template <typename T, int GAM>
struct Engine<3, MRLBM_D3Q6, T, GAM> {
  using Real = T;
  static constexpr int DIM = 3, Q = 6;

  static const Inst<T> *I(mrlbm_ctx *c) { return (const Inst<T> *)c->inst; }
  static int transport_kernels(const mrlbm_ctx *) { return 1; }
  static unsigned list_blocks(mrlbm_ctx *c) {  // four chunks of 64 items per block
    return list_grid((c->P.ctotal + 4 * CHUNK - 1) / (4 * CHUNK), c->grid_all);
  }
  static unsigned level_list_blocks(mrlbm_ctx *c, int l) {
    long long n = 0;
    for (int i = 0; i < c->P.B; ++i)
      if (l >= c->P.jmin && l <= c->P.inst[i].jmax) n += ((1ll << (3 * l)) + CHUNK - 1) / CHUNK;
    return list_grid((n + 3) / 4, c->grid_level);
  }
  static dim3 level_grid(mrlbm_ctx *c, int l) {  // CPT cells per thread
    const long long n = 1ll << (3 * l);
    return dim3((unsigned)((n + BLK * d3::CPT - 1) / (BLK * d3::CPT)), (unsigned)c->P.B);
  }
  static dim3 level_word_grid(mrlbm_ctx *c, int l) {  // one word of eight cells per thread
    const long long n = 1ll << (3 * l);
    return dim3((unsigned)((n / 8 + BLK - 1) / BLK), (unsigned)c->P.B);
  }

  // Lists of mesh m (every level active: the 3D passes keep no activity history).
  static void compact(mrlbm_ctx *c, int m) {
    const Plan &P = c->P;
    k_fill_u32<<<1, BLK, 0, c->stream>>>((uint32_t *)c->act, (long long)ACT * P.B, (uint32_t)ACT_ALL);
    k_compact_count<3, T><<<P.nblocks, BLK, 0, c->stream>>>(c->bt, I(c), c->binfo, c->code[m], c->bcnt, P.nblocks,
                                                             c->act, c->ne[m]);
    k_compact_scan<T><<<P.B, 1024, 0, c->stream>>>(c->bt, I(c), c->cbp, c->bcnt, c->boff, c->lvl[m], P.nblocks,
                                                   c->act, c->ne[m]);
    k_compact_scatter<3, Q, T, 1><<<P.nblocks, BLK, 0, c->stream>>>(c->bt, I(c), c->binfo, c->code[m], c->boff,
                                                                     c->lists[m], P.nblocks, nullptr, nullptr,
                                                                     nullptr, c->act);
  }

  // Levels up to lc of every chain share one launch (one block per instance),
  // finer levels take a launch each: levels of at most 4096 cells with 32
  // instances or more, else of at most 512 (a larger level spreads better over
  // the blocks of a launch of its own).
  static int coarse_cap(const mrlbm_ctx *c) { return std::min(c->P.B >= 32 ? 4 : 3, c->P.maxJ); }

  // Codes of the membership bytes tnew into code[m], the ghost marks, the lists.
  static void classify(mrlbm_ctx *c, int m) {
    const Plan &P = c->P;
    const int lc = coarse_cap(c);
    uint8_t *gm = c->mark;  // ghost flags (the 3D engine keeps no reconstruction marks)
    d3::k3_classify<T><<<P.nblocks, BLK, 0, c->stream>>>(I(c), c->binfo, c->tnew, c->code[m], gm);
    d3::k3_ghost_leaf<T><<<P.nblocks, BLK, 0, c->stream>>>(I(c), c->binfo, c->code[m], gm);
    for (int l = P.maxJ; l > std::max(P.jmin, lc); --l)
      d3::k3_ghost_up<T><<<level_word_grid(c, l), BLK, 0, c->stream>>>(I(c), c->code[m], gm, l);
    if (lc > P.jmin) d3::k3_dense_coarse<T, 2><<<P.B, CBLK, 0, c->stream>>>(I(c), gm, c->code[m], lc);
    d3::k3_ghost_codes<T><<<P.nblocks, BLK, 0, c->stream>>>(I(c), c->binfo, c->code[m], gm);
    compact(c, m);
  }

  // Reconstruction of mesh m in F: projections fine to coarse, ghost
  // predictions coarse to fine.
  static void reconstruct(mrlbm_ctx *c, T *F, int m) {
    const Plan &P = c->P;
    const int lc = coarse_cap(c);
    const uint32_t *li = c->lists[m] + (size_t)CAT_INTERNAL * P.ctotal;
    const uint32_t *lg = c->lists[m] + (size_t)CAT_GHOST * P.ctotal;
    for (int l = P.maxJ - 1; l > lc; --l)
      d3::k3_project<T><<<level_list_blocks(c, l), BLK, 0, c->stream>>>(c->bt, I(c), F, li, c->lvl[m], l);
    d3::k3_project_coarse<T><<<P.B, CBLK, 0, c->stream>>>(I(c), F, li, c->lvl[m], lc);
    if (lc > P.jmin) d3::k3_ghost_coarse<T><<<P.B, CBLK, 0, c->stream>>>(I(c), F, lg, c->lvl[m], lc);
    for (int l = std::max(P.jmin, lc) + 1; l <= P.maxJ; ++l)
      d3::k3_ghost<T><<<level_list_blocks(c, l), BLK, 0, c->stream>>>(c->bt, I(c), F, lg, c->lvl[m], l);
  }

  static int adapt(mrlbm_ctx *c) {
    const Plan &P = c->P;
    const int mo = c->mcur, mn = 1 - c->mcur;
    T *Fc = (T *)c->F[c->cur];
    phase_mark(c, PH_ADAPT, true);
    reconstruct(c, Fc, mo);  // the details read the tree, the transfer the ghosts
    const uint32_t *li = c->lists[mo] + (size_t)CAT_INTERNAL * P.ctotal;
    auto det = P.metric_mode == 0 ? d3::k3_details<T, 0> : P.metric_mode == 1 ? d3::k3_details<T, 1> : d3::k3_details<T, 2>;
    det<<<list_blocks(c), BLK, 0, c->stream>>>(c->bt, I(c), Fc, li, c->lvl[mo], c->refg);
    d3::k3_keep<T><<<P.nblocks, BLK, 0, c->stream>>>(I(c), c->binfo, c->code[mo], c->refg, c->keep, c->tnew);
    const int lc = coarse_cap(c);
    for (int l = P.maxJ; l >= std::max(P.jmin + 2, lc + 1); --l)
      d3::k3_closure<T><<<level_word_grid(c, l), BLK, 0, c->stream>>>(I(c), c->keep, l);
    if (lc >= P.jmin + 2) d3::k3_dense_coarse<T, 0><<<P.B, CBLK, 0, c->stream>>>(I(c), c->keep, nullptr, lc);
    d3::k3_enlarge<T><<<P.nblocks, BLK, 0, c->stream>>>(I(c), c->binfo, c->keep, c->refg, c->tnew);
    for (int l = P.maxJ; l >= std::max(P.jmin + 1, lc + 1); --l)
      d3::k3_grade<T><<<level_word_grid(c, l), BLK, 0, c->stream>>>(I(c), c->tnew, l);
    if (lc >= P.jmin + 1) d3::k3_dense_coarse<T, 1><<<P.B, CBLK, 0, c->stream>>>(I(c), c->tnew, nullptr, lc);
    classify(c, mn);
    // the transfer: new leaves outside the old mesh are predicted from their
    // parent's level, whose stencil the old mesh's ghosts cover
    d3::k3_transfer<T><<<list_blocks(c), BLK, 0, c->stream>>>(c->bt, I(c), Fc,
                                                              c->lists[mn] + (size_t)CAT_LEAF * P.ctotal, c->lvl[mn],
                                                              c->code[mo]);
    phase_mark(c, PH_ADAPT, false);
    c->mcur = mn;
    return hipPeekAtLastError() == hipSuccess ? MRLBM_OK : MRLBM_ERR_HIP;
  }

  static int transport(mrlbm_ctx *c, T * = nullptr) {
    phase_mark(c, PH_RECON, true);
    reconstruct(c, (T *)c->F[c->cur], c->mcur);
    phase_mark(c, PH_RECON, false);
    return transport_kernel(c);
  }

  static int transport_kernel(mrlbm_ctx *c) {
    const Plan &P = c->P;
    const int m = c->mcur;
    phase_mark(c, PH_TRANSPORT, true);
    d3::k3_transport_collide<T><<<list_blocks(c), BLK, 0, c->stream>>>(
        c->bt, I(c), (const T *)c->F[c->cur], (T *)c->F[1 - c->cur], c->code[m],
        c->lists[m] + (size_t)CAT_LEAF * P.ctotal, c->lvl[m], (const T *)c->W, (const T *)c->C, c->cnt);
    phase_mark(c, PH_TRANSPORT, false);
    c->cur = 1 - c->cur;
    return hipPeekAtLastError() == hipSuccess ? MRLBM_OK : MRLBM_ERR_HIP;
  }

  static int step_graph(mrlbm_ctx *c) { return step_graph_impl<Engine>(c); }
  static int time_dry_steps(mrlbm_ctx *c, int reps, float *ms) { return time_dry_steps_impl<Engine>(c, reps, ms); }

  static int init(mrlbm_ctx *c, int i, const void *mom) {
    const Plan &P = c->P;
    T *F = (T *)c->F[c->cur];
    const long long nf = 1ll << (3 * P.inst[i].jmax);
    k_init_equilibrium<3, MRLBM_D3Q6, T><<<grid_cap((nf + BLK - 1) / BLK, DENSE_GRID), BLK, 0, c->stream>>>(
        I(c), i, F, (const T *)mom);
    k_full_tree<T><<<grid_cap((P.inst[i].total + BLK - 1) / BLK, DENSE_GRID), BLK, 0, c->stream>>>(I(c), i,
                                                                                                  c->code[c->mcur]);
    compact(c, c->mcur);
    c->has_state[i] = 1;
    c->recon_reuse = false;
    return hipPeekAtLastError() == hipSuccess ? MRLBM_OK : MRLBM_ERR_HIP;
  }

  static int mass(mrlbm_ctx *c) {
    k_mass_partial<3, Q, T><<<dim3(RED_BLOCKS, c->P.B), BLK, 0, c->stream>>>(
        c->bt, I(c), (const T *)c->F[c->cur], c->lists[c->mcur] + (size_t)CAT_LEAF * c->P.ctotal, c->lvl[c->mcur],
        c->red, c->bad);
    return MRLBM_OK;
  }

  static int exportl(mrlbm_ctx *c, int i, uint32_t *cells, void *vals) {
    k_export<3, Q, T><<<grid_cap((c->P.inst[i].total + BLK - 1) / BLK, DENSE_GRID), BLK, 0, c->stream>>>(
        I(c), i, (const T *)c->F[c->cur], c->lists[c->mcur] + (size_t)CAT_LEAF * c->P.ctotal, c->lvl[c->mcur], cells,
        (T *)vals);
    return MRLBM_OK;
  }

  static int leaf_fields(mrlbm_ctx *c, int i, int what, void *out) {
    const long long n = c->P.inst[i].total;
    const unsigned g = grid_cap((n + BLK - 1) / BLK, DENSE_GRID);
    const uint32_t *lf = c->lists[c->mcur] + (size_t)CAT_LEAF * c->P.ctotal;
    if (what == MRLBM_FIELD_MOMENTS)
      k_moments<3, MRLBM_D3Q6, T><<<g, BLK, 0, c->stream>>>(I(c), i, (const T *)c->F[c->cur], lf, c->lvl[c->mcur],
                                                             (T *)out);
    else
      k_export<3, Q, T><<<g, BLK, 0, c->stream>>>(I(c), i, (const T *)c->F[c->cur], lf, c->lvl[c->mcur],
                                                  what == MRLBM_FIELD_LEAF_TABLE ? (uint32_t *)out : nullptr,
                                                  what == MRLBM_FIELD_POPULATIONS ? (T *)out : nullptr);
    return hipPeekAtLastError() == hipSuccess ? MRLBM_OK : MRLBM_ERR_HIP;
  }

  // The double-hat reconstruction on the finest level: the mesh's
  // reconstruction, then every other cell outside the tree, level by level.
  static int finest(mrlbm_ctx *c, int i, void *out) {
    const Inst<double> &In = c->P.inst[i];
    T *F = (T *)c->F[c->cur];
    reconstruct(c, F, c->mcur);
    for (int l = In.jmin + 1; l <= In.jmax; ++l)
      d3::k3_predict_outside<T><<<level_grid(c, l), BLK, 0, c->stream>>>(I(c), F, c->code[c->mcur], l);
    const size_t bytes = sizeof(T) * Q * ((size_t)1 << (3 * In.jmax));
    HIPCHK(hipMemcpyAsync(out, F + (size_t)Q * In.loff[In.jmax], bytes, hipMemcpyDeviceToDevice, c->stream));
    return hipPeekAtLastError() == hipSuccess ? MRLBM_OK : MRLBM_ERR_HIP;
  }

  static int frozen(mrlbm_ctx *c, const uint8_t *trees) {
    const Plan &P = c->P;
    const int mo = c->mcur, mn = 1 - mo;
    T *Fc = (T *)c->F[c->cur];
    reconstruct(c, Fc, mo);
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(c->tnew, trees, P.ctotal, hipMemcpyHostToDevice));
    classify(c, mn);
    d3::k3_transfer<T><<<list_blocks(c), BLK, 0, c->stream>>>(c->bt, I(c), Fc,
                                                              c->lists[mn] + (size_t)CAT_LEAF * P.ctotal, c->lvl[mn],
                                                              c->code[mo]);
    c->mcur = mn;
    return transport(c);
  }

  static int upload_inst(mrlbm_ctx *c) { return Engine<2, MRLBM_D2Q9, T, 1>::upload_inst(c); }
  static int record(mrlbm_ctx *, int, int) { return MRLBM_ERR_INVALID; }
  static int adjoint(mrlbm_ctx *, const void *, void *, double *) { return MRLBM_ERR_INVALID; }
};

template <template <int, int, typename, int> class Op, int G, typename... A>
int dispatch_g(mrlbm_ctx *c, A... a) {
  const bool dbl = c->p[0].precision == 8;
  switch (c->p[0].scheme) {
    case MRLBM_D1Q2: return dbl ? Op<1, 1, double, G>::run(c, a...) : Op<1, 1, float, G>::run(c, a...);
    case MRLBM_D1Q3: return dbl ? Op<1, 2, double, G>::run(c, a...) : Op<1, 2, float, G>::run(c, a...);
    case MRLBM_D2Q4_EULER: return dbl ? Op<2, 4, double, G>::run(c, a...) : Op<2, 4, float, G>::run(c, a...);
    case MRLBM_D3Q6:
      if constexpr (G == 1) return dbl ? Op<3, 5, double, 1>::run(c, a...) : Op<3, 5, float, 1>::run(c, a...);
      else return MRLBM_ERR_INVALID;  // validation admits gamma = 1 only
    default: return dbl ? Op<2, 3, double, G>::run(c, a...) : Op<2, 3, float, G>::run(c, a...);
  }
}
template <template <int, int, typename, int> class Op, typename... A>
int dispatch(mrlbm_ctx *c, A... a) {
  return c->P.gamma > 1 ? dispatch_g<Op, 0>(c, a...) : dispatch_g<Op, 1>(c, a...);
}
template <int D, int S, typename T, int G>
struct AdaptOp { static int run(mrlbm_ctx *c) { return Engine<D, S, T, G>::adapt(c); } };
template <int D, int S, typename T, int G>
struct TransportOp { static int run(mrlbm_ctx *c) { return Engine<D, S, T, G>::transport(c); } };
template <int D, int S, typename T, int G>
struct DryOp { static int run(mrlbm_ctx *c, int reps, float *ms) { return Engine<D, S, T, G>::time_dry_steps(c, reps, ms); } };
template <int D, int S, typename T, int G>
struct StepGraphOp { static int run(mrlbm_ctx *c) { return Engine<D, S, T, G>::step_graph(c); } };
template <int D, int S, typename T, int G>
struct InitOp { static int run(mrlbm_ctx *c, int i, const void *m) { return Engine<D, S, T, G>::init(c, i, m); } };
template <int D, int S, typename T, int G>
struct ClassifyOp { static int run(mrlbm_ctx *c, int m) { Engine<D, S, T, G>::classify(c, m); return MRLBM_OK; } };
template <int D, int S, typename T, int G>
struct MassOp { static int run(mrlbm_ctx *c) { return Engine<D, S, T, G>::mass(c); } };
template <int D, int S, typename T, int G>
struct ExportOp {
  static int run(mrlbm_ctx *c, int i, uint32_t *cells, void *vals) { return Engine<D, S, T, G>::exportl(c, i, cells, vals); }
};
template <int D, int S, typename T, int G>
struct LeafFieldsOp {
  static int run(mrlbm_ctx *c, int i, int what, void *out) { return Engine<D, S, T, G>::leaf_fields(c, i, what, out); }
};
template <int D, int S, typename T, int G>
struct FinestOp { static int run(mrlbm_ctx *c, int i, void *out) { return Engine<D, S, T, G>::finest(c, i, out); } };
template <int D, int S, typename T, int G>
struct FrozenOp { static int run(mrlbm_ctx *c, const uint8_t *t) { return Engine<D, S, T, G>::frozen(c, t); } };
template <int D, int S, typename T, int G>
struct UploadOp { static int run(mrlbm_ctx *c) { return Engine<D, S, T, G>::upload_inst(c); } };
// The adjoint covers gamma = 1 and the schemes D1Q2, D1Q3 and D2Q9.
template <int D, int S, typename T, int G>
struct RecordOp {
  static int run(mrlbm_ctx *c, int n, int K) {
    if constexpr (G == 1 && S <= MRLBM_D2Q9) return Engine<D, S, T, G>::record(c, n, K);
    else return MRLBM_ERR_INVALID;
  }
};
template <int D, int S, typename T, int G>
struct AdjointOp {
  static int run(mrlbm_ctx *c, const void *a, void *mb, double *sb) {
    if constexpr (G == 1 && S <= MRLBM_D2Q9) return Engine<D, S, T, G>::adjoint(c, a, mb, sb);
    else return MRLBM_ERR_INVALID;
  }
};

// Host check of a 0/1 tree of instance i: level jmin complete, sibling groups
// complete, every tree cell's parent and prediction stencil present.
bool tree_is_graded(const mrlbm_ctx *c, int inst, const uint8_t *t) {
  const Inst<double> &I = c->P.inst[inst];
  const int d = c->P.dim;
  auto at = [&](int l, long long k) { return t[I.loff[l] - I.cbase + k]; };
  // cell (x, y, z) of level l (coordinates beyond the dimension are 0)
  auto idx = [&](int l, long long x, long long y, long long z) { return x + ((y + (z << l)) << l); };
  for (long long k = 0; k < (1ll << (d * I.jmin)); ++k)
    if (!at(I.jmin, k)) return false;
  const int g = I.gamma;  // grading box of half-width gamma
  const int gy = d >= 2 ? g : 0, gz = d == 3 ? g : 0;
  for (int l = I.jmin + 1; l <= I.jmax; ++l) {
    const int np = 1 << (l - 1);
    for (int pz = 0; pz < (d == 3 ? np : 1); ++pz)
      for (int py = 0; py < (d >= 2 ? np : 1); ++py)
        for (int px = 0; px < np; ++px) {
          int cnt = 0;
          for (int dz = 0; dz < (d == 3 ? 2 : 1); ++dz)
            for (int dy = 0; dy < (d >= 2 ? 2 : 1); ++dy)
              for (int dx = 0; dx < 2; ++dx) cnt += at(l, idx(l, 2 * px + dx, 2 * py + dy, 2 * pz + dz)) ? 1 : 0;
          if (cnt == 0) continue;
          if (cnt != (1 << d)) return false;
          for (int e = -gz; e <= gz; ++e)
            for (int b = -gy; b <= gy; ++b)
              for (int a = -g; a <= g; ++a) {
                if (((I.walls & 1) && (px + a < 0 || px + a >= np)) || ((I.walls & 2) && (py + b < 0 || py + b >= np)))
                  continue;  // no cell beyond a wall
                const int x = (px + a) & (np - 1), y = (py + b) & (np - 1), z = (pz + e) & (np - 1);
                if (!at(l - 1, idx(l - 1, x, y, z))) return false;
              }
        }
  }
  return true;
}

// Host check that every cell of the new tree t outside the old tree `old`
// (membership bytes of instance inst) has its parent in the old tree: the
// adaptation refines by at most one level per step, which the in-place
// transfer relies on (a created cell is predicted from its parent's level).
bool refines_by_one(const mrlbm_ctx *c, int inst, const uint8_t *old, const uint8_t *t) {
  const Inst<double> &I = c->P.inst[inst];
  const int d = c->P.dim;
  for (int l = I.jmin + 1; l <= I.jmax; ++l) {
    const long long n = 1ll << (d * l), o = I.loff[l] - I.cbase, op = I.loff[l - 1] - I.cbase;
    const long long m = (1ll << l) - 1;
    for (long long k = 0; k < n; ++k) {
      if (!t[o + k] || old[o + k]) continue;
      const long long x = k & m, y = (k >> l) & m, z = k >> (2 * l);
      const long long pk = (x >> 1) + (((y >> 1) + ((z >> 1) << (l - 1))) << (l - 1));
      if (!old[op + pk]) return false;
    }
  }
  return true;
}

__global__ void k_membership(const uint8_t *__restrict__ code, uint8_t *__restrict__ t, long long n) {
  for (long long i = blockIdx.x * (long long)BLK + threadIdx.x; i < n; i += (long long)gridDim.x * BLK)
    t[i] = code[i] >= C_INTERNAL ? 1 : 0;
}

bool bad_instance(const mrlbm_ctx *c, int i) { return !c || i < 0 || i >= c->P.B; }

}  // namespace

// ====================================================================== C-ABI

namespace {
// Workspace of the contexts made by mrlbm_create_static: one per GPU, held
// from the library's load on that GPU until the process ends. Host code never
// passes the array's name to a kernel or a copy (on the host it is only a
// stand-in for the symbol); it uses the device address that
// hipGetSymbolAddress returns, looked up once per device.
constexpr size_t STATIC_WS_BYTES = (size_t)MRLBM_STATIC_WORKSPACE_BYTES;
static __device__ __align__(256) unsigned char scratch[STATIC_WS_BYTES];
constexpr int STATIC_MAX_DEVICES = 64;
std::mutex static_mutex;
void *static_ptr[STATIC_MAX_DEVICES];     // device address of `scratch` on each device (null until looked up)
bool static_busy[STATIC_MAX_DEVICES];     // a live static context uses that device's array

int create_ctx(const mrlbm_params *p, int batch, void *workspace, size_t ws_bytes, void *stream, int static_dev,
               mrlbm_ctx **out);
}  // namespace

extern "C" {

int mrlbm_workspace_size(const mrlbm_params *p, int batch, size_t *bytes) {
  if (!bytes) return MRLBM_ERR_INVALID;
  const int rc = validate(p, batch);
  if (rc) return rc;
  Plan P;
  make_plan(p, batch, P);
  *bytes = P.bytes;
  return MRLBM_OK;
}


int mrlbm_create(const mrlbm_params *p, int batch, void *workspace, size_t ws_bytes, void *stream, mrlbm_ctx **out) {
  if (!out || !workspace) return MRLBM_ERR_INVALID;
  return create_ctx(p, batch, workspace, ws_bytes, stream, -1, out);
}

int mrlbm_create_static(const mrlbm_params *p, int batch, void *stream, mrlbm_ctx **out) {
  if (!out) return MRLBM_ERR_INVALID;
  *out = nullptr;
  int rc = validate(p, batch);
  if (rc) return rc;
  Plan P;
  make_plan(p, batch, P);
  if (P.bytes > STATIC_WS_BYTES) return MRLBM_ERR_CAPACITY;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MRLBM_ERR_HIP;
  if (dev < 0 || dev >= STATIC_MAX_DEVICES) return MRLBM_ERR_INVALID;
  std::lock_guard<std::mutex> lock(static_mutex);
  if (static_busy[dev]) return MRLBM_ERR_STATE;
  if (!static_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return MRLBM_ERR_HIP;
    static_ptr[dev] = ptr;
  }
  rc = create_ctx(p, batch, static_ptr[dev], STATIC_WS_BYTES, stream, dev, out);
  if (rc == MRLBM_OK) static_busy[dev] = true;
  return rc;
}

}  // extern "C"

namespace {
int create_ctx(const mrlbm_params *p, int batch, void *workspace, size_t ws_bytes, void *stream, int static_dev,
               mrlbm_ctx **out) {
  *out = nullptr;
  const int rc = validate(p, batch);
  if (rc) return rc;
  mrlbm_ctx *c = new (std::nothrow) mrlbm_ctx();
  if (!c) return MRLBM_ERR_INVALID;
  c->p.assign(p, p + batch);
  make_plan(p, batch, c->P);
  const Plan &P = c->P;
  c->static_dev = static_dev;
  if (ws_bytes < P.bytes) {
    delete c;
    return MRLBM_ERR_CAPACITY;
  }
  c->bt.B = P.B;
  c->bt.dim = P.dim;
  c->bt.q = P.q;
  c->bt.jmin = P.jmin;
  c->bt.maxJ = P.maxJ;
  c->bt.ctotal = P.ctotal;
  c->stream = (hipStream_t)stream;
  char *b = (char *)(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
  for (int k = 0; k < 2; ++k) {
    c->F[k] = b + P.off_F[k];
    c->code[k] = (uint8_t *)(b + P.off_code[k]);
    c->lists[k] = (uint32_t *)(b + P.off_lists[k]);
    c->lvl[k] = (int *)(b + P.off_lvl[k]);
  }
  c->keep = (uint8_t *)(b + P.off_keep);
  c->refg = (uint8_t *)(b + P.off_refg);
  c->tnew = (uint8_t *)(b + P.off_tnew);
  c->mark = (uint8_t *)(b + P.off_mark);
  c->act = (int *)(b + P.off_act);
  c->sync = (unsigned *)(b + P.off_sync);
  for (int k = 0; k < 2; ++k) c->ne[k] = (int *)(b + P.off_ne[k]);
  c->bcnt = (int *)(b + P.off_bcnt);
  c->boff = (int *)(b + P.off_boff);
  c->W = b + P.off_W;
  c->C = b + P.off_C;
  c->Wb = b + P.off_Wb;
  c->Cb = b + P.off_Cb;
  c->Nb = b + P.off_Nb;
  c->red = (double *)(b + P.off_red);
  c->bad = (int *)(b + P.off_bad);
  c->cnt = (unsigned long long *)(b + P.off_cnt);
  c->inst = b + P.off_inst;
  c->cb = (long long *)(b + P.off_cb);
  c->cbp = (int *)(b + P.off_cbp);
  c->dtab = (int *)(b + P.off_dtab);
  c->binfo = (uint32_t *)(b + P.off_binfo);
  c->dinfo = (uint32_t *)(b + P.off_dinfo);
  c->wband = (uint32_t *)(b + P.off_wband);
  c->gtile = (uint32_t *)(b + P.off_gtile);
  c->cur = 0;
  c->mcur = 0;
  c->has_state.assign(P.B, 0);
  c->profiling = false;
  c->timing_period = TIMING_PERIOD;
  c->graph_steps = 0;
  c->ev_used = 0;
  c->adj_ws = nullptr;
  c->adj_nsteps = 0;
  c->adj_K = 0;
  c->adj_taped = false;
  c->use_graph = static_dev < 0;  // a static context creates no capture stream: kernels launched one by one
  c->cap_stream = nullptr;
  for (auto &row : c->graph)
    for (auto &g : row) g = nullptr;
  for (auto &g : c->timed_src) g = nullptr;
  c->ev_placeholder = nullptr;
  if (static_dev < 0) {
    if (timing_event(&c->ev_placeholder) != hipSuccess) {
      delete c;
      return MRLBM_ERR_HIP;
    }
    if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
      (void)mrlbm_destroy(c);
      return MRLBM_ERR_HIP;
    }
  }
  c->transport_variant = 0;
  c->pair_links = false;
  c->grid_all = LIST_GRID_ALL;
  c->grid_level = LIST_GRID_LEVEL;
  // transport weight tables, rounded once to the working precision
  const int q = P.q, d = P.dim, ws = d == 2 ? 25 : 5, cs = d == 2 ? 36 : 6;
  const int nn = std::max(1, P.nmax);
  // (gamma = 1: the fast kernels' periodic tables; unused for gamma > 1)
  std::vector<double> W((size_t)nn * q * ws, 0.0), C((size_t)nn * q * cs, 0.0), w25(q * 25), c36(q * 36);
  ImpulseSums imp1(1);
  const bool d3q6 = p[0].scheme == MRLBM_D3Q6;  // the D1Q2 rows of the velocity's sign (see mr_kernels3d.h)
  for (int n = 1; n <= P.nmax && P.gamma == 1; ++n) {
    transport_tables(d3q6 ? MRLBM_D1Q2 : p[0].scheme, n, w25.data(), c36.data(), 0, 0, nullptr, 1, &imp1);
    for (int h = 0; h < q; ++h) {
      const int hs = d3q6 ? (h & 1) : h;
      for (int k = 0; k < ws; ++k) W[((size_t)(n - 1) * q + h) * ws + k] = d == 2 ? w25[hs * 25 + k] : w25[hs * 25 + 10 + k];
      for (int k = 0; k < cs; ++k) C[((size_t)(n - 1) * q + h) * cs + k] = d == 2 ? c36[hs * 36 + k] : c36[hs * 36 + 12 + k];
    }
  }
  // the general path's tables, per wall case (index wx + 3 wy; case 0: no wall
  // touched, the periodic tables), over the boxes of half-width 2 gamma
  const int g = P.gamma, R = 2 * g, WW = 2 * R + 1, CW = 2 * R + 2;
  const int wsg = wide_ws(d, g), csg = wide_cs(d, g);
  std::vector<double> Wb((size_t)nn * 9 * q * wsg, 0.0), Cb((size_t)nn * 9 * q * csg, 0.0), Nb((size_t)nn * 9 * q * 2, 0.0);
  std::vector<double> wg((size_t)q * WW * WW), cg((size_t)q * CW * CW), n2(q * 2);
  ImpulseSums impg(g);
  for (int n = 1; n <= P.nmax && (P.any_walls || g > 1); ++n)
    for (int wc = 0; wc < (d == 2 ? 9 : 3); ++wc) {
      transport_tables(p[0].scheme, n, wg.data(), cg.data(), wc % 3, wc / 3, n2.data(), g, &impg);
      for (int h = 0; h < q; ++h) {
        const size_t r = ((size_t)(n - 1) * 9 + wc) * q + h;
        // a 1D scheme keeps the middle row
        for (int k = 0; k < wsg; ++k) Wb[r * wsg + k] = wg[(size_t)h * WW * WW + (d == 2 ? k : R * WW + k)];
        for (int k = 0; k < csg; ++k) Cb[r * csg + k] = cg[(size_t)h * CW * CW + (d == 2 ? k : R * CW + k)];
        Nb[r * 2] = n2[2 * h];
        Nb[r * 2 + 1] = n2[2 * h + 1];
      }
    }
  hipError_t e = hipSuccess;
  auto put = [&](void *dst, const std::vector<double> &v) {
    if (e != hipSuccess) return;
    if (P.rs == 8) {
      e = hipMemcpy(dst, v.data(), v.size() * 8, hipMemcpyHostToDevice);
    } else {
      const std::vector<float> f(v.begin(), v.end());
      e = hipMemcpy(dst, f.data(), f.size() * 4, hipMemcpyHostToDevice);
    }
  };
  put(c->W, W);
  put(c->C, C);
  put(c->Wb, Wb);
  put(c->Cb, Cb);
  put(c->Nb, Nb);
  if (e == hipSuccess) e = hipMemcpy(c->cb, P.cb.data(), sizeof(long long) * P.cb.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->cbp, P.cbp.data(), sizeof(int) * P.cbp.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->dtab, P.dtab.data(), sizeof(int) * P.dtab.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->binfo, P.binfo.data(), sizeof(uint32_t) * P.binfo.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !P.dinfo.empty())
    e = hipMemcpy(c->dinfo, P.dinfo.data(), sizeof(uint32_t) * P.dinfo.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !P.wband.empty())
    e = hipMemcpy(c->wband, P.wband.data(), sizeof(uint32_t) * P.wband.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !P.gtile.empty())
    e = hipMemcpy(c->gtile, P.gtile.data(), sizeof(uint32_t) * P.gtile.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(c->cnt, 0, 4 * sizeof(unsigned long long));
  for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipMemset(c->code[k], 0, P.ctotal);
  if (e == hipSuccess) e = hipMemset(c->keep, 0, P.ctotal);
  if (e == hipSuccess) e = hipMemset(c->refg, 0, P.ctotal);
  if (e == hipSuccess) e = hipMemset(c->mark, 0, P.ctotal);
  if (e == hipSuccess) {
    const unsigned sync0[4] = {0u, 0u, PAIR_WAIT_BUDGET, 0u};
    e = hipMemcpy(c->sync, sync0, sizeof sync0, hipMemcpyHostToDevice);
  }
  for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipMemset(c->ne[k], 0, sizeof(int) * NCAT * LVL_STRIDE);
  if (e == hipSuccess) {  // every level active until two meshes were built
    const std::vector<int> all(ACT * P.B, ACT_ALL);
    e = hipMemcpy(c->act, all.data(), sizeof(int) * all.size(), hipMemcpyHostToDevice);
  }
  // Value buffers start at zero: cells outside the mesh hold scratch that then
  // depends only on the sequence of calls.
  for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipMemset(c->F[k], 0, P.rs * P.q * P.ctotal);
  if (e != hipSuccess || dispatch<UploadOp>(c) != MRLBM_OK) {
    c->static_dev = -1;  // the caller of a static create still holds the array's lock and flag
    (void)mrlbm_destroy(c);
    return MRLBM_ERR_HIP;
  }
  *out = c;
  return MRLBM_OK;
}
}  // namespace

extern "C" {

int mrlbm_init_equilibrium(mrlbm_ctx *c, int instance, const void *moments) {
  if (bad_instance(c, instance) || !moments) return MRLBM_ERR_INVALID;
  return dispatch<InitOp>(c, instance, moments);
}

int mrlbm_adapt(mrlbm_ctx *c) {
  if (!c) return MRLBM_ERR_INVALID;
  if (!c->all_ready()) return MRLBM_ERR_STATE;
  return dispatch<AdaptOp>(c);
}

int mrlbm_transport_collide(mrlbm_ctx *c) {
  if (!c) return MRLBM_ERR_INVALID;
  if (!c->all_ready()) return MRLBM_ERR_STATE;
  return dispatch<TransportOp>(c);
}

int mrlbm_step(mrlbm_ctx *c, int nsteps) {
  if (!c || nsteps < 0) return MRLBM_ERR_INVALID;
  if (!c->all_ready()) return MRLBM_ERR_STATE;
  for (int s = 0; s < nsteps; ++s) {
    int rc;
    if (c->use_graph) {
      rc = dispatch<StepGraphOp>(c);
    } else {
      rc = dispatch<AdaptOp>(c);
      if (!rc) rc = dispatch<TransportOp>(c);
    }
    if (rc) return rc;
  }
  return MRLBM_OK;
}

int mrlbm_get_state(mrlbm_ctx *c, int instance, uint8_t *tree, void *values) {
  if (bad_instance(c, instance) || !tree || !values) return MRLBM_ERR_INVALID;
  if (!c->has_state[instance]) return MRLBM_ERR_STATE;
  const Inst<double> &I = c->P.inst[instance];
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(tree, c->code[c->mcur] + I.cbase, I.total, hipMemcpyDeviceToHost));
  for (long long k = 0; k < I.total; ++k) tree[k] = tree[k] >= C_INTERNAL ? 1 : 0;
  HIPCHK(hipMemcpy(values, (char *)c->F[c->cur] + c->P.rs * c->P.q * I.cbase, c->P.rs * c->P.q * I.total,
                   hipMemcpyDeviceToHost));
  return sync_status(c);
}

int mrlbm_set_state(mrlbm_ctx *c, int instance, const uint8_t *tree, const void *values) {
  if (bad_instance(c, instance) || !tree || !values) return MRLBM_ERR_INVALID;
  if (!tree_is_graded(c, instance, tree)) return MRLBM_ERR_INVALID;
  const Inst<double> &I = c->P.inst[instance];
  HIPCHK(hipStreamSynchronize(c->stream));
  k_membership<<<grid_cap((c->P.ctotal + BLK - 1) / BLK, DENSE_GRID), BLK, 0, c->stream>>>(c->code[c->mcur], c->tnew,
                                                                                          c->P.ctotal);
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(c->tnew + I.cbase, tree, I.total, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy((char *)c->F[c->cur] + c->P.rs * c->P.q * I.cbase, values, c->P.rs * c->P.q * I.total,
                   hipMemcpyHostToDevice));
  c->recon_reuse = false;  // the new values need a full reconstruction
  activity_reset(c);
  int rc = dispatch<ClassifyOp>(c, c->mcur);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(c->stream));
  c->has_state[instance] = 1;
  return MRLBM_OK;
}

int mrlbm_sizes(const mrlbm_ctx *c, int instance, int64_t *total_cells, int *q) {
  if (!c || instance < 0 || instance >= c->P.B) return MRLBM_ERR_INVALID;
  if (total_cells) *total_cells = c->P.inst[instance].total;
  if (q) *q = c->P.q;
  return MRLBM_OK;
}

int mrlbm_stats(mrlbm_ctx *c, int instance, double *mass, int64_t *leaves, int64_t *internal, int64_t *ghosts) {
  if (bad_instance(c, instance)) return MRLBM_ERR_INVALID;
  if (!c->has_state[instance]) return MRLBM_ERR_STATE;
  const Inst<double> &I = c->P.inst[instance];
  int rc = MRLBM_OK;
  if (mass) {
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemset(c->bad, 0, sizeof(int) * c->P.B));
    dispatch<MassOp>(c);
    std::vector<double> part(2 * RED_BLOCKS * c->P.B);
    int bad = 0;
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(part.data(), c->red, sizeof(double) * part.size(), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&bad, c->bad + instance, sizeof bad, hipMemcpyDeviceToHost));
    // compensated sum of the per-block (sum, compensation) pairs, fixed order
    double s = 0.0, e = 0.0;
    for (int k = 0; k < 2 * RED_BLOCKS; ++k) {
      const double t = part[2 * instance * RED_BLOCKS + k], u = s + t;
      e += std::fabs(s) >= std::fabs(t) ? (s - u) + t : (t - u) + s;
      s = u;
    }
    *mass = s + e;
    if (bad) rc = MRLBM_ERR_NONFINITE;
  }
  {
    const int st = sync_status(c);
    if (st) rc = st;
  }
  int lvl[NCAT * LVL_STRIDE];
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(lvl, c->lvl[c->mcur] + instance * NCAT * LVL_STRIDE, sizeof lvl, hipMemcpyDeviceToHost));
  int64_t *outs[NCAT] = {leaves, internal, ghosts};
  for (int k = 0; k < NCAT; ++k) {
    if (!outs[k]) continue;
    for (int l = 0; l <= I.jmax; ++l)
      outs[k][l] = l < I.jmin ? 0 : lvl[k * LVL_STRIDE + l + 1] - lvl[k * LVL_STRIDE + l];
  }
  return rc;
}

int mrlbm_leaves(mrlbm_ctx *c, int instance, uint32_t *cells, void *values, int64_t capacity, int64_t *count) {
  if (bad_instance(c, instance) || !count) return MRLBM_ERR_INVALID;
  if (!c->has_state[instance]) return MRLBM_ERR_STATE;
  const Inst<double> &I = c->P.inst[instance];
  int lvl[LVL_STRIDE];
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(lvl, c->lvl[c->mcur] + (instance * NCAT + CAT_LEAF) * LVL_STRIDE, sizeof lvl,
                   hipMemcpyDeviceToHost));
  const int64_t n = lvl[I.jmax + 1] - lvl[I.jmin];
  *count = n;
  if (capacity < n) return MRLBM_ERR_CAPACITY;
  if (!cells || !values) return MRLBM_ERR_INVALID;
  dispatch<ExportOp>(c, instance, cells, values);
  return sync_status(c);
}

int mrlbm_fields(mrlbm_ctx *c, int instance, int what, void *out, size_t out_bytes, int64_t *n_written) {
  if (bad_instance(c, instance) || !n_written) return MRLBM_ERR_INVALID;
  if (what < MRLBM_FIELD_LEAF_TABLE || what > MRLBM_FIELD_FINEST) return MRLBM_ERR_INVALID;
  if (!c->has_state[instance]) return MRLBM_ERR_STATE;
  const Inst<double> &I = c->P.inst[instance];
  size_t need = 0;
  if (what == MRLBM_FIELD_FINEST) {
    *n_written = (int64_t)c->P.q << (c->P.dim * I.jmax);
    need = c->P.rs * (size_t)*n_written;
  } else {
    int lvl[LVL_STRIDE];
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(lvl, c->lvl[c->mcur] + (instance * NCAT + CAT_LEAF) * LVL_STRIDE, sizeof lvl,
                     hipMemcpyDeviceToHost));
    const int64_t n = lvl[I.jmax + 1] - lvl[I.jmin];
    *n_written = what == MRLBM_FIELD_LEAF_TABLE ? n : n * c->P.q;
    need = (what == MRLBM_FIELD_LEAF_TABLE ? sizeof(uint32_t) : c->P.rs) * (size_t)*n_written;
  }
  if (out_bytes < need) return MRLBM_ERR_CAPACITY;
  if (!out && need) return MRLBM_ERR_INVALID;
  if (need) {
    const int rc = what == MRLBM_FIELD_FINEST ? dispatch<FinestOp>(c, instance, out)
                                              : dispatch<LeafFieldsOp>(c, instance, what, out);
    if (rc) return rc;
  }
  return sync_status(c);
}

int mrlbm_get_mesh(mrlbm_ctx *c, int instance, uint8_t *tree) {
  if (bad_instance(c, instance) || !tree) return MRLBM_ERR_INVALID;
  if (!c->has_state[instance]) return MRLBM_ERR_STATE;
  const Inst<double> &I = c->P.inst[instance];
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(tree, c->code[c->mcur] + I.cbase, I.total, hipMemcpyDeviceToHost));
  for (long long k = 0; k < I.total; ++k) tree[k] = tree[k] >= C_INTERNAL ? 1 : 0;
  return sync_status(c);
}

int mrlbm_step_frozen(mrlbm_ctx *c, const uint8_t *trees) {
  if (!c || !trees) return MRLBM_ERR_INVALID;
  if (!c->all_ready()) return MRLBM_ERR_STATE;
  const Plan &P = c->P;
  std::vector<uint8_t> old(P.ctotal);
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(old.data(), c->code[c->mcur], P.ctotal, hipMemcpyDeviceToHost));
  for (auto &v : old) v = v >= C_INTERNAL ? 1 : 0;
  for (int i = 0; i < P.B; ++i) {
    const uint8_t *t = trees + P.inst[i].cbase;
    if (!tree_is_graded(c, i, t) || !refines_by_one(c, i, old.data() + P.inst[i].cbase, t))
      return MRLBM_ERR_INVALID;
  }
  return dispatch<FrozenOp>(c, trees);
}

int mrlbm_debug_pair_wait(mrlbm_ctx *c, uint32_t budget, int32_t count) {
  if (!c) return MRLBM_ERR_INVALID;
  const unsigned v[2] = {(unsigned)count, budget ? budget : PAIR_WAIT_BUDGET};
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(c->sync, &v[0], sizeof(unsigned), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->sync + 2, &v[1], sizeof(unsigned), hipMemcpyHostToDevice));
  return MRLBM_OK;
}

int mrlbm_profile(mrlbm_ctx *c, int enable) {
  if (!c) return MRLBM_ERR_INVALID;
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemset(c->cnt, 0, 4 * sizeof(unsigned long long)));
  if (enable < 0 || enable > 2) return MRLBM_ERR_INVALID;
  c->profiling = enable != 0;
  c->timing_period = enable == 2 ? 1 : TIMING_PERIOD;
  c->graph_steps = 0;
  c->ev_used = 0;
  c->ev_marks.clear();
  return MRLBM_OK;
}

int mrlbm_read_counters(mrlbm_ctx *c, mrlbm_counters *out) {
  if (!c || !out) return MRLBM_ERR_INVALID;
  HIPCHK(hipStreamSynchronize(c->stream));
  unsigned long long cnt[4];
  HIPCHK(hipMemcpy(cnt, c->cnt, sizeof cnt, hipMemcpyDeviceToHost));
  std::memset(out, 0, sizeof *out);
  out->leaf_updates = cnt[0];
  out->transport_launches = cnt[1];
  for (const auto &m : c->ev_marks) {
    float ms = 0.f;
    if (m.second + 1 >= c->ev_used) continue;
    HIPCHK(hipEventElapsedTime(&ms, c->ev_pool[m.second], c->ev_pool[m.second + 1]));
    if (m.first == PH_TRANSPORT) { out->transport_ms += ms; out->timed_launches++; }
    else if (m.first == PH_RECON) out->reconstruct_ms += ms;
    else out->adapt_ms += ms;
  }
  return MRLBM_OK;
}

int mrlbm_adjoint_workspace_size(const mrlbm_ctx *c, int nsteps, int ckpt_every, size_t *bytes) {
  if (!c || !bytes || nsteps < 1 || ckpt_every < 1 || c->P.B != 1) return MRLBM_ERR_INVALID;
  *bytes = adj_layout(c->P, nsteps, ckpt_every).bytes;
  return MRLBM_OK;
}

int mrlbm_forward_record(mrlbm_ctx *c, void *adj_workspace, size_t bytes, int nsteps, int ckpt_every) {
  if (!c || !adj_workspace || nsteps < 1 || ckpt_every < 1 || c->P.B != 1) return MRLBM_ERR_INVALID;
  if (c->P.inst[0].walls) return MRLBM_ERR_INVALID;  // the adjoint covers periodic boundaries
  if (c->p[0].scheme == MRLBM_D2Q4_EULER || c->p[0].scheme == MRLBM_D3Q6 || c->P.gamma > 1) return MRLBM_ERR_INVALID;
  if (!c->all_ready()) return MRLBM_ERR_STATE;
  if (bytes < adj_layout(c->P, nsteps, ckpt_every).bytes) return MRLBM_ERR_CAPACITY;
  c->adj_ws = (char *)(((uintptr_t)adj_workspace + 255) & ~(uintptr_t)255);
  c->adj_nsteps = nsteps;
  c->adj_K = ckpt_every;
  c->adj_taped = false;
  return dispatch<RecordOp>(c, nsteps, ckpt_every);
}

int mrlbm_adjoint(mrlbm_ctx *c, const void *abar_final, void *mbar0, double *sbar) {
  if (!c || !abar_final || !mbar0 || !sbar || c->P.B != 1) return MRLBM_ERR_INVALID;
  if (!c->adj_ws || c->adj_nsteps < 1) return MRLBM_ERR_STATE;
  return dispatch<AdjointOp>(c, abar_final, mbar0, sbar);
}

// ---------------------------------------------------------------- autotuner
namespace {
// A schedule is kept per device, scheme, precision, leaf-count octave and
// kernel class (walls, gamma, metric: they select other kernels).
struct TuneKey {
  std::string arch;
  int scheme, precision, bucket, walls, gamma, metric;
  bool operator<(const TuneKey &o) const {
    return std::tie(arch, scheme, precision, bucket, walls, gamma, metric) <
           std::tie(o.arch, o.scheme, o.precision, o.bucket, o.walls, o.gamma, o.metric);
  }
};
std::mutex tune_mutex;
std::map<TuneKey, mrlbm_tuning> tune_cache;

int apply_tuning(mrlbm_ctx *c, const mrlbm_tuning &t) {
  if ((t.transport_variant != 1 && t.transport_variant != 2) || t.list_grid_all < 8 || t.list_grid_all > 65536 ||
      t.list_grid_level < 8 || t.list_grid_level > 65536 || (t.graph != 0 && t.graph != 1) ||
      (t.pair_links != 0 && t.pair_links != 1))
    return MRLBM_ERR_INVALID;
  if (t.graph == 1 && !c->cap_stream) return MRLBM_ERR_STATE;  // static context: no capture stream
  if (c->transport_variant != t.transport_variant || c->grid_all != (unsigned)t.list_grid_all ||
      c->grid_level != (unsigned)t.list_grid_level || c->use_graph != (t.graph == 1) ||
      c->pair_links != (t.pair_links == 1)) {
    (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
  }
  c->use_graph = t.graph == 1;
  c->transport_variant = t.transport_variant;
  c->grid_all = (unsigned)t.list_grid_all;
  c->grid_level = (unsigned)t.list_grid_level;
  c->pair_links = t.pair_links == 1;
  return MRLBM_OK;
}

int leaf_total(mrlbm_ctx *c, long long *n) {
  std::vector<int> lvl((size_t)c->P.B * NCAT * LVL_STRIDE);
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(lvl.data(), c->lvl[c->mcur], sizeof(int) * lvl.size(), hipMemcpyDeviceToHost));
  long long t = 0;
  for (int i = 0; i < c->P.B; ++i) {
    const int *L = &lvl[((size_t)i * NCAT + CAT_LEAF) * LVL_STRIDE];
    t += L[c->P.inst[i].jmax + 1] - L[c->P.inst[i].jmin];
  }
  *n = t;
  return MRLBM_OK;
}
}  // namespace

int mrlbm_get_tuning(const mrlbm_ctx *c, mrlbm_tuning *out) {
  if (!c || !out) return MRLBM_ERR_INVALID;
  std::memset(out, 0, sizeof *out);
  out->transport_variant = c->transport_variant ? c->transport_variant
                                                 : (c->P.ctotal >= LEAF_KERNEL_CELLS ? 1 : 2);
  out->list_grid_all = (int)c->grid_all;
  out->list_grid_level = (int)c->grid_level;
  out->graph = c->use_graph ? 1 : 0;
  out->pair_links = c->pair_links ? 1 : 0;
  return MRLBM_OK;
}

int mrlbm_set_tuning(mrlbm_ctx *c, const mrlbm_tuning *t) {
  if (!c || !t) return MRLBM_ERR_INVALID;
  return apply_tuning(c, *t);
}

int mrlbm_autotune(mrlbm_ctx *c, int reps, mrlbm_tuning *out) {
  if (!c || !out || reps < 1) return MRLBM_ERR_INVALID;
  if (!c->all_ready() || !c->use_graph) return MRLBM_ERR_STATE;
  long long leaves = 0;
  int rc = leaf_total(c, &leaves);
  if (rc) return rc;
  hipDeviceProp_t prop;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipGetDeviceProperties(&prop, dev));
  int bucket = 0;
  while ((2ll << bucket) <= leaves) ++bucket;  // floor(log2(leaves))
  const TuneKey key{prop.gcnArchName, c->p[0].scheme, c->p[0].precision, bucket,
                    c->P.any_walls ? 1 : 0, c->P.gamma, c->P.metric_mode};
  {
    std::lock_guard<std::mutex> lock(tune_mutex);
    auto it = tune_cache.find(key);
    if (it != tune_cache.end()) {
      *out = it->second;
      out->from_cache = 1;
      return apply_tuning(c, *out);
    }
  }
  // leaf counts are device-side; the timed steps must not disturb them
  unsigned long long cnt[4];
  HIPCHK(hipMemcpy(cnt, c->cnt, sizeof cnt, hipMemcpyDeviceToHost));
  mrlbm_tuning best{};
  best.ms_per_step = 1e30;
  const int variants[2] = {1, 2};
  const int all_caps[4] = {1024, 2048, 4096, 8192};
  const int level_caps[3] = {256, 1024, 4096};
  for (int v : variants)
    for (int ga : all_caps)
      for (int gl : level_caps)
        for (int pl = 0; pl < 2; ++pl) {
          mrlbm_tuning t{};
          t.transport_variant = v;
          t.list_grid_all = ga;
          t.list_grid_level = gl;
          t.graph = 1;
          t.pair_links = pl;
          rc = apply_tuning(c, t);
          float ms = 0.f;
          if (!rc) rc = dispatch<DryOp>(c, reps, &ms);
          if (rc) return rc;
          if (ms < best.ms_per_step) {
            best = t;
            best.ms_per_step = ms;
          }
        }
  HIPCHK(hipMemcpy(c->cnt, cnt, sizeof cnt, hipMemcpyHostToDevice));
  rc = apply_tuning(c, best);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> lock(tune_mutex);
    tune_cache[key] = best;
  }
  *out = best;
  return MRLBM_OK;
}

int mrlbm_destroy(mrlbm_ctx *c) {
  if (!c) return MRLBM_OK;
  (void)hipStreamSynchronize(c->stream);
  drop_graphs(c);
  for (auto e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->ev_placeholder) (void)hipEventDestroy(c->ev_placeholder);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->static_dev >= 0) {
    std::lock_guard<std::mutex> lock(static_mutex);
    static_busy[c->static_dev] = false;
  }
  delete c;
  return MRLBM_OK;
}

int mrlbm_copy(void *dst, const void *src, size_t bytes, void *stream) {
  if (!dst || !src || bytes % 16 || ((uintptr_t)dst | (uintptr_t)src) % 16) return MRLBM_ERR_INVALID;
  const long long n = (long long)(bytes / 16);
  if (n == 0) return MRLBM_OK;
  k_copy_u4<<<grid_cap((n + BLK - 1) / BLK, 8192), BLK, 0, (hipStream_t)stream>>>((uint4 *)dst, (const uint4 *)src,
                                                                                  n);
  return hipPeekAtLastError() == hipSuccess ? MRLBM_OK : MRLBM_ERR_HIP;
}

const char *mrlbm_status_string(int s) {
  switch (s) {
    case MRLBM_OK: return "ok";
    case MRLBM_ERR_INVALID: return "invalid argument";
    case MRLBM_ERR_CAPACITY: return "buffer too small";
    case MRLBM_ERR_NONFINITE: return "non-finite leaf value";
    case MRLBM_ERR_HIP: return "HIP runtime error";
    case MRLBM_ERR_STATE: return "call out of order";
    case MRLBM_ERR_SYNC: return "device-side wait gave up";
    default: return "unknown status";
  }
}

int mrlbm_transport_tables(int scheme, int n, double *W, double *C) {
  if (scheme < MRLBM_D1Q2 || scheme > MRLBM_D2Q4_EULER || n < 1 || n > 25 || !W || !C) return MRLBM_ERR_INVALID;
  if (scheme_dim(scheme) == 2 && n > 13) return MRLBM_ERR_INVALID;
  transport_tables(scheme, n, W, C);
  return MRLBM_OK;
}

int mrlbm_transport_tables_general(int scheme, int n, int gamma, int wall_x, int wall_y, double *W, double *C,
                                   double *N) {
  if (scheme < MRLBM_D1Q2 || scheme > MRLBM_D2Q4_EULER || n < 1 || n > 25 || !W || !C || !N) return MRLBM_ERR_INVALID;
  if (scheme_dim(scheme) == 2 && n > 13) return MRLBM_ERR_INVALID;
  if (gamma < 1 || gamma > 3 || wall_x < 0 || wall_x > 2 || wall_y < 0 || wall_y > 2) return MRLBM_ERR_INVALID;
  if (scheme_dim(scheme) == 1 && wall_y) return MRLBM_ERR_INVALID;
  const int q = scheme_q(scheme), R = 2 * gamma, WW = 2 * R + 1, CW = 2 * R + 2;
  std::vector<double> w((size_t)q * WW * WW), c((size_t)q * CW * CW);
  transport_tables(scheme, n, w.data(), c.data(), wall_x, wall_y, N, gamma);
  const int d = scheme_dim(scheme), ws = wide_ws(d, gamma), cs = wide_cs(d, gamma);
  for (int h = 0; h < q; ++h) {  // a 1D scheme keeps the middle row
    for (int k = 0; k < ws; ++k) W[(size_t)h * ws + k] = w[(size_t)h * WW * WW + (d == 2 ? k : R * WW + k)];
    for (int k = 0; k < cs; ++k) C[(size_t)h * cs + k] = c[(size_t)h * CW * CW + (d == 2 ? k : R * CW + k)];
  }
  return MRLBM_OK;
}

}  // extern "C"
