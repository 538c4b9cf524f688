// C-ABI of the MR-LBM hot path (declared in include/mrlbm.h): context set-up in a
// caller-owned workspace, the flattened transport weights, and the per-step
// launch sequence of Algorithm 1 of arXiv 2103.02903.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "mr_kernels.h"
#include "mrlbm.h"

using namespace mrlbm;

namespace {

int scheme_dim(int s) { return s == MRLBM_D2Q9 ? 2 : 1; }
int scheme_q(int s) { return s == MRLBM_D1Q2 ? 2 : s == MRLBM_D1Q3 ? 3 : 9; }
int scheme_nc(int s) { return s == MRLBM_D2Q9 ? 3 : 1; }
void scheme_eta(int s, int h, int &ex, int &ey) {
  static const int d1q2[2] = {1, -1};
  static const int d1q3[3] = {0, 1, -1};
  static const int d2q9x[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  static const int d2q9y[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  if (s == MRLBM_D1Q2) { ex = d1q2[h]; ey = 0; }
  else if (s == MRLBM_D1Q3) { ex = d1q3[h]; ey = 0; }
  else { ex = d2q9x[h]; ey = d2q9y[h]; }
}
bool conserved(int s, int i) { return s == MRLBM_D2Q9 ? i < 3 : i == 0; }

int validate(const mrlbm_params *p) {
  if (!p) return MRLBM_ERR_INVALID;
  if (p->scheme < MRLBM_D1Q2 || p->scheme > MRLBM_D2Q9) return MRLBM_ERR_INVALID;
  const int dim = scheme_dim(p->scheme);
  const int maxj = dim == 2 ? 13 : 25;
  if (p->jmin < 1 || p->jmax < p->jmin || p->jmax > maxj) return MRLBM_ERR_INVALID;
  if (p->precision != 4 && p->precision != 8) return MRLBM_ERR_INVALID;
  if (!(p->lambda > 0.0) || !std::isfinite(p->lambda)) return MRLBM_ERR_INVALID;
  if (!(p->eps >= 0.0)) return MRLBM_ERR_INVALID;
  if (!(p->mu_bar >= 0.0 && p->mu_bar <= 3.0)) return MRLBM_ERR_INVALID;
  for (int i = 0; i < scheme_q(p->scheme); ++i) {
    if (!std::isfinite(p->s[i])) return MRLBM_ERR_INVALID;
    if (conserved(p->scheme, i) && p->s[i] != 0.0) return MRLBM_ERR_INVALID;
  }
  return MRLBM_OK;
}

// ---------------------------------------------------------------- transport weights
// Reconstruction of an impulse placed on one cell of a coarse level, n levels
// down, by repeated 1D prediction (gamma = 1). `v` covers indices [lo, lo+size).
void predict_down(std::vector<double> &v, long long &lo, int n) {
  for (int k = 0; k < n; ++k) {
    const long long sz = (long long)v.size();
    std::vector<double> w(2 * sz, 0.0);
    auto at = [&](long long i) { return (i < 0 || i >= sz) ? 0.0 : v[i]; };
    for (long long i = 0; i < sz; ++i) {
      const double q = -0.125 * (at(i + 1) - at(i - 1));
      w[2 * i] = v[i] + q;
      w[2 * i + 1] = v[i] - q;
    }
    v.swap(w);
    lo *= 2;
  }
}

// Sum over the finest cells [-e, 2^n - e) (the leaf's finest cells shifted by
// -e) of the reconstruction of a unit impulse at cell `a` of level J - m
// (the leaf covers [0, 2^n) finest cells, n >= m).
double impulse_sum(int n, int m, int e, int a) {
  const long long pad = 8;
  std::vector<double> v(2 * pad + 1, 0.0);
  long long lo = -pad;
  v[a - lo] = 1.0;
  predict_down(v, lo, m);
  double s = 0.0;
  const long long b0 = -e, b1 = (1ll << n) - e;
  for (long long i = b0; i < b1; ++i) {
    const long long k = i - lo;
    if (k >= 0 && k < (long long)v.size()) s += v[k];
  }
  return s;
}

// W[h][25] and C[h][36] of a leaf n >= 1 levels above the finest (see header).
void transport_tables(int scheme, int n, double *W, double *C) {
  const int q = scheme_q(scheme), dim = scheme_dim(scheme);
  for (int h = 0; h < q; ++h) {
    int ex, ey;
    scheme_eta(scheme, h, ex, ey);
    double Sx[5], Sy[5], Tx[6], Ty[6];
    for (int a = -2; a <= 2; ++a) {
      Sx[a + 2] = impulse_sum(n, n, ex, a);
      Sy[a + 2] = dim == 2 ? impulse_sum(n, n, ey, a) : (a == 0 ? 1.0 : 0.0);
    }
    // detail impulses live one level below the leaf, on cells 2k + y, y in [-2, 3];
    // the leaf's range is then [0, 2) cells of that level = [0, 2^n) finest cells
    for (int y = -2; y <= 3; ++y) {
      Tx[y + 2] = impulse_sum(n, n - 1, ex, y);
      Ty[y + 2] = dim == 2 ? impulse_sum(n, n - 1, ey, y) : (y == 0 ? 1.0 : 0.0);
    }
    const double full = std::ldexp(1.0, dim * n);
    for (int b = -2; b <= 2; ++b)
      for (int a = -2; a <= 2; ++a) {
        double w = Sx[a + 2] * Sy[b + 2];
        if (a == 0 && b == 0) w -= (ex == 0 && ey == 0) ? w : full;  // E - A form; rest velocity: 0
        W[h * 25 + (b + 2) * 5 + (a + 2)] = w;
      }
    for (int y2 = -2; y2 <= 3; ++y2)
      for (int y1 = -2; y1 <= 3; ++y1) C[h * 36 + (y2 + 2) * 6 + (y1 + 2)] = (ex == 0 && ey == 0) ? 0.0 : Tx[y1 + 2] * Ty[y2 + 2];
  }
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  long long total;
  int nb, nmax, q, dim;
  size_t rs;  // sizeof(real)
  size_t off_F[2], off_code[2], off_lists[2], off_lvl[2], off_keep, off_refg, off_tnew, off_bcnt, off_boff,
      off_W, off_C, off_red, off_bad, bytes;
};

void make_geo(const mrlbm_params *p, Geo &g, Layout &L) {
  std::memset(&g, 0, sizeof g);
  g.dim = scheme_dim(p->scheme);
  g.q = scheme_q(p->scheme);
  g.jmin = p->jmin;
  g.jmax = p->jmax;
  long long off = 0;
  int blocks = 0;
  for (int l = 0; l <= MAXLEV + 1; ++l) {
    g.loff[l] = off;
    g.bstart[l] = blocks;
    if (l >= p->jmin && l <= p->jmax) {
      const long long n = 1ll << (g.dim * l);
      off += n;
      blocks += (int)((n + CCHUNK - 1) / CCHUNK);
    }
  }
  L.total = g.loff[p->jmax + 1];
  L.nb = g.bstart[p->jmax + 1];
  L.nmax = p->jmax - p->jmin;
  L.q = g.q;
  L.dim = g.dim;
  L.rs = p->precision == 8 ? 8 : 4;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
  for (int k = 0; k < 2; ++k) L.off_F[k] = take(L.rs * L.q * L.total);
  for (int k = 0; k < 2; ++k) L.off_code[k] = take(L.total);
  for (int k = 0; k < 2; ++k) L.off_lists[k] = take(sizeof(uint32_t) * NCAT * L.total);
  for (int k = 0; k < 2; ++k) L.off_lvl[k] = take(sizeof(int) * NCAT * LVL_STRIDE);
  L.off_keep = take(L.total);
  L.off_refg = take(L.total);
  L.off_tnew = take(L.total);
  L.off_bcnt = take(sizeof(int) * NCAT * L.nb);
  L.off_boff = take(sizeof(int) * NCAT * L.nb);
  const int ws = g.dim == 2 ? 25 : 5, cs = g.dim == 2 ? 36 : 6;
  L.off_W = take(L.rs * std::max(1, L.nmax) * L.q * ws);
  L.off_C = take(L.rs * std::max(1, L.nmax) * L.q * cs);
  L.off_red = take(sizeof(double) * RED_BLOCKS);
  L.off_bad = take(sizeof(int) * 4);
  L.bytes = o + 256;  // slack for aligning the base pointer
}

unsigned grid_for(long long n, unsigned cap = 4096) {
  long long b = (n + BLK - 1) / BLK;
  if (b < 1) b = 1;
  return (unsigned)(b > cap ? cap : b);
}

}  // namespace

struct mrlbm_ctx {
  mrlbm_params p;
  Geo geo;
  Layout L;
  hipStream_t stream;
  char *base;
  void *F[2];
  uint8_t *code[2];
  uint32_t *lists[2];
  int *lvl[2];
  uint8_t *keep, *refg, *tnew;
  int *bcnt, *boff;
  void *W, *C;
  double *red;
  int *bad;
  int cur;   // F[cur] holds the state
  int mcur;  // code/lists/lvl[mcur] describe the current mesh
  bool has_state;
  double eps_l[MAXLEV + 2], ref_l[MAXLEV + 2];
};

namespace {

#define HIPCHK(x)                                      \
  do {                                                 \
    if ((x) != hipSuccess) return MRLBM_ERR_HIP;       \
  } while (0)

template <typename T>
Thresholds<T> thresholds(const mrlbm_ctx *c) {
  Thresholds<T> t;
  for (int l = 0; l < MAXLEV + 2; ++l) {
    t.eps_l[l] = (T)c->eps_l[l];
    t.ref_l[l] = (T)c->ref_l[l];
  }
  return t;
}

template <typename T>
SchemeC<T> scheme_consts(const mrlbm_params &p) {
  SchemeC<T> s;
  s.lam = (T)p.lambda;
  s.inv_lam = (T)(1.0 / p.lambda);
  s.eq = (T)p.eq_param;
  for (int i = 0; i < 9; ++i) s.s[i] = (T)p.s[i];
  return s;
}

// Leaves / internal cells / ghosts of the mesh `code[m]` into lists[m], lvl[m].
int compact(mrlbm_ctx *c, int m) {
  const Geo &g = c->geo;
  k_compact_count<<<dim3(c->L.nb), dim3(BLK), 0, c->stream>>>(g, c->code[m], c->bcnt);
  k_compact_scan<<<dim3(1), dim3(1024), 0, c->stream>>>(g, c->bcnt, c->boff, c->lvl[m]);
  k_compact_scatter<<<dim3(c->L.nb), dim3(BLK), 0, c->stream>>>(g, c->code[m], c->boff, c->lists[m], (long long)c->L.total);
  return MRLBM_OK;
}

// Codes (leaf / internal / ghost) of the membership array tnew into code[m].
template <int DIM>
int classify(mrlbm_ctx *c, int m) {
  const Geo &g = c->geo;
  k_classify_tree<DIM><<<dim3(grid_for(c->L.total)), dim3(BLK), 0, c->stream>>>(g, c->tnew, c->code[m]);
  for (int l = g.jmax; l > g.jmin; --l)
    k_classify_ghost<DIM><<<dim3(grid_for(1ll << (DIM * l))), dim3(BLK), 0, c->stream>>>(g, c->code[m], l);
  return compact(c, m);
}

// Reconstruction on the mesh m inside buffer F: projections upward, ghost
// predictions downward.
template <int DIM, typename T>
void reconstruct(mrlbm_ctx *c, T *F, int m) {
  const Geo &g = c->geo;
  for (int l = g.jmax - 1; l >= g.jmin; --l)
    k_project<DIM, T><<<dim3(grid_for(1ll << (DIM * l), 1024)), dim3(BLK), 0, c->stream>>>(g, F, c->lists[m] + (size_t)CAT_INTERNAL * c->L.total, c->lvl[m], l);
  for (int l = g.jmin + 1; l <= g.jmax; ++l)
    k_ghost<DIM, T><<<dim3(grid_for(1ll << (DIM * l), 1024)), dim3(BLK), 0, c->stream>>>(g, F, c->lists[m] + (size_t)CAT_GHOST * c->L.total, c->lvl[m], l);
}

template <int DIM, int SCHEME, typename T>
int adapt_impl(mrlbm_ctx *c) {
  const Geo &g = c->geo;
  const int mo = c->mcur, mn = 1 - c->mcur;
  T *Fc = (T *)c->F[c->cur];
  T *Fn = (T *)c->F[1 - c->cur];
  const long long tot = c->L.total;
  reconstruct<DIM, T>(c, Fc, mo);
  // keep and refg are adjacent byte arrays; clear both (256-byte aligned) with one fill
  {
    const long long n4 = (long long)(2 * align256((size_t)tot) / 4);
    k_fill_u32<<<dim3(grid_for(n4)), dim3(BLK), 0, c->stream>>>((uint32_t *)c->keep, n4, 0u);
  }
  k_details<DIM, T><<<dim3(grid_for(tot)), dim3(BLK), 0, c->stream>>>(g, Fc, c->lists[mo] + (size_t)CAT_INTERNAL * tot, c->lvl[mo], thresholds<T>(c), c->keep, c->refg);
  for (int l = g.jmax; l >= g.jmin + 2; --l)
    k_ancestor<DIM><<<dim3(grid_for(1ll << (DIM * (l - 2)))), dim3(BLK), 0, c->stream>>>(g, c->keep, l);
  k_enlarge<DIM, SCHEME><<<dim3(grid_for(tot)), dim3(BLK), 0, c->stream>>>(g, c->keep, c->refg, c->tnew);
  for (int l = g.jmax; l >= g.jmin + 1; --l)
    k_grade<DIM><<<dim3(grid_for(1ll << (DIM * (l - 1)))), dim3(BLK), 0, c->stream>>>(g, c->tnew, l);
  classify<DIM>(c, mn);
  k_transfer<DIM, T><<<dim3(grid_for(tot)), dim3(BLK), 0, c->stream>>>(g, Fc, Fn, c->code[mo], c->lists[mn] + (size_t)CAT_LEAF * tot, c->lvl[mn]);
  c->mcur = mn;
  c->cur = 1 - c->cur;
  return hipPeekAtLastError() == hipSuccess ? MRLBM_OK : MRLBM_ERR_HIP;
}

template <int DIM, int SCHEME, typename T>
int transport_impl(mrlbm_ctx *c) {
  const Geo &g = c->geo;
  const int m = c->mcur;
  T *Fc = (T *)c->F[c->cur];
  T *Fn = (T *)c->F[1 - c->cur];
  reconstruct<DIM, T>(c, Fc, m);
  k_transport_collide<DIM, SCHEME, T><<<dim3(grid_for(c->L.total)), dim3(BLK), 0, c->stream>>>(g, Fc, Fn, c->code[m], c->lists[m] + (size_t)CAT_LEAF * c->L.total, c->lvl[m], (const T *)c->W, (const T *)c->C, scheme_consts<T>(c->p));
  c->cur = 1 - c->cur;
  return hipPeekAtLastError() == hipSuccess ? MRLBM_OK : MRLBM_ERR_HIP;
}

template <int DIM, int SCHEME, typename T>
int init_impl(mrlbm_ctx *c, const void *mom) {
  const Geo &g = c->geo;
  T *F = (T *)c->F[c->cur];
  k_init_equilibrium<DIM, SCHEME, T><<<dim3(grid_for(1ll << (DIM * g.jmax))), dim3(BLK), 0, c->stream>>>(g, F, (const T *)mom, scheme_consts<T>(c->p));
  k_full_tree<<<dim3(grid_for(c->L.total)), dim3(BLK), 0, c->stream>>>(g, c->code[c->mcur]);
  compact(c, c->mcur);
  c->has_state = true;
  return hipPeekAtLastError() == hipSuccess ? MRLBM_OK : MRLBM_ERR_HIP;
}

// Dispatch on (scheme, precision).
template <template <int, int, typename> class Op, typename... A>
int dispatch(mrlbm_ctx *c, A... a) {
  const bool dbl = c->p.precision == 8;
  switch (c->p.scheme) {
    case MRLBM_D1Q2: return dbl ? Op<1, 1, double>::run(c, a...) : Op<1, 1, float>::run(c, a...);
    case MRLBM_D1Q3: return dbl ? Op<1, 2, double>::run(c, a...) : Op<1, 2, float>::run(c, a...);
    default: return dbl ? Op<2, 3, double>::run(c, a...) : Op<2, 3, float>::run(c, a...);
  }
}
template <int D, int S, typename T>
struct AdaptOp { static int run(mrlbm_ctx *c) { return adapt_impl<D, S, T>(c); } };
template <int D, int S, typename T>
struct TransportOp { static int run(mrlbm_ctx *c) { return transport_impl<D, S, T>(c); } };
template <int D, int S, typename T>
struct InitOp { static int run(mrlbm_ctx *c, const void *m) { return init_impl<D, S, T>(c, m); } };
template <int D, int S, typename T>
struct ClassifyOp { static int run(mrlbm_ctx *c, int m) { return classify<D>(c, m); } };
template <int D, int S, typename T>
struct MassOp {
  static int run(mrlbm_ctx *c, int) {
    k_mass_partial<T><<<dim3(RED_BLOCKS), dim3(BLK), 0, c->stream>>>(c->geo, (const T *)c->F[c->cur], c->lists[c->mcur] + (size_t)CAT_LEAF * c->L.total, c->lvl[c->mcur], c->red, c->bad);
    return MRLBM_OK;
  }
};
template <int D, int S, typename T>
struct ExportOp {
  static int run(mrlbm_ctx *c, uint32_t *cells, void *vals) {
    k_export<T><<<dim3(grid_for(c->L.total)), dim3(BLK), 0, c->stream>>>(c->geo, (const T *)c->F[c->cur], c->lists[c->mcur] + (size_t)CAT_LEAF * c->L.total, c->lvl[c->mcur], cells, (T *)vals);
    return MRLBM_OK;
  }
};

// Host check of a 0/1 tree: level jmin complete, sibling groups complete, every
// tree cell's parent and prediction stencil present.
bool tree_is_graded(const mrlbm_ctx *c, const uint8_t *t) {
  const Geo &g = c->geo;
  const int d = g.dim;
  for (long long i = 0; i < (1ll << (d * g.jmin)); ++i)
    if (!t[g.loff[g.jmin] + i]) return false;
  for (int l = g.jmin + 1; l <= g.jmax; ++l) {
    const int np = 1 << (l - 1);
    const uint8_t *tl = t + g.loff[l], *tp = t + g.loff[l - 1];
    for (int py = 0; py < (d == 2 ? np : 1); ++py)
      for (int px = 0; px < np; ++px) {
        int cnt = 0;
        for (int dy = 0; dy < (d == 2 ? 2 : 1); ++dy)
          for (int dx = 0; dx < 2; ++dx) {
            const long long ci = d == 2 ? (long long)(2 * px + dx) + ((long long)(2 * py + dy) << l) : 2 * px + dx;
            cnt += tl[ci] ? 1 : 0;
          }
        if (cnt == 0) continue;
        if (cnt != (1 << d)) return false;
        for (int b = (d == 2 ? -1 : 0); b <= (d == 2 ? 1 : 0); ++b)
          for (int a = -1; a <= 1; ++a) {
            const int x = (px + a) & (np - 1), y = (py + b) & (np - 1);
            const long long pi = d == 2 ? (long long)x + ((long long)y << (l - 1)) : x;
            if (!tp[pi]) return false;
          }
      }
  }
  return true;
}

}  // namespace

// ====================================================================== C-ABI

extern "C" {

int mrlbm_workspace_size(const mrlbm_params *p, size_t *bytes) {
  if (!bytes) return MRLBM_ERR_INVALID;
  const int rc = validate(p);
  if (rc) return rc;
  Geo g;
  Layout L;
  make_geo(p, g, L);
  *bytes = L.bytes;
  return MRLBM_OK;
}

int mrlbm_create(const mrlbm_params *p, void *workspace, size_t ws_bytes, void *stream, mrlbm_ctx **out) {
  if (!out || !workspace) return MRLBM_ERR_INVALID;
  *out = nullptr;
  const int rc = validate(p);
  if (rc) return rc;
  mrlbm_ctx *c = new (std::nothrow) mrlbm_ctx();
  if (!c) return MRLBM_ERR_INVALID;
  c->p = *p;
  make_geo(p, c->geo, c->L);
  if (ws_bytes < c->L.bytes) { delete c; return MRLBM_ERR_CAPACITY; }
  c->stream = (hipStream_t)stream;
  char *b = (char *)(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
  c->base = b;
  const Layout &L = c->L;
  for (int k = 0; k < 2; ++k) {
    c->F[k] = b + L.off_F[k];
    c->code[k] = (uint8_t *)(b + L.off_code[k]);
    c->lists[k] = (uint32_t *)(b + L.off_lists[k]);
    c->lvl[k] = (int *)(b + L.off_lvl[k]);
  }
  c->keep = (uint8_t *)(b + L.off_keep);
  c->refg = (uint8_t *)(b + L.off_refg);
  c->tnew = (uint8_t *)(b + L.off_tnew);
  c->bcnt = (int *)(b + L.off_bcnt);
  c->boff = (int *)(b + L.off_boff);
  c->W = b + L.off_W;
  c->C = b + L.off_C;
  c->red = (double *)(b + L.off_red);
  c->bad = (int *)(b + L.off_bad);
  c->cur = 0;
  c->mcur = 0;
  c->has_state = false;
  const int d = c->geo.dim;
  for (int l = 0; l < MAXLEV + 2; ++l) {
    c->eps_l[l] = std::ldexp(p->eps, d * (l - p->jmax));
    c->ref_l[l] = std::ldexp(c->eps_l[l], d) * std::exp2(p->mu_bar);
  }
  // transport weight tables, rounded once to the working precision
  const int q = L.q, ws = d == 2 ? 25 : 5, cs = d == 2 ? 36 : 6;
  const int nn = std::max(1, L.nmax);
  std::vector<double> W((size_t)nn * q * ws, 0.0), C((size_t)nn * q * cs, 0.0), w25(q * 25), c36(q * 36);
  for (int n = 1; n <= L.nmax; ++n) {
    transport_tables(p->scheme, n, w25.data(), c36.data());
    for (int h = 0; h < q; ++h) {
      for (int k = 0; k < ws; ++k) W[((size_t)(n - 1) * q + h) * ws + k] = d == 2 ? w25[h * 25 + k] : w25[h * 25 + 10 + k];
      for (int k = 0; k < cs; ++k) C[((size_t)(n - 1) * q + h) * cs + k] = d == 2 ? c36[h * 36 + k] : c36[h * 36 + 12 + k];
    }
  }
  hipError_t e;
  if (p->precision == 8) {
    e = hipMemcpy(c->W, W.data(), W.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->C, C.data(), C.size() * 8, hipMemcpyHostToDevice);
  } else {
    std::vector<float> Wf(W.begin(), W.end()), Cf(C.begin(), C.end());
    e = hipMemcpy(c->W, Wf.data(), Wf.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->C, Cf.data(), Cf.size() * 4, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) { delete c; return MRLBM_ERR_HIP; }
  *out = c;
  return MRLBM_OK;
}

int mrlbm_init_equilibrium(mrlbm_ctx *c, const void *moments) {
  if (!c || !moments) return MRLBM_ERR_INVALID;
  return dispatch<InitOp>(c, moments);
}

int mrlbm_adapt(mrlbm_ctx *c) {
  if (!c) return MRLBM_ERR_INVALID;
  if (!c->has_state) return MRLBM_ERR_STATE;
  return dispatch<AdaptOp>(c);
}

int mrlbm_transport_collide(mrlbm_ctx *c) {
  if (!c) return MRLBM_ERR_INVALID;
  if (!c->has_state) return MRLBM_ERR_STATE;
  return dispatch<TransportOp>(c);
}

int mrlbm_step(mrlbm_ctx *c, int nsteps) {
  if (!c || nsteps < 0) return MRLBM_ERR_INVALID;
  if (!c->has_state) return MRLBM_ERR_STATE;
  for (int s = 0; s < nsteps; ++s) {
    int rc = dispatch<AdaptOp>(c);
    if (rc) return rc;
    rc = dispatch<TransportOp>(c);
    if (rc) return rc;
  }
  return MRLBM_OK;
}

int mrlbm_get_state(mrlbm_ctx *c, uint8_t *tree, void *values) {
  if (!c || !tree || !values) return MRLBM_ERR_INVALID;
  if (!c->has_state) return MRLBM_ERR_STATE;
  const long long tot = c->L.total;
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(tree, c->code[c->mcur], tot, hipMemcpyDeviceToHost));
  for (long long i = 0; i < tot; ++i) tree[i] = tree[i] >= C_INTERNAL ? 1 : 0;
  HIPCHK(hipMemcpy(values, c->F[c->cur], c->L.rs * c->L.q * tot, hipMemcpyDeviceToHost));
  return MRLBM_OK;
}

int mrlbm_set_state(mrlbm_ctx *c, const uint8_t *tree, const void *values) {
  if (!c || !tree || !values) return MRLBM_ERR_INVALID;
  if (!tree_is_graded(c, tree)) return MRLBM_ERR_INVALID;
  const long long tot = c->L.total;
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(c->tnew, tree, tot, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->F[c->cur], values, c->L.rs * c->L.q * tot, hipMemcpyHostToDevice));
  int rc = dispatch<ClassifyOp>(c, c->mcur);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(c->stream));
  c->has_state = true;
  return MRLBM_OK;
}

int mrlbm_sizes(const mrlbm_ctx *c, int64_t *total_cells, int *q) {
  if (!c) return MRLBM_ERR_INVALID;
  if (total_cells) *total_cells = c->L.total;
  if (q) *q = c->L.q;
  return MRLBM_OK;
}

int mrlbm_stats(mrlbm_ctx *c, double *mass, int64_t *leaves, int64_t *internal, int64_t *ghosts) {
  if (!c) return MRLBM_ERR_INVALID;
  if (!c->has_state) return MRLBM_ERR_STATE;
  int lvl[NCAT * LVL_STRIDE];
  int rc = MRLBM_OK;
  if (mass) {
    HIPCHK(hipMemsetAsync(c->bad, 0, sizeof(int), c->stream));
    dispatch<MassOp>(c, 0);
    double part[RED_BLOCKS];
    int bad = 0;
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(part, c->red, sizeof part, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&bad, c->bad, sizeof bad, hipMemcpyDeviceToHost));
    double s = 0.0;
    for (int i = 0; i < RED_BLOCKS; ++i) s += part[i];
    *mass = s;
    if (bad) rc = MRLBM_ERR_NONFINITE;
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(lvl, c->lvl[c->mcur], sizeof lvl, hipMemcpyDeviceToHost));
  int64_t *outs[NCAT] = {leaves, internal, ghosts};
  for (int k = 0; k < NCAT; ++k) {
    if (!outs[k]) continue;
    for (int l = 0; l <= c->p.jmax; ++l)
      outs[k][l] = l < c->p.jmin ? 0 : lvl[k * LVL_STRIDE + l + 1] - lvl[k * LVL_STRIDE + l];
  }
  return rc;
}

int mrlbm_leaves(mrlbm_ctx *c, uint32_t *cells, void *values, int64_t capacity, int64_t *count) {
  if (!c || !count) return MRLBM_ERR_INVALID;
  if (!c->has_state) return MRLBM_ERR_STATE;
  int lvl[NCAT * LVL_STRIDE];
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(lvl, c->lvl[c->mcur], sizeof lvl, hipMemcpyDeviceToHost));
  const int64_t n = lvl[CAT_LEAF * LVL_STRIDE + c->p.jmax + 1] - lvl[CAT_LEAF * LVL_STRIDE + c->p.jmin];
  *count = n;
  if (capacity < n) return MRLBM_ERR_CAPACITY;
  if (!cells || !values) return MRLBM_ERR_INVALID;
  dispatch<ExportOp>(c, cells, values);
  HIPCHK(hipStreamSynchronize(c->stream));
  return MRLBM_OK;
}

int mrlbm_destroy(mrlbm_ctx *c) {
  delete c;
  return MRLBM_OK;
}

const char *mrlbm_status_string(int s) {
  switch (s) {
    case MRLBM_OK: return "ok";
    case MRLBM_ERR_INVALID: return "invalid argument";
    case MRLBM_ERR_CAPACITY: return "buffer too small";
    case MRLBM_ERR_NONFINITE: return "non-finite leaf value";
    case MRLBM_ERR_HIP: return "HIP runtime error";
    case MRLBM_ERR_STATE: return "call out of order";
    default: return "unknown status";
  }
}

int mrlbm_transport_tables(int scheme, int n, double *W, double *C) {
  if (scheme < MRLBM_D1Q2 || scheme > MRLBM_D2Q9 || n < 1 || n > 25 || !W || !C) return MRLBM_ERR_INVALID;
  if (scheme_dim(scheme) == 2 && n > 13) return MRLBM_ERR_INVALID;
  transport_tables(scheme, n, W, C);
  return MRLBM_OK;
}

}  // extern "C"
