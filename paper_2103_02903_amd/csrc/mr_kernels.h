// Kernels of one MR-LBM time step (Algorithm 1 of arXiv 2103.02903).
//
// Every launch is a grid-stride loop whose trip count is either a dense level
// size (known on the host) or a list length that the compaction left in device
// memory, so a whole step is enqueued without any host synchronisation.
#pragma once

#include "mr_device.h"

namespace mrlbm {

constexpr int BLK = 256;

__device__ __forceinline__ int lvl_count(const int *lvl, int cat, int l) {
  return lvl[cat * LVL_STRIDE + l + 1] - lvl[cat * LVL_STRIDE + l];
}

// ---------------------------------------------------------------- reconstruction
// Projection P_nabla on the internal cells of level l (section "Projection and
// prediction operators"), children read at level l+1 of the same buffer.
template <int DIM, typename T>
__global__ void __launch_bounds__(BLK) k_project(Geo g, T *__restrict__ F, const uint32_t *__restrict__ lst,
                                                 const int *__restrict__ lvl, int l) {
  const int beg = lvl[CAT_INTERNAL * LVL_STRIDE + l], n = lvl_count(lvl, CAT_INTERNAL, l);
  for (int i = blockIdx.x * BLK + threadIdx.x; i < n; i += gridDim.x * BLK) {
    const uint32_t c = lst[beg + i] & CELL_MASK;
    int x, y;
    coords<DIM>(l, c, x, y);
    for (int h = 0; h < g.q; ++h) F[foff(g, l, h) + c] = project<DIM, T>(F + foff(g, l + 1, h), l + 1, x, y);
  }
}

// Zero-detail prediction P_delta on the ghost cells of level l, from level l-1.
template <int DIM, typename T>
__global__ void __launch_bounds__(BLK) k_ghost(Geo g, T *__restrict__ F, const uint32_t *__restrict__ lst,
                                               const int *__restrict__ lvl, int l) {
  const int beg = lvl[CAT_GHOST * LVL_STRIDE + l], n = lvl_count(lvl, CAT_GHOST, l);
  for (int i = blockIdx.x * BLK + threadIdx.x; i < n; i += gridDim.x * BLK) {
    const uint32_t c = lst[beg + i] & CELL_MASK;
    int x, y;
    coords<DIM>(l, c, x, y);
    for (int h = 0; h < g.q; ++h) F[foff(g, l, h) + c] = predict<DIM, T>(F + foff(g, l - 1, h), l, x, y);
  }
}

// ---------------------------------------------------------------- mesh adaptation
// Details and the sibling l-infinity metric over all populations (section "Mesh
// coarsening"), one thread per internal cell p (level l-1) of the old tree:
// keep the children (T_eps, eq. Thresholding) if the metric reaches eps_l, flag
// the group for refinement (H_eps) if it reaches 2^{mu_bar + d} eps_l.
template <int DIM, typename T>
__global__ void __launch_bounds__(BLK) k_details(Geo g, const T *__restrict__ F, const uint32_t *__restrict__ lst,
                                                 const int *__restrict__ lvl, Thresholds<T> thr,
                                                 uint8_t *__restrict__ keep, uint8_t *__restrict__ refg) {
  const int beg = lvl[CAT_INTERNAL * LVL_STRIDE + g.jmin];
  const int n = lvl[CAT_INTERNAL * LVL_STRIDE + g.jmax + 1] - beg;
  for (int i = blockIdx.x * BLK + threadIdx.x; i < n; i += gridDim.x * BLK) {
    const uint32_t e = lst[beg + i];
    const int lp = (int)(e >> LEVEL_SHIFT), l = lp + 1;
    const uint32_t p = e & CELL_MASK;
    int px, py;
    coords<DIM>(lp, p, px, py);
    T dmax = T(0);
    for (int h = 0; h < g.q; ++h) {
      ParentStencil<DIM, T> st;
      st.load(F + foff(g, lp, h), lp, px, py);
      const T *C = F + foff(g, l, h);
      for (int dy = 0; dy < (DIM == 2 ? 2 : 1); ++dy)
        for (int dx = 0; dx < 2; ++dx) {
          const T d = C[cidx<DIM>(l, 2 * px + dx, 2 * py + dy)] - st.child(dx, dy);
          const T a = d < T(0) ? -d : d;
          dmax = a > dmax ? a : dmax;
        }
    }
    if (dmax >= thr.eps_l[l]) {
      uint8_t *k = keep + g.loff[l];
      for (int dy = 0; dy < (DIM == 2 ? 2 : 1); ++dy)
        for (int dx = 0; dx < 2; ++dx) k[cidx<DIM>(l, 2 * px + dx, 2 * py + dy)] = 1;
    }
    if (l > g.jmin && l < g.jmax && dmax >= thr.ref_l[l]) refg[g.loff[lp] + p] = 1;
  }
}

// Ancestor closure of the thresholded set: the group of the parent of every kept
// cell of level l is kept. One thread per cell g of level l-2 looks at its
// 4^d grandchildren.
template <int DIM>
__global__ void __launch_bounds__(BLK) k_ancestor(Geo g, uint8_t *__restrict__ keep, int l) {
  const int lg = l - 2;
  const long long n = ncells(g, lg);
  const uint8_t *kl = keep + g.loff[l];
  uint8_t *kp = keep + g.loff[l - 1];
  for (long long i = blockIdx.x * (long long)BLK + threadIdx.x; i < n; i += (long long)gridDim.x * BLK) {
    int x, y;
    coords<DIM>(lg, (uint32_t)i, x, y);
    bool any = false;
    if (DIM == 1) {
      for (int a = 0; a < 4; ++a) any |= kl[4 * x + a] != 0;
    } else {
      for (int b = 0; b < 4; ++b)
        for (int a = 0; a < 4; ++a) any |= kl[cidx<2>(l, 4 * x + a, 4 * y + b)] != 0;
    }
    if (any)
      for (int dy = 0; dy < (DIM == 2 ? 2 : 1); ++dy)
        for (int dx = 0; dx < 2; ++dx) kp[cidx<DIM>(l - 1, 2 * x + dx, 2 * y + dy)] = 1;
  }
}

// H_eps (section "Construction of the time adaptive mesh"): a cell of level l is
// in the enlarged set if it is kept, if it is k - eta^h for a kept k (eq.
// AdditionNeigh), or if its parent belongs to a group flagged for refinement.
// Level jmin is always complete. One thread per cell of every level.
template <int DIM, int SCHEME>
__global__ void __launch_bounds__(BLK) k_enlarge(Geo g, const uint8_t *__restrict__ keep,
                                                 const uint8_t *__restrict__ refg, uint8_t *__restrict__ tnew) {
  const long long total = g.loff[g.jmax + 1];
  for (long long gc = blockIdx.x * (long long)BLK + threadIdx.x; gc < total; gc += (long long)gridDim.x * BLK) {
    const int l = level_of_cell(g, gc);
    const uint32_t c = (uint32_t)(gc - g.loff[l]);
    uint8_t v = 1;
    if (l > g.jmin) {
      int x, y;
      coords<DIM>(l, c, x, y);
      const uint8_t *kl = keep + g.loff[l];
      v = kl[c];
#pragma unroll
      for (int h = 0; h < Vel<SCHEME>::Q; ++h) {
        constexpr int dummy = 0;
        (void)dummy;
        const int ex = Vel<SCHEME>::ex(h), ey = Vel<SCHEME>::ey(h);
        if (ex == 0 && ey == 0) continue;
        v |= kl[cidx<DIM>(l, wrapl(x + ex, l), wrapl(y + ey, l))];
      }
      if (l >= g.jmin + 2) v |= refg[g.loff[l - 2] + cidx<DIM>(l - 2, x >> 2, y >> 2)];
    }
    tnew[gc] = v ? 1 : 0;
  }
}

// Grading G, level l: every sibling group of level l that has one member gets
// all of them, and every cell of level l-1 whose 3^d box holds a parent of a
// level-l tree cell joins the tree. One thread per cell of level l-1.
template <int DIM>
__global__ void __launch_bounds__(BLK) k_grade(Geo g, uint8_t *__restrict__ tnew, int l) {
  const int lp = l - 1;
  const long long n = ncells(g, lp);
  uint8_t *tl = tnew + g.loff[l];
  uint8_t *tp = tnew + g.loff[lp];
  for (long long i = blockIdx.x * (long long)BLK + threadIdx.x; i < n; i += (long long)gridDim.x * BLK) {
    int x, y;
    coords<DIM>(lp, (uint32_t)i, x, y);
    bool own = false, box = false;
    for (int b = (DIM == 2 ? -1 : 0); b <= (DIM == 2 ? 1 : 0); ++b)
      for (int a = -1; a <= 1; ++a) {
        const int px = wrapl(x + a, lp), py = DIM == 2 ? wrapl(y + b, lp) : 0;
        bool any = false;
        for (int dy = 0; dy < (DIM == 2 ? 2 : 1); ++dy)
          for (int dx = 0; dx < 2; ++dx) any |= tl[cidx<DIM>(l, 2 * px + dx, 2 * py + dy)] != 0;
        box |= any;
        if (a == 0 && b == 0) own = any;
      }
    if (own)
      for (int dy = 0; dy < (DIM == 2 ? 2 : 1); ++dy)
        for (int dx = 0; dx < 2; ++dx) tl[cidx<DIM>(l, 2 * x + dx, 2 * y + dy)] = 1;
    if (box) tp[i] = 1;
  }
}

// Codes of the tree cells of a 0/1 membership array: leaf or internal.
template <int DIM>
__global__ void __launch_bounds__(BLK) k_classify_tree(Geo g, const uint8_t *__restrict__ tnew,
                                                       uint8_t *__restrict__ code) {
  const long long total = g.loff[g.jmax + 1];
  for (long long gc = blockIdx.x * (long long)BLK + threadIdx.x; gc < total; gc += (long long)gridDim.x * BLK) {
    const int l = level_of_cell(g, gc);
    uint8_t v = C_NONE;
    if (tnew[gc]) {
      v = C_LEAF;
      if (l < g.jmax) {
        int x, y;
        coords<DIM>(l, (uint32_t)(gc - g.loff[l]), x, y);
        if (tnew[g.loff[l + 1] + cidx<DIM>(l + 1, 2 * x, 2 * y)]) v = C_INTERNAL;
      }
    }
    code[gc] = v;
  }
}

// Ghost cells of level l (run from the finest level down): a cell outside the
// tree is a ghost if a leaf of its own level lies in its 5^d box (transport and
// transfer stencils), or if it lies in the 3^d parent box of a ghost of level
// l+1 (prediction of that ghost).
template <int DIM>
__global__ void __launch_bounds__(BLK) k_classify_ghost(Geo g, uint8_t *__restrict__ code, int l) {
  const long long n = ncells(g, l);
  uint8_t *cl = code + g.loff[l];
  for (long long i = blockIdx.x * (long long)BLK + threadIdx.x; i < n; i += (long long)gridDim.x * BLK) {
    if (cl[i] != C_NONE) continue;
    int x, y;
    coords<DIM>(l, (uint32_t)i, x, y);
    bool need = false;
    for (int b = (DIM == 2 ? -2 : 0); b <= (DIM == 2 ? 2 : 0) && !need; ++b)
      for (int a = -2; a <= 2; ++a)
        need |= cl[cidx<DIM>(l, wrapl(x + a, l), DIM == 2 ? wrapl(y + b, l) : 0)] == C_LEAF;
    if (!need && l < g.jmax) {
      const uint8_t *cf = code + g.loff[l + 1];
      for (int b = (DIM == 2 ? -2 : 0); b <= (DIM == 2 ? 3 : 0) && !need; ++b)
        for (int a = -2; a <= 3; ++a)
          need |= cf[cidx<DIM>(l + 1, wrapl(2 * x + a, l + 1), DIM == 2 ? wrapl(2 * y + b, l + 1) : 0)] == C_GHOST;
    }
    if (need) cl[i] = C_GHOST;
  }
}

// Codes of the initial full finest mesh: internal below jmax, leaf on jmax.
__global__ void __launch_bounds__(BLK) k_full_tree(Geo g, uint8_t *__restrict__ code) {
  const long long total = g.loff[g.jmax + 1];
  for (long long gc = blockIdx.x * (long long)BLK + threadIdx.x; gc < total; gc += (long long)gridDim.x * BLK)
    code[gc] = gc >= g.loff[g.jmax] ? C_LEAF : C_INTERNAL;
}

__global__ void __launch_bounds__(BLK) k_fill_u32(uint32_t *__restrict__ p, long long n, uint32_t v) {
  for (long long i = blockIdx.x * (long long)BLK + threadIdx.x; i < n; i += (long long)gridDim.x * BLK) p[i] = v;
}

// ---------------------------------------------------------------- compaction
// Lists of leaves, internal cells and ghosts in (level, cell) order: per-block
// counts, one exclusive scan, then a scatter with wavefront ballots.
constexpr int CITER = 4;
constexpr int CCHUNK = BLK * CITER;

__device__ __forceinline__ int block_level(const Geo &g, int b) {
  int l = g.jmin;
  while (l < g.jmax && b >= g.bstart[l + 1]) ++l;
  return l;
}

__device__ __forceinline__ int cat_of(uint8_t v) {
  return v == C_LEAF ? CAT_LEAF : v == C_INTERNAL ? CAT_INTERNAL : v == C_GHOST ? CAT_GHOST : -1;
}

__global__ void __launch_bounds__(BLK) k_compact_count(Geo g, const uint8_t *__restrict__ code,
                                                       int *__restrict__ bcnt) {
  __shared__ int cnt[NCAT];
  const int b = blockIdx.x, l = block_level(g, b);
  const long long nl = ncells(g, l), base = (long long)(b - g.bstart[l]) * CCHUNK;
  if (threadIdx.x < NCAT) cnt[threadIdx.x] = 0;
  __syncthreads();
  int mine[NCAT] = {0, 0, 0};
  for (int it = 0; it < CITER; ++it) {
    const long long c = base + it * BLK + threadIdx.x;
    if (c < nl) {
      const int k = cat_of(code[g.loff[l] + c]);
      if (k >= 0) mine[k]++;
    }
  }
  for (int k = 0; k < NCAT; ++k)
    if (mine[k]) atomicAdd(&cnt[k], mine[k]);
  __syncthreads();
  const int nb = g.bstart[g.jmax + 1];
  if (threadIdx.x < NCAT) bcnt[threadIdx.x * nb + b] = cnt[threadIdx.x];
}

// Single-block exclusive scan of the block counts; level offsets follow.
__global__ void __launch_bounds__(1024) k_compact_scan(Geo g, const int *__restrict__ bcnt, int *__restrict__ boff,
                                                       int *__restrict__ lvl) {
  __shared__ int buf[1024];
  const int nb = g.bstart[g.jmax + 1];
  for (int k = 0; k < NCAT; ++k) {
    int carry = 0;
    for (int base = 0; base < nb; base += 1024) {
      const int i = base + threadIdx.x;
      const int v = i < nb ? bcnt[k * nb + i] : 0;
      buf[threadIdx.x] = v;
      __syncthreads();
      for (int off = 1; off < 1024; off <<= 1) {
        const int t = threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
        __syncthreads();
        buf[threadIdx.x] += t;
        __syncthreads();
      }
      if (i < nb) boff[k * nb + i] = carry + buf[threadIdx.x] - v;
      const int tot = buf[1023];
      __syncthreads();
      carry += tot;
    }
    __syncthreads();
    if (threadIdx.x <= g.jmax + 1) {
      const int l = threadIdx.x;
      int v = 0;
      if (l >= g.jmin) v = g.bstart[l] < nb ? boff[k * nb + g.bstart[l]] : carry;
      if (l == g.jmax + 1) v = carry;
      lvl[k * LVL_STRIDE + l] = v;
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(BLK) k_compact_scatter(Geo g, const uint8_t *__restrict__ code,
                                                         const int *__restrict__ boff, uint32_t *__restrict__ lists,
                                                         long long cap) {
  __shared__ int wcnt[NCAT][BLK / 64];
  const int b = blockIdx.x, l = block_level(g, b);
  const int nb = g.bstart[g.jmax + 1];
  const long long nl = ncells(g, l), base = (long long)(b - g.bstart[l]) * CCHUNK;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long lt = (1ull << lane) - 1ull;
  int off[NCAT];
  for (int k = 0; k < NCAT; ++k) off[k] = boff[k * nb + b];
  for (int it = 0; it < CITER; ++it) {
    const long long c = base + it * BLK + threadIdx.x;
    const int k = c < nl ? cat_of(code[g.loff[l] + c]) : -1;
    int rank[NCAT];
    for (int kk = 0; kk < NCAT; ++kk) {
      const unsigned long long m = __ballot(k == kk);
      rank[kk] = __popcll(m & lt);
      if (lane == 0) wcnt[kk][wave] = __popcll(m);
    }
    __syncthreads();
    for (int kk = 0; kk < NCAT; ++kk) {
      int before = 0, tot = 0;
      for (int w = 0; w < BLK / 64; ++w) {
        before += w < wave ? wcnt[kk][w] : 0;
        tot += wcnt[kk][w];
      }
      if (k == kk) lists[kk * cap + off[kk] + before + rank[kk]] = ((uint32_t)l << LEVEL_SHIFT) | (uint32_t)c;
      off[kk] += tot;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- transfer
// Data of the new complete leaves from the old reconstruction: copy (old leaf),
// projection (merged cell: old internal), prediction (created cell; an old
// ghost already holds it).
template <int DIM, typename T>
__global__ void __launch_bounds__(BLK) k_transfer(Geo g, const T *__restrict__ Fold, T *__restrict__ Fnew,
                                                  const uint8_t *__restrict__ code_old,
                                                  const uint32_t *__restrict__ leaves, const int *__restrict__ lvl) {
  const int beg = lvl[CAT_LEAF * LVL_STRIDE + g.jmin];
  const int n = lvl[CAT_LEAF * LVL_STRIDE + g.jmax + 1] - beg;
  for (int i = blockIdx.x * BLK + threadIdx.x; i < n; i += gridDim.x * BLK) {
    const uint32_t e = leaves[beg + i];
    const int l = (int)(e >> LEVEL_SHIFT);
    const uint32_t c = e & CELL_MASK;
    if (code_old[g.loff[l] + c] != C_NONE) {
      for (int h = 0; h < g.q; ++h) Fnew[foff(g, l, h) + c] = Fold[foff(g, l, h) + c];
    } else {
      int x, y;
      coords<DIM>(l, c, x, y);
      for (int h = 0; h < g.q; ++h) Fnew[foff(g, l, h) + c] = predict<DIM, T>(Fold + foff(g, l - 1, h), l, x, y);
    }
  }
}

// ---------------------------------------------------------------- transport + collision
// MR transport of eq. (AdaptiveAdvectionPhase) on every complete leaf, then the
// collision of eq. (AdaptiveCollision). For a leaf n = J - l > 0 levels above the
// finest, sum_E - sum_A of the reconstruction is the dot product of the leaf
// level's 5^d neighbourhood with the flattened weights W[n][h]
// (eq. PredictionWithMatrixNew), plus, for every neighbour refined one level
// further, its children's details weighted by C[n][h]. Finest leaves stream by
// the plain shift f(k - eta).
template <int DIM, int SCHEME, typename T>
__global__ void __launch_bounds__(BLK) k_transport_collide(Geo g, const T *__restrict__ Fs, T *__restrict__ Fo,
                                                           const uint8_t *__restrict__ code,
                                                           const uint32_t *__restrict__ leaves,
                                                           const int *__restrict__ lvl, const T *__restrict__ Wt,
                                                           const T *__restrict__ Ct, SchemeC<T> sc) {
  using V = Vel<SCHEME>;
  constexpr int Q = V::Q;
  constexpr int WS = DIM == 2 ? 25 : 5, CS = DIM == 2 ? 36 : 6;
  const int beg = lvl[CAT_LEAF * LVL_STRIDE + g.jmin];
  const int nleaf = lvl[CAT_LEAF * LVL_STRIDE + g.jmax + 1] - beg;
  const int J = g.jmax;
  for (int i = blockIdx.x * BLK + threadIdx.x; i < nleaf; i += gridDim.x * BLK) {
    const uint32_t e = leaves[beg + i];
    const int l = (int)(e >> LEVEL_SHIFT);
    const uint32_t c = e & CELL_MASK;
    int x, y;
    coords<DIM>(l, c, x, y);
    const int n = J - l;
    T f[Q];
#pragma unroll
    for (int h = 0; h < Q; ++h) f[h] = Fs[foff(g, l, h) + c];
    if (n == 0) {
#pragma unroll
      for (int h = 0; h < Q; ++h) {
        const int ex = V::ex(h), ey = V::ey(h);
        if (ex == 0 && ey == 0) continue;
        f[h] = Fs[foff(g, J, h) + cidx<DIM>(J, wrapl(x - ex, J), wrapl(y - ey, J))];
      }
    } else {
      // neighbours refined one level further (internal cells of level l)
      const uint8_t *cl = code + g.loff[l];
      unsigned nbr = 0;
      for (int b = (DIM == 2 ? -1 : 0), bit = 0; b <= (DIM == 2 ? 1 : 0); ++b)
        for (int a = -1; a <= 1; ++a) {
          if (a == 0 && b == 0) continue;
          if (cl[cidx<DIM>(l, wrapl(x + a, l), DIM == 2 ? wrapl(y + b, l) : 0)] == C_INTERNAL) nbr |= 1u << bit;
          ++bit;
        }
      const T scale = (T)ldexp(1.0, -DIM * n);
#pragma unroll
      for (int h = 0; h < Q; ++h) {
        const int ex = V::ex(h), ey = V::ey(h);
        if (ex == 0 && ey == 0) continue;
        const T *W = Wt + ((long long)(n - 1) * Q + h) * WS;
        const T *Fl = Fs + foff(g, l, h);
        T acc = T(0);
        if (DIM == 1) {
#pragma unroll
          for (int a = -2; a <= 2; ++a) acc = fma(W[a + 2], Fl[wrapl(x + a, l)], acc);
        } else if (ey == 0) {  // x-axis velocity: the y sums collapse on the leaf's row
          const long long row = (long long)y << l;
#pragma unroll
          for (int a = -2; a <= 2; ++a) acc = fma(W[10 + a + 2], Fl[row + wrapl(x + a, l)], acc);
        } else if (ex == 0) {  // y-axis velocity: the leaf's column
#pragma unroll
          for (int b = -2; b <= 2; ++b) acc = fma(W[(b + 2) * 5 + 2], Fl[((long long)wrapl(y + b, l) << l) + x], acc);
        } else {
#pragma unroll
          for (int b = -2; b <= 2; ++b) {
            const long long row = (long long)wrapl(y + b, l) << l;
#pragma unroll
            for (int a = -2; a <= 2; ++a) acc = fma(W[(b + 2) * 5 + a + 2], Fl[row + wrapl(x + a, l)], acc);
          }
        }
        if (nbr) {
          const T *Cw = Ct + ((long long)(n - 1) * Q + h) * CS;
          const T *Ff = Fs + foff(g, l + 1, h);
          for (int b = (DIM == 2 ? -1 : 0), bit = 0; b <= (DIM == 2 ? 1 : 0); ++b)
            for (int a = -1; a <= 1; ++a) {
              if (a == 0 && b == 0) continue;
              if (nbr & (1u << bit)) {
                const int px = wrapl(x + a, l), py = DIM == 2 ? wrapl(y + b, l) : 0;
                ParentStencil<DIM, T> st;
                st.load(Fl, l, px, py);
                for (int dy = 0; dy < (DIM == 2 ? 2 : 1); ++dy)
                  for (int dx = 0; dx < 2; ++dx) {
                    const T d = Ff[cidx<DIM>(l + 1, 2 * px + dx, 2 * py + dy)] - st.child(dx, dy);
                    const int y1 = 2 * a + dx + 2, y2 = DIM == 2 ? 2 * b + dy + 2 : 0;
                    acc = fma(Cw[y2 * 6 + y1], d, acc);
                  }
              }
              ++bit;
            }
        }
        f[h] = fma(scale, acc, f[h]);
      }
    }
    collide<SCHEME, T>(f, sc);
#pragma unroll
    for (int h = 0; h < Q; ++h) Fo[foff(g, l, h) + c] = f[h];
  }
}

// ---------------------------------------------------------------- init / diagnostics
template <int DIM, int SCHEME, typename T>
__global__ void __launch_bounds__(BLK) k_init_equilibrium(Geo g, T *__restrict__ F, const T *__restrict__ mom,
                                                          SchemeC<T> sc) {
  using V = Vel<SCHEME>;
  const long long n = ncells(g, g.jmax);
  for (long long c = blockIdx.x * (long long)BLK + threadIdx.x; c < n; c += (long long)gridDim.x * BLK) {
    T mc[3], f[V::Q];
    for (int k = 0; k < V::NC; ++k) mc[k] = mom[k * n + c];
    equilibrium_populations<SCHEME, T>(mc, f, sc);
    for (int h = 0; h < V::Q; ++h) F[foff(g, g.jmax, h) + c] = f[h];
  }
}

constexpr int RED_BLOCKS = 256;

// Mass partial sums per block (fixed grid, fixed order => reproducible) and a
// non-finite flag.
template <typename T>
__global__ void __launch_bounds__(BLK) k_mass_partial(Geo g, const T *__restrict__ F,
                                                      const uint32_t *__restrict__ leaves, const int *__restrict__ lvl,
                                                      double *__restrict__ part, int *__restrict__ bad) {
  __shared__ double red[BLK];
  const int beg = lvl[CAT_LEAF * LVL_STRIDE + g.jmin];
  const int n = lvl[CAT_LEAF * LVL_STRIDE + g.jmax + 1] - beg;
  double acc = 0.0;
  int nonfinite = 0;
  for (int i = blockIdx.x * BLK + threadIdx.x; i < n; i += gridDim.x * BLK) {
    const uint32_t e = leaves[beg + i];
    const int l = (int)(e >> LEVEL_SHIFT);
    const uint32_t c = e & CELL_MASK;
    double s = 0.0;
    for (int h = 0; h < g.q; ++h) {
      const double v = (double)F[foff(g, l, h) + c];
      nonfinite |= !isfinite(v);
      s += v;
    }
    acc += ldexp(s, g.dim * (g.jmax - l));
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = BLK / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
  if (nonfinite) atomicOr(bad, 1);
}

template <typename T>
__global__ void __launch_bounds__(BLK) k_export(Geo g, const T *__restrict__ F, const uint32_t *__restrict__ leaves,
                                                const int *__restrict__ lvl, uint32_t *__restrict__ cells,
                                                T *__restrict__ vals) {
  const int beg = lvl[CAT_LEAF * LVL_STRIDE + g.jmin];
  const int n = lvl[CAT_LEAF * LVL_STRIDE + g.jmax + 1] - beg;
  for (int i = blockIdx.x * BLK + threadIdx.x; i < n; i += gridDim.x * BLK) {
    const uint32_t e = leaves[beg + i];
    const int l = (int)(e >> LEVEL_SHIFT);
    const uint32_t c = e & CELL_MASK;
    cells[i] = e;
    for (int h = 0; h < g.q; ++h) vals[(long long)i * g.q + h] = F[foff(g, l, h) + c];
  }
}

}  // namespace mrlbm
