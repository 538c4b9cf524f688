// Adjoint of the MR-LBM step on frozen meshes (the meshes of a recorded forward
// run): the transposes of the step's linear maps (transfer, reconstruction,
// MR transport) and of the linearised collision, applied in reverse order.
//
//   forward:  f_{n+1} = C(T_new R_new X R_old f_n ; s)
//   adjoint:  a_n = R_old^T X^T R_new^T T_new^T (dC/dh)^T a_{n+1},
//             dJ/ds += (dC/ds)^T a_{n+1}
//
// Scatters of the transposed stencils use atomic adds (the sum order of the
// adjoint fields is not fixed); the gradient with respect to the relaxation
// rates is summed in double through fixed per-block partials.
#pragma once

#include "mr_kernels.h"

namespace mrlbm {

template <typename T>
struct MomentMats {
  T M[81];     // moment matrix, row-major q x q
  T Minv[81];  // its inverse
};

// Prediction stencil of child (cx, cy) at level l: parent-level indices and
// weights with prediction = sum_k w[k] P[idx[k]] (same operator as predict()).
template <int DIM, typename T>
__device__ __forceinline__ int predict_stencil(int l, int cx, int cy, long long *idx, T *w) {
  const int lp = l - 1, px = cx >> 1;
  const T c1 = T(-0.125);
  const T sx = (cx & 1) ? T(-1) : T(1);
  if (DIM == 1) {
    idx[0] = px; w[0] = T(1);
    idx[1] = wrapl(px + 1, lp); w[1] = sx * c1;
    idx[2] = wrapl(px - 1, lp); w[2] = -sx * c1;
    return 3;
  }
  const int py = cy >> 1;
  const T sy = (cy & 1) ? T(-1) : T(1), c2 = sx * sy * T(0.015625);
  const int xm = wrapl(px - 1, lp), xp = wrapl(px + 1, lp), ym = wrapl(py - 1, lp), yp = wrapl(py + 1, lp);
  idx[0] = cidx<2>(lp, px, py); w[0] = T(1);
  idx[1] = cidx<2>(lp, xp, py); w[1] = sx * c1;
  idx[2] = cidx<2>(lp, xm, py); w[2] = -sx * c1;
  idx[3] = cidx<2>(lp, px, yp); w[3] = sy * c1;
  idx[4] = cidx<2>(lp, px, ym); w[4] = -sy * c1;
  idx[5] = cidx<2>(lp, xp, yp); w[5] = c2;
  idx[6] = cidx<2>(lp, xm, yp); w[6] = -c2;
  idx[7] = cidx<2>(lp, xp, ym); w[7] = -c2;
  idx[8] = cidx<2>(lp, xm, ym); w[8] = c2;
  return 9;
}

// d m_eq / d m (rows: equilibrium moments, columns: conserved moments).
template <int SCHEME, typename T>
__device__ __forceinline__ void eq_jacobian(const T *m, const SchemeC<T> &sc, T *Je /* q x q */) {
  constexpr int Q = Vel<SCHEME>::Q;
  for (int k = 0; k < Q * Q; ++k) Je[k] = T(0);
  if constexpr (SCHEME == 1) {
    Je[0] = T(1);
    Je[1 * Q + 0] = sc.eq;
  } else if constexpr (SCHEME == 2) {
    Je[0] = T(1);
    Je[1 * Q + 0] = m[0];
    Je[2 * Q + 0] = sc.eq * sc.lam * sc.lam;
  } else {
    const T rho = m[0], qx = m[1], qy = m[2], cs2 = (sc.lam * sc.lam) / T(3);
    const T ir = T(1) / rho, q2 = qx * qx + qy * qy;
    Je[0] = T(1);
    Je[1 * Q + 1] = T(1);
    Je[2 * Q + 2] = T(1);
    Je[3 * Q + 0] = T(-6) * cs2 - T(3) * q2 * ir * ir;
    Je[3 * Q + 1] = T(6) * qx * ir;
    Je[3 * Q + 2] = T(6) * qy * ir;
    Je[4 * Q + 1] = T(-3) * cs2;
    Je[5 * Q + 2] = T(-3) * cs2;
    Je[6 * Q + 0] = T(9) * (cs2 * cs2 + cs2 * q2 * ir * ir);
    Je[6 * Q + 1] = T(-18) * cs2 * qx * ir;
    Je[6 * Q + 2] = T(-18) * cs2 * qy * ir;
    Je[7 * Q + 0] = -(qx * qx - qy * qy) * ir * ir;
    Je[7 * Q + 1] = T(2) * qx * ir;
    Je[7 * Q + 2] = T(-2) * qy * ir;
    Je[8 * Q + 0] = -qx * qy * ir * ir;
    Je[8 * Q + 1] = qy * ir;
    Je[8 * Q + 2] = qx * ir;
  }
}

template <int SCHEME, typename T>
__device__ __forceinline__ void equilibrium_moments(const T *m, const SchemeC<T> &sc, T *meq) {
  constexpr int Q = Vel<SCHEME>::Q;
  if constexpr (SCHEME == 1) {
    meq[0] = m[0];
    meq[1] = sc.eq * m[0];
  } else if constexpr (SCHEME == 2) {
    meq[0] = m[0];
    meq[1] = T(0.5) * m[0] * m[0];
    meq[2] = sc.eq * (sc.lam * sc.lam) * m[0];
  } else {
    meq[0] = m[0];
    meq[1] = m[1];
    meq[2] = m[2];
    d2q9_equilibrium(m[0], m[1], m[2], sc.lam, meq);
  }
  (void)Q;
}

// ------------------------------------------------------------------ kernels
// Per-leaf loop helper: blocks of 4 wavefronts, one chunk of 64 list items per
// wavefront (segments of one category over all levels, or of one level).
#define MRLBM_CHUNK_LOOP(s, B)                                                                   \
  const int wave_ = threadIdx.x >> 6, lane_ = threadIdx.x & 63;                                 \
  MRLBM_FOR_CHUNKS(ch, (s).pre[(B)], BLK / 64, wave_) {                                            \
    const int i = upper_index((s).pre, (B), ch);                                                \
    const int item = (ch - (s).pre[i]) * CHUNK + lane_;                                         \
    if (item >= (s).cnt[i]) continue;

#define MRLBM_CHUNK_END }

// Adjoint of the collision on the leaves of a mesh: from the pre-collision
// values h (tape) and the adjoint a of the post-collision values, the adjoint of
// h (into hb at the same slots) and per-block partials of dJ/ds_k.
template <int DIM, int SCHEME, typename T>
__global__ void __launch_bounds__(BLK) k_adj_collide(Batch bt, const Inst<T> *__restrict__ I, MomentMats<T> mm,
                                                     const T *__restrict__ h, const T *__restrict__ a,
                                                     T *__restrict__ hb, const uint32_t *__restrict__ leaves,
                                                     const int *__restrict__ lvl, double *__restrict__ spart) {
  constexpr int Q = Vel<SCHEME>::Q;
  __shared__ SegLDS s;
  __shared__ double red[BLK / 64][9];
  load_segments(s, I, lvl, bt.B, CAT_LEAF, -1);
  double sacc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  MRLBM_CHUNK_LOOP(s, bt.B)
  const Inst<T> &In = I[i];
  const uint32_t e = leaves[s.beg[i] + item];
  const int l = (int)(e >> LEVEL_SHIFT);
  const uint32_t c = e & CELL_MASK;
  const long long o = (long long)Q * In.loff[l] + c, st = ncells_d(DIM, l);
  T f[Q], av[Q], m[Q], meq[Q], b[Q], cv[Q], Je[Q * Q];
  for (int k = 0; k < Q; ++k) {
    f[k] = h[o + k * st];
    av[k] = a[o + k * st];
  }
  for (int r = 0; r < Q; ++r) {
    T acc = T(0);
    for (int j = 0; j < Q; ++j) acc += mm.M[r * Q + j] * f[j];
    m[r] = acc;
  }
  equilibrium_moments<SCHEME, T>(m, In.sc, meq);
  eq_jacobian<SCHEME, T>(m, In.sc, Je);
  for (int k = 0; k < Q; ++k) {  // b = M^{-T} a
    T acc = T(0);
    for (int j = 0; j < Q; ++j) acc += mm.Minv[j * Q + k] * av[j];
    b[k] = acc;
  }
  for (int r = 0; r < Q; ++r) {
    T acc = (T(1) - In.sc.s[r]) * b[r];
    for (int k = 0; k < Q; ++k) acc += Je[k * Q + r] * In.sc.s[k] * b[k];
    cv[r] = acc;
  }
  for (int j = 0; j < Q; ++j) {  // hb = M^T c
    T acc = T(0);
    for (int r = 0; r < Q; ++r) acc += mm.M[r * Q + j] * cv[r];
    hb[o + j * st] = acc;
  }
  for (int k = 0; k < Q; ++k) sacc[k] += (double)b[k] * (double)(meq[k] - m[k]);
  MRLBM_CHUNK_END
  // fixed-order reduction: wavefront sums, then the four wavefronts in order
  for (int k = 0; k < 9; ++k) {
    double v = sacc[k];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < 9) {
    double v = 0.0;
    for (int w = 0; w < BLK / 64; ++w) v += red[w][threadIdx.x];
    spart[blockIdx.x * 9 + threadIdx.x] += v;
  }
}

// Transpose of the MR transport, in two launches. First, every cell of the
// mesh (leaf, internal or ghost: the cells a leaf's transport reads at its own
// level) gathers what the leaves of its level took from it: its own value (a
// leaf's identity term), the flattened weights of the leaves within +-2 (their
// 5^d boxes) times 2^{-dn} and the leaves' adjoints hb, or at the finest level
// the leaf it streamed to. A cell and population is written by one thread, so
// no atomics. One population per grid layer (blockIdx.z): a thread's chain of
// dependent memory accesses is then the list entry, the codes of the box, the
// box's adjoints and the update, whatever the number of populations. The
// layer's weights (one row of 5^d per level difference) are staged in LDS.
constexpr int ADJ_GATHER_GRID = 32;
template <int DIM, int SCHEME, typename T>
__global__ void __launch_bounds__(BLK) k_adj_transport_gather(Batch bt, const Inst<T> *__restrict__ I,
                                                              const T *__restrict__ hb, T *__restrict__ gs,
                                                              const uint8_t *__restrict__ code,
                                                              const uint32_t *__restrict__ lists,
                                                              const int *__restrict__ lvl, const T *__restrict__ Wt,
                                                              int nmax) {
  using V = Vel<SCHEME>;
  constexpr int Q = V::Q, WS = DIM == 2 ? 25 : 5;
  constexpr int MAXN = DIM == 2 ? 12 : 24;  // J - jmin: at most 12 in 2D (J <= 13), 24 in 1D (J <= 25)
  __shared__ T Ws[MAXN * WS];
  __shared__ SegLDS s;
  const int hh = blockIdx.z, ex = V::ex(hh), ey = V::ey(hh);
  for (int k = threadIdx.x; k < nmax * WS; k += BLK) Ws[k] = Wt[((k / WS) * Q + hh) * WS + k % WS];
  const int cat = blockIdx.y;  // CAT_LEAF, CAT_INTERNAL, CAT_GHOST
  load_segments(s, I, lvl, bt.B, cat, -1);  // its first barrier also publishes Ws
  const uint32_t *lst = lists + (size_t)cat * bt.ctotal;
  MRLBM_CHUNK_LOOP(s, bt.B)
  const Inst<T> &In = I[i];
  const uint32_t e = lst[s.beg[i] + item];
  const int l = (int)(e >> LEVEL_SHIFT);
  const uint32_t c = e & CELL_MASK;
  int x, y;
  coords<DIM>(l, c, x, y);
  const int J = In.jmax, n = J - l;
  const long long nl = ncells_d(DIM, l);
  const uint8_t *cl = code + In.loff[l];
  auto at = [&](int a, int b) -> long long {
    return cidx<DIM>(l, wrapl(x + a, l), DIM == 2 ? wrapl(y + b, l) : 0);
  };
  // the leaves of the 5^d box around the cell: bit (b + 2) * 5 + (a + 2)
  uint32_t lm = 0;
  for (int b = (DIM == 2 ? -2 : 0); b <= (DIM == 2 ? 2 : 0); ++b)
    for (int a = -2; a <= 2; ++a)
      if (cl[at(a, b)] == C_LEAF) lm |= 1u << ((b + 2) * 5 + a + 2);
  if (!lm) continue;
  const bool own = (lm >> 12) & 1u;
  const T *Hl = hb + (long long)Q * In.loff[l] + hh * nl;
  T acc = T(0);
  if (ex == 0 && ey == 0) {
    if (own) acc = Hl[c];
  } else if (n == 0) {  // the finest leaf c + eta streamed from here
    if ((lm >> ((ey + 2) * 5 + ex + 2)) & 1u) acc = Hl[at(ex, ey)];
  } else {
    const T *W = Ws + (n - 1) * WS;
    // slot k = (b + 2) * 5 + (a + 2): the leaf at offset (-a, -b) weighted this
    // cell with W(a, b); every load first, then the sum in slot order
    T hv[WS];
    bool use[WS];
#pragma unroll
    for (int k = 0; k < WS; ++k) {
      const int a = k % 5 - 2, b = DIM == 2 ? k / 5 - 2 : 0;
      use[k] = ((lm >> ((2 - b) * 5 + 2 - a)) & 1u) && W[k] != T(0);
      hv[k] = use[k] ? Hl[at(-a, -b)] : T(0);
    }
    T sacc = T(0);
#pragma unroll
    for (int k = 0; k < WS; ++k)
      if (use[k]) sacc += W[k] * hv[k];
    acc = (T)ldexp(1.0, -DIM * n) * sacc;
    if (own) acc += Hl[c];
  }
  if (acc != T(0)) gs[(long long)Q * In.loff[l] + hh * nl + c] += acc;
  MRLBM_CHUNK_END
}

// Second, the detail corrections: a leaf next to a finer cell scatters its
// weighted adjoint into that cell's children and, through the prediction they
// were compared with, into the parent level (atomic adds).
template <int DIM, int SCHEME, typename T>
__global__ void __launch_bounds__(BLK) k_adj_transport(Batch bt, const Inst<T> *__restrict__ I,
                                                       const T *__restrict__ hb, T *__restrict__ gs,
                                                       const uint8_t *__restrict__ code,
                                                       const uint32_t *__restrict__ leaves,
                                                       const int *__restrict__ lvl, const T *__restrict__ Ct) {
  using V = Vel<SCHEME>;
  constexpr int Q = V::Q, CS = DIM == 2 ? 36 : 6;
  __shared__ SegLDS s;
  load_segments(s, I, lvl, bt.B, CAT_LEAF, -1);
  MRLBM_CHUNK_LOOP(s, bt.B)
  const Inst<T> &In = I[i];
  const uint32_t e = leaves[s.beg[i] + item];
  const int l = (int)(e >> LEVEL_SHIFT);
  const uint32_t c = e & CELL_MASK;
  const int J = In.jmax, n = J - l;
  if (n == 0) continue;
  int x, y;
  coords<DIM>(l, c, x, y);
  const unsigned nbr = refined_neighbours<DIM>(code + In.loff[l], l, x, y);
  if (!nbr) continue;
  const long long nl = ncells_d(DIM, l);
  for (int hh = 0; hh < Q; ++hh) {
    const int ex = V::ex(hh), ey = V::ey(hh);
    const unsigned m = nbr & correction_mask<DIM>(ex, ey, n);
    if ((ex == 0 && ey == 0) || !m) continue;
    const T v = hb[(long long)Q * In.loff[l] + hh * nl + c];
    const T sv = (T)ldexp(1.0, -DIM * n) * v;
    T *Gl = gs + (long long)Q * In.loff[l] + hh * nl;
    const T *Cw = Ct + ((long long)(n - 1) * Q + hh) * CS;
    T *Gf = gs + (long long)Q * In.loff[l + 1] + hh * ncells_d(DIM, l + 1);
    for (int b = (DIM == 2 ? -1 : 0), bit = 0; b <= (DIM == 2 ? 1 : 0); ++b)
      for (int a = -1; a <= 1; ++a) {
        if (a == 0 && b == 0) continue;
        const int k = bit++;
        if (!(m & (1u << k))) continue;
        const int px = wrapl(x + a, l), py = DIM == 2 ? wrapl(y + b, l) : 0;
        for (int dy = 0; dy < (DIM == 2 ? 2 : 1); ++dy)
          for (int dx = 0; dx < 2; ++dx) {
            const int y1 = 2 * a + dx + 2, y2 = DIM == 2 ? 2 * b + dy + 2 : 0;
            const T cw = Cw[y2 * 6 + y1] * sv;
            if (cw == T(0)) continue;
            const int cx = 2 * px + dx, cy = 2 * py + dy;
            atomicAdd(&Gf[cidx<DIM>(l + 1, cx, cy)], cw);  // the child's own value
            long long idx[9];
            T w[9];
            const int nk = predict_stencil<DIM, T>(l + 1, cx, cy, idx, w);  // minus its prediction
            for (int k2 = 0; k2 < nk; ++k2) atomicAdd(&Gl[idx[k2]], -w[k2] * cw);
          }
      }
  }
  MRLBM_CHUNK_END
}

// Transpose of the ghost prediction of cell c of level l: its adjoint goes to
// the parent's 3^d box at level l-1 (atomic adds) and its slot is cleared. The
// populations are all read before the first write: the slots of the two
// levels are distinct, and the reads then need one memory round trip.
template <int DIM, int Q, typename T>
__device__ __forceinline__ void adj_ghost_cell(const Inst<T> &In, T *__restrict__ G, int l, uint32_t c) {
  int x, y;
  coords<DIM>(l, c, x, y);
  long long idx[9];
  T w[9];
  const int nk = predict_stencil<DIM, T>(l, x, y, idx, w);
  const long long nl = ncells_d(DIM, l), np = ncells_d(DIM, l - 1);
  T *Gl = G + (long long)Q * In.loff[l], *Gp = G + (long long)Q * In.loff[l - 1];
  T v[Q];
#pragma unroll
  for (int hh = 0; hh < Q; ++hh) v[hh] = Gl[hh * nl + c];
#pragma unroll
  for (int hh = 0; hh < Q; ++hh) {
    Gl[hh * nl + c] = T(0);
    for (int k = 0; k < nk; ++k) atomicAdd(&Gp[hh * np + idx[k]], w[k] * v[hh]);
  }
}

// Transpose of the projection onto internal cell c of level l: its adjoint
// times 2^-d goes to its 2^d children (each child has this one parent, so no
// atomics) and its slot is cleared; every read comes before the first write.
template <int DIM, int Q, typename T>
__device__ __forceinline__ void adj_project_cell(const Inst<T> &In, T *__restrict__ G, int l, uint32_t c) {
  constexpr int NCH = DIM == 2 ? 4 : 2;
  const T inv = DIM == 2 ? T(0.25) : T(0.5);
  int x, y;
  coords<DIM>(l, c, x, y);
  const long long nl = ncells_d(DIM, l), nf = ncells_d(DIM, l + 1);
  T *Gl = G + (long long)Q * In.loff[l], *Gc = G + (long long)Q * In.loff[l + 1];
  long long ch[NCH];
  for (int dy = 0; dy < (DIM == 2 ? 2 : 1); ++dy)
    for (int dx = 0; dx < 2; ++dx) ch[dy * 2 + dx] = cidx<DIM>(l + 1, 2 * x + dx, 2 * y + dy);
  T v[Q], cv[Q][NCH];
#pragma unroll
  for (int hh = 0; hh < Q; ++hh) {
    v[hh] = inv * Gl[hh * nl + c];
#pragma unroll
    for (int k = 0; k < NCH; ++k) cv[hh][k] = Gc[hh * nf + ch[k]];
  }
#pragma unroll
  for (int hh = 0; hh < Q; ++hh) {
    Gl[hh * nl + c] = T(0);
#pragma unroll
    for (int k = 0; k < NCH; ++k) Gc[hh * nf + ch[k]] = cv[hh][k] + v[hh];
  }
}

// Transpose of the ghost predictions of level l: push each ghost's adjoint to
// its parent's 3^d box at level l-1 (run from the finest level down).
template <int DIM, int Q, typename T>
__global__ void __launch_bounds__(BLK) k_adj_ghost(Batch bt, const Inst<T> *__restrict__ I, T *__restrict__ G,
                                                   const uint32_t *__restrict__ lst, const int *__restrict__ lvl, int l) {
  __shared__ SegLDS s;
  load_segments(s, I, lvl, bt.B, CAT_GHOST, l);
  MRLBM_CHUNK_LOOP(s, bt.B)
  adj_ghost_cell<DIM, Q, T>(I[i], G, l, lst[s.beg[i] + item] & CELL_MASK);
  MRLBM_CHUNK_END
}

// Transpose of the projections of level l: each internal cell's adjoint goes
// to its 2^d children (run from the coarsest level up).
template <int DIM, int Q, typename T>
__global__ void __launch_bounds__(BLK) k_adj_project(Batch bt, const Inst<T> *__restrict__ I, T *__restrict__ G,
                                                     const uint32_t *__restrict__ lst, const int *__restrict__ lvl,
                                                     int l) {
  __shared__ SegLDS s;
  load_segments(s, I, lvl, bt.B, CAT_INTERNAL, l);
  MRLBM_CHUNK_LOOP(s, bt.B)
  adj_project_cell<DIM, Q, T>(I[i], G, l, lst[s.beg[i] + item] & CELL_MASK);
  MRLBM_CHUNK_END
}

// The coarse levels (up to lc) of both transposes in one launch, one block of
// CBLK threads per instance: the ghost transposes of levels lc .. jmin+1, then
// the projection transposes of levels jmin .. lc-1, with a block barrier after
// each level (the finer ghost levels run before, the finer projection levels
// after).
template <int DIM, int Q, typename T>
__global__ void __launch_bounds__(CBLK) k_adj_coarse(const Inst<T> *__restrict__ I, T *__restrict__ G,
                                                     const uint32_t *__restrict__ lg, const uint32_t *__restrict__ li,
                                                     const int *__restrict__ lvl, int lc) {
  const Inst<T> &In = I[blockIdx.x];
  const int *Lg = lvl + (blockIdx.x * NCAT + CAT_GHOST) * LVL_STRIDE;
  const int *Li = lvl + (blockIdx.x * NCAT + CAT_INTERNAL) * LVL_STRIDE;
  const int top = min(lc, In.jmax);
  for (int l = top; l >= In.jmin + 1; --l) {
    for (int k = Lg[l] + (int)threadIdx.x; k < Lg[l + 1]; k += CBLK) adj_ghost_cell<DIM, Q, T>(In, G, l, lg[k] & CELL_MASK);
    __syncthreads();
  }
  for (int l = In.jmin; l <= top - 1; ++l) {
    for (int k = Li[l] + (int)threadIdx.x; k < Li[l + 1]; k += CBLK) adj_project_cell<DIM, Q, T>(In, G, l, li[k] & CELL_MASK);
    __syncthreads();
  }
}

// Transpose of the transfer: a new leaf that was an old tree or ghost cell read
// the old reconstruction at its own slot; a created one predicted from level l-1.
template <int DIM, int Q, typename T>
__global__ void __launch_bounds__(BLK) k_adj_transfer(Batch bt, const Inst<T> *__restrict__ I,
                                                      const T *__restrict__ gnew, T *__restrict__ gold,
                                                      const uint8_t *__restrict__ code_old,
                                                      const uint32_t *__restrict__ leaves, const int *__restrict__ lvl) {
  __shared__ SegLDS s;
  load_segments(s, I, lvl, bt.B, CAT_LEAF, -1);
  MRLBM_CHUNK_LOOP(s, bt.B)
  const Inst<T> &In = I[i];
  const uint32_t e = leaves[s.beg[i] + item];
  const int l = (int)(e >> LEVEL_SHIFT);
  const uint32_t c = e & CELL_MASK;
  const long long nl = ncells_d(DIM, l);
  if (code_old[In.loff[l] + c] != C_NONE) {
    for (int hh = 0; hh < Q; ++hh) {
      const long long o = (long long)Q * In.loff[l] + hh * nl + c;
      atomicAdd(&gold[o], gnew[o]);
    }
  } else {
    int x, y;
    coords<DIM>(l, c, x, y);
    long long idx[9];
    T w[9];
    const int nk = predict_stencil<DIM, T>(l, x, y, idx, w);
    for (int hh = 0; hh < Q; ++hh) {
      const T v = gnew[(long long)Q * In.loff[l] + hh * nl + c];
      T *Gp = gold + (long long)Q * In.loff[l - 1] + hh * ncells_d(DIM, l - 1);
      for (int k = 0; k < nk; ++k) atomicAdd(&Gp[idx[k]], w[k] * v);
    }
  }
  MRLBM_CHUNK_END
}

// Transpose of the initial datum f = M^{-1} m_eq(m0) on the finest level of
// instance 0: the adjoint of the conserved moments m0 ([nc][N_J^d]).
template <int DIM, int SCHEME, typename T>
__global__ void __launch_bounds__(BLK) k_adj_init(const Inst<T> *__restrict__ I, MomentMats<T> mm,
                                                  const T *__restrict__ f0, const T *__restrict__ a,
                                                  T *__restrict__ mbar) {
  using V = Vel<SCHEME>;
  constexpr int Q = V::Q;
  const Inst<T> &In = I[0];
  const int J = In.jmax;
  const long long n = ncells_d(DIM, J), base = (long long)Q * In.loff[J];
  for (long long c = blockIdx.x * (long long)BLK + threadIdx.x; c < n; c += (long long)gridDim.x * BLK) {
    T m[Q], b[Q], Je[Q * Q];
    for (int r = 0; r < Q; ++r) {
      T acc = T(0);
      for (int j = 0; j < Q; ++j) acc += mm.M[r * Q + j] * f0[base + j * n + c];
      m[r] = acc;
    }
    eq_jacobian<SCHEME, T>(m, In.sc, Je);
    for (int k = 0; k < Q; ++k) {
      T acc = T(0);
      for (int j = 0; j < Q; ++j) acc += mm.Minv[j * Q + k] * a[base + j * n + c];
      b[k] = acc;
    }
    for (int j = 0; j < V::NC; ++j) {
      T acc = T(0);
      for (int k = 0; k < Q; ++k) acc += Je[k * Q + j] * b[k];
      mbar[j * n + c] = acc;
    }
  }
}

}  // namespace mrlbm
