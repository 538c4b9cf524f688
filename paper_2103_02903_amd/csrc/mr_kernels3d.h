// Kernels of the three-dimensional step (D3Q6 advection, section "Three
// dimensional advection equation", with the d = 3 prediction of section
// "Projection and prediction operators"), gamma = 1, periodic boundaries.
//
// Layout as in two dimensions: level l holds 8^l cells per population, cell
// index x + 2^l (y + 2^l z), list entries (l << 26) | cell. Mesh sets are byte
// codes per cell; the set operations of the adaptation (thresholding, ancestor
// closure, neighbour addition, grading, ghost marking) are dense byte passes,
// the value kernels (projection, prediction, details, transfer, transport +
// collision) walk the compacted lists, one list item per lane with all six
// populations.
//
// The transport of a D3Q6 leaf needs no 3D weight table: every velocity lies
// along one axis a, the prediction is a tensor product whose children of a
// cell average to the cell along each axis, so the sums over the faces of the
// leaf's block B of the finest-level reconstruction collapse, across the two
// other axes, onto the leaf's own row along a. There the one-dimensional
// flattened weights of the D1Q2 velocity of the same sign apply to the row's
// level-l values (offsets -2..2), and a row neighbour at +-1 refined one level
// further corrects them with the 1D details of its two child slabs: the mean of
// the four children of a slab minus the 1D prediction of that slab from the
// row. The grading box keeps any finer level out of reach of E and A.
#pragma once

#include "mr_kernels.h"

namespace mrlbm {
namespace d3 {

constexpr int Q = 6;
constexpr int SCHEME = 5;
constexpr int CPT = 16;  // cells per thread of a dense pass (strided by the block)

__device__ __forceinline__ void xyz(int l, uint32_t c, int &x, int &y, int &z) {
  const uint32_t m = (1u << l) - 1u;
  x = (int)(c & m);
  y = (int)((c >> l) & m);
  z = (int)(c >> (2 * l));
}
// Cell (x, y, z) of level l, every coordinate wrapped (periodic).
__device__ __forceinline__ uint32_t cw(int l, int x, int y, int z) {
  const int m = (1 << l) - 1;
  return (uint32_t)(x & m) | ((uint32_t)(y & m) << l) | ((uint32_t)(z & m) << (2 * l));
}
// Child sigma (bit 0 x, bit 1 y, bit 2 z) of (x, y, z) of level l, at level l+1.
__device__ __forceinline__ uint32_t child(int l, int x, int y, int z, int sigma) {
  const int L = l + 1;
  return (uint32_t)(2 * x + (sigma & 1)) | ((uint32_t)(2 * y + ((sigma >> 1) & 1)) << L) |
         ((uint32_t)(2 * z + ((sigma >> 2) & 1)) << (2 * L));
}

// Prediction of the eight children of a parent (gamma = 1, c_1 = -1/8), the
// d = 3 formula as a tensor product: with P the parent level around (px, py, pz),
//   Qx = c_1 (P(+1,0,0) - P(-1,0,0)), Qy, Qz alike,
//   Qxy = c_1^2 (((P(+,+,0) - P(-,+,0)) - P(+,-,0)) + P(-,-,0)), Qxz, Qyz alike,
//   Qxyz = c_1^3 (((((((P(+++) - P(-++)) - P(+-+)) - P(++-)) + P(--+)) + P(-+-))
//          + P(+--)) - P(---)),
//   child = ((((((P + s_x Qx) + s_y Qy) + s_z Qz) + s_x s_y Qxy) + s_x s_z Qxz)
//           + s_y s_z Qyz) + s_x s_y s_z Qxyz,
// s = +1 for the lower child along an axis and -1 for the upper one. The order
// of evaluation is part of the contract: the details decide the mesh.
template <typename T>
struct Pred3 {
  T f0, qx, qy, qz, qxy, qxz, qyz, qxyz;
  __device__ __forceinline__ void load(const T *__restrict__ P, int lp, int px, int py, int pz) {
    auto at = [&](int a, int b, int t) -> T { return P[cw(lp, px + a, py + b, pz + t)]; };
    const T c1 = T(-0.125), c2 = c1 * c1, c3 = c2 * c1;
    f0 = at(0, 0, 0);
    qx = c1 * (at(1, 0, 0) - at(-1, 0, 0));
    qy = c1 * (at(0, 1, 0) - at(0, -1, 0));
    qz = c1 * (at(0, 0, 1) - at(0, 0, -1));
    qxy = c2 * (((at(1, 1, 0) - at(-1, 1, 0)) - at(1, -1, 0)) + at(-1, -1, 0));
    qxz = c2 * (((at(1, 0, 1) - at(-1, 0, 1)) - at(1, 0, -1)) + at(-1, 0, -1));
    qyz = c2 * (((at(0, 1, 1) - at(0, -1, 1)) - at(0, 1, -1)) + at(0, -1, -1));
    qxyz = c3 * (((((((at(1, 1, 1) - at(-1, 1, 1)) - at(1, -1, 1)) - at(1, 1, -1)) + at(-1, -1, 1)) +
                   at(-1, 1, -1)) + at(1, -1, -1)) - at(-1, -1, -1));
  }
  __device__ __forceinline__ T child(int dx, int dy, int dz) const {
    const T sx = dx ? T(-1) : T(1), sy = dy ? T(-1) : T(1), sz = dz ? T(-1) : T(1);
    return ((((((f0 + sx * qx) + sy * qy) + sz * qz) + (sx * sy) * qxy) + (sx * sz) * qxz) + (sy * sz) * qyz) +
           ((sx * sy) * sz) * qxyz;
  }
};

template <typename T>
__device__ __forceinline__ const T *pop(const Inst<T> &In, const T *F, int l, int h) {
  return F + foff(In, 3, Q, l, h);
}
template <typename T>
__device__ __forceinline__ T *pop(const Inst<T> &In, T *F, int l, int h) {
  return F + foff(In, 3, Q, l, h);
}

// ---------------------------------------------------------------- list kernels
// Calls f(instance, level, cell) for the items of category `cat` at level l
// (l >= 0) or at every level (l < 0), one item per lane, four wavefronts per
// block, all instances in one launch.
template <typename T, typename Fn>
__device__ __forceinline__ void for_items(SegLDS &s, const Batch &bt, const Inst<T> *__restrict__ I,
                                          const uint32_t *__restrict__ lst, const int *__restrict__ lvl, int cat, int l,
                                          Fn &&f) {
  load_segments(s, I, lvl, bt.B, cat, l);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  MRLBM_FOR_CHUNKS(ch, s.pre[bt.B], BLK / 64, wave) {
    const int i = upper_index(s.pre, bt.B, ch);
    const int item = (ch - s.pre[i]) * CHUNK + lane;
    if (item >= s.cnt[i]) continue;
    const uint32_t e = lst[s.beg[i] + item];
    f(I[i], (int)(e >> LEVEL_SHIFT), e & CELL_MASK);
  }
}

// Projection P_nabla on the internal cells of level l: the mean of the eight
// children summed in the order of sigma (x fastest).
template <typename T>
__global__ void __launch_bounds__(BLK) k3_project(Batch bt, const Inst<T> *__restrict__ I, T *__restrict__ F,
                                                  const uint32_t *__restrict__ lst, const int *__restrict__ lvl,
                                                  int l) {
  __shared__ SegLDS s;
  for_items(s, bt, I, lst, lvl, CAT_INTERNAL, l, [&](const Inst<T> &In, int lv, uint32_t c) {
    int x, y, z;
    xyz(lv, c, x, y, z);
    uint32_t k[8];
#pragma unroll
    for (int sg = 0; sg < 8; ++sg) k[sg] = child(lv, x, y, z, sg);
#pragma unroll
    for (int h = 0; h < Q; ++h) {
      const T *C = pop(In, (const T *)F, lv + 1, h);
      T acc = C[k[0]];
#pragma unroll
      for (int sg = 1; sg < 8; ++sg) acc = acc + C[k[sg]];
      pop(In, F, lv, h)[c] = T(0.125) * acc;
    }
  });
}

// Zero-detail prediction on the ghost cells of level l (category cat = ghosts),
// or, for the transfer, on the new leaves of every level that lay outside the
// old mesh (old code C_NONE in code_old).
template <typename T>
__device__ __forceinline__ void predict_cell(const Inst<T> &In, T *__restrict__ F, int l, uint32_t c) {
  int x, y, z;
  xyz(l, c, x, y, z);
#pragma unroll
  for (int h = 0; h < Q; ++h) {
    Pred3<T> p;
    p.load(pop(In, (const T *)F, l - 1, h), l - 1, x >> 1, y >> 1, z >> 1);
    pop(In, F, l, h)[c] = p.child(x & 1, y & 1, z & 1);
  }
}
template <typename T>
__global__ void __launch_bounds__(BLK) k3_ghost(Batch bt, const Inst<T> *__restrict__ I, T *__restrict__ F,
                                                const uint32_t *__restrict__ lst, const int *__restrict__ lvl, int l) {
  __shared__ SegLDS s;
  for_items(s, bt, I, lst, lvl, CAT_GHOST, l, [&](const Inst<T> &In, int lv, uint32_t c) { predict_cell(In, F, lv, c); });
}
template <typename T>
__global__ void __launch_bounds__(BLK) k3_transfer(Batch bt, const Inst<T> *__restrict__ I, T *__restrict__ F,
                                                   const uint32_t *__restrict__ lst, const int *__restrict__ lvl,
                                                   const uint8_t *__restrict__ code_old) {
  __shared__ SegLDS s;
  for_items(s, bt, I, lst, lvl, CAT_LEAF, -1, [&](const Inst<T> &In, int lv, uint32_t c) {
    if (code_old[In.loff[lv] + c] == C_NONE) predict_cell(In, F, lv, c);
  });
}

// Details of every internal cell p (sections "Details and local regularity",
// "Mesh coarsening"): over the populations and the eight children, the max of
// |f_child - prediction| (MET 0) or of 2^{-3} sum_children (f - prediction)^2
// (MET 1, the l2 form kept squared; MET 2: per instance). The thresholds of the
// children's level give the flags of the group: bit 0 keep (eq. Thresholding),
// bit 1 refine (the refinement rule), stored at p in refg.
template <typename T, int MET>
__global__ void __launch_bounds__(BLK) k3_details(Batch bt, const Inst<T> *__restrict__ I, const T *__restrict__ F,
                                                  const uint32_t *__restrict__ lst, const int *__restrict__ lvl,
                                                  uint8_t *__restrict__ refg) {
  __shared__ SegLDS s;
  for_items(s, bt, I, lst, lvl, CAT_INTERNAL, -1, [&](const Inst<T> &In, int lv, uint32_t c) {
    int x, y, z;
    xyz(lv, c, x, y, z);
    const bool l2 = MET == 1 || (MET == 2 && In.metric == 1);
    T dmax = T(0);
    for (int h = 0; h < Q; ++h) {
      Pred3<T> p;
      p.load(pop(In, F, lv, h), lv, x, y, z);
      const T *C = pop(In, F, lv + 1, h);
      T s2 = T(0);
#pragma unroll
      for (int sg = 0; sg < 8; ++sg) {
        const T d = C[child(lv, x, y, z, sg)] - p.child(sg & 1, (sg >> 1) & 1, (sg >> 2) & 1);
        if (l2) s2 = s2 + d * d;
        else if (fabs(d) > dmax) dmax = fabs(d);
      }
      if (l2) {
        s2 = ldexp(s2, -3);
        if (s2 > dmax) dmax = s2;
      }
    }
    refg[In.loff[lv] + c] = (uint8_t)((dmax >= In.eps_l[lv + 1] ? 1 : 0) | (dmax >= In.ref_l[lv + 1] ? 2 : 0));
  });
}

// ---------------------------------------------------------------- dense byte passes
// Calls f(instance, level, cell) for every cell of every level of every
// instance (blocks from binfo: CCHUNK cells of one instance and level each).
template <typename T, typename Fn>
__device__ __forceinline__ void for_all_cells(const Inst<T> *__restrict__ I, const uint32_t *__restrict__ binfo,
                                              Fn &&f) {
  int i, l;
  long long base;
  chunk_block(binfo, i, l, base);
  const long long nl = 1ll << (3 * l);
  for (int k = 0; k < CPT; ++k) {
    const long long c = base + threadIdx.x + (long long)k * BLK;
    if (c >= nl) break;
    f(I[i], l, (uint32_t)c);
  }
}
// Calls f(instance, cell) for every cell of level l of every instance that has
// it (grid.y = instance).
template <typename T, typename Fn>
__device__ __forceinline__ void for_level_cells(const Inst<T> *__restrict__ I, int l, Fn &&f) {
  const Inst<T> &In = I[blockIdx.y];
  if (l < In.jmin || l > In.jmax) return;
  const long long nl = 1ll << (3 * l);
  for (int k = 0; k < CPT; ++k) {
    const long long c = (long long)blockIdx.x * (BLK * CPT) + threadIdx.x + (long long)k * BLK;
    if (c >= nl) break;
    f(In, (uint32_t)c);
  }
}

// T_eps (eq. Thresholding): level jmin always, deeper cells of the old tree
// whose group's detail reached eps_l. Clears the new tree's membership.
template <typename T>
__global__ void __launch_bounds__(BLK) k3_keep(const Inst<T> *__restrict__ I, const uint32_t *__restrict__ binfo,
                                               const uint8_t *__restrict__ code_old, const uint8_t *__restrict__ refg,
                                               uint8_t *__restrict__ keep, uint8_t *__restrict__ tnew) {
  for_all_cells(I, binfo, [&](const Inst<T> &In, int l, uint32_t c) {
    const long long g = In.loff[l] + c;
    uint8_t k = 1;
    if (l > In.jmin) {
      int x, y, z;
      xyz(l, c, x, y, z);
      k = code_old[g] >= C_INTERNAL && (refg[In.loff[l - 1] + cw(l - 1, x >> 1, y >> 1, z >> 1)] & 1) ? 1 : 0;
    }
    keep[g] = k;
    tnew[g] = 0;
  });
}

// Ancestor closure, level l (fine to coarse): a kept cell keeps its parent's
// sibling group (the children at level l-1 of its grandparent).
template <typename T>
__global__ void __launch_bounds__(BLK) k3_closure(const Inst<T> *__restrict__ I, uint8_t *__restrict__ keep, int l) {
  for_level_cells(I, l, [&](const Inst<T> &In, uint32_t c) {
    if (!keep[In.loff[l] + c]) return;
    int x, y, z;
    xyz(l, c, x, y, z);
    uint8_t *kp = keep + In.loff[l - 1];
#pragma unroll
    for (int sg = 0; sg < 8; ++sg) kp[child(l - 2, x >> 2, y >> 2, z >> 2, sg)] = 1;
  });
}

// H_eps (eq. AdditionNeigh and the refinement rule): a kept cell, its
// neighbours c - eta^h along the six velocities, and the children of a kept
// cell of a group whose detail reached 2^{mu_bar + d} eps_l; all of level jmin.
template <typename T>
__global__ void __launch_bounds__(BLK) k3_enlarge(const Inst<T> *__restrict__ I, const uint32_t *__restrict__ binfo,
                                                  const uint8_t *__restrict__ keep, const uint8_t *__restrict__ refg,
                                                  uint8_t *__restrict__ tnew) {
  for_all_cells(I, binfo, [&](const Inst<T> &In, int l, uint32_t c) {
    const long long g = In.loff[l] + c;
    if (l == In.jmin) tnew[g] = 1;
    if (!keep[g]) return;
    int x, y, z;
    xyz(l, c, x, y, z);
    uint8_t *tl = tnew + In.loff[l];
    tl[c] = 1;
    tl[cw(l, x - 1, y, z)] = 1;
    tl[cw(l, x + 1, y, z)] = 1;
    tl[cw(l, x, y - 1, z)] = 1;
    tl[cw(l, x, y + 1, z)] = 1;
    tl[cw(l, x, y, z - 1)] = 1;
    tl[cw(l, x, y, z + 1)] = 1;
    if (l > In.jmin && l < In.jmax && (refg[In.loff[l - 1] + cw(l - 1, x >> 1, y >> 1, z >> 1)] & 2)) {
      uint8_t *tc = tnew + In.loff[l + 1];
#pragma unroll
      for (int sg = 0; sg < 8; ++sg) tc[child(l, x, y, z, sg)] = 1;
    }
  });
}

// Grading G at level l (fine to coarse): a new cell completes its sibling group
// and puts the 3^3 box around its parent into level l-1.
template <typename T>
__global__ void __launch_bounds__(BLK) k3_grade(const Inst<T> *__restrict__ I, uint8_t *__restrict__ tnew, int l) {
  for_level_cells(I, l, [&](const Inst<T> &In, uint32_t c) {
    if (!tnew[In.loff[l] + c]) return;
    int x, y, z;
    xyz(l, c, x, y, z);
    const int px = x >> 1, py = y >> 1, pz = z >> 1;
    uint8_t *tl = tnew + In.loff[l], *tp = tnew + In.loff[l - 1];
#pragma unroll
    for (int sg = 0; sg < 8; ++sg) tl[child(l - 1, px, py, pz, sg)] = 1;
    for (int c3 = -1; c3 <= 1; ++c3)
      for (int b = -1; b <= 1; ++b)
        for (int a = -1; a <= 1; ++a) tp[cw(l - 1, px + a, py + b, pz + c3)] = 1;
  });
}

// Codes of the new tree: leaf (in the tree, no child in it, or at J),
// internal, or none; ghost marks follow.
template <typename T>
__global__ void __launch_bounds__(BLK) k3_classify(const Inst<T> *__restrict__ I, const uint32_t *__restrict__ binfo,
                                                   const uint8_t *__restrict__ tnew, uint8_t *__restrict__ code) {
  for_all_cells(I, binfo, [&](const Inst<T> &In, int l, uint32_t c) {
    const long long g = In.loff[l] + c;
    uint8_t v = C_NONE;
    if (tnew[g]) {
      v = C_LEAF;
      if (l < In.jmax) {
        int x, y, z;
        xyz(l, c, x, y, z);
        if (tnew[In.loff[l + 1] + child(l, x, y, z, 0)]) v = C_INTERNAL;
      }
    }
    code[g] = v;
  });
}

// Ghost cells of a mesh: the cells outside the tree that the transport, the
// transfer and the ghost predictions read. (a) At the level of every leaf: its
// 3^3 box (the parent stencil of a child created there by the next adaptation)
// and its rows +-2 along the three axes (the transport). (b) Level by level,
// fine to coarse: the 3^3 box at level l-1 around the parent of a ghost of
// level l (its prediction stencil).
template <typename T>
__global__ void __launch_bounds__(BLK) k3_ghost_leaf(const Inst<T> *__restrict__ I, const uint32_t *__restrict__ binfo,
                                                     uint8_t *__restrict__ code) {
  for_all_cells(I, binfo, [&](const Inst<T> &In, int l, uint32_t c) {
    uint8_t *cl = code + In.loff[l];
    if (cl[c] != C_LEAF) return;
    int x, y, z;
    xyz(l, c, x, y, z);
    for (int c3 = -1; c3 <= 1; ++c3)
      for (int b = -1; b <= 1; ++b)
        for (int a = -1; a <= 1; ++a) {
          const uint32_t n = cw(l, x + a, y + b, z + c3);
          if (cl[n] == C_NONE) cl[n] = C_GHOST;
        }
    const uint32_t far[6] = {cw(l, x - 2, y, z), cw(l, x + 2, y, z), cw(l, x, y - 2, z),
                             cw(l, x, y + 2, z), cw(l, x, y, z - 2), cw(l, x, y, z + 2)};
#pragma unroll
    for (int k2 = 0; k2 < 6; ++k2)
      if (cl[far[k2]] == C_NONE) cl[far[k2]] = C_GHOST;
  });
}
template <typename T>
__global__ void __launch_bounds__(BLK) k3_ghost_up(const Inst<T> *__restrict__ I, uint8_t *__restrict__ code, int l) {
  for_level_cells(I, l, [&](const Inst<T> &In, uint32_t c) {
    if (code[In.loff[l] + c] != C_GHOST) return;
    int x, y, z;
    xyz(l, c, x, y, z);
    uint8_t *cp = code + In.loff[l - 1];
    for (int c3 = -1; c3 <= 1; ++c3)
      for (int b = -1; b <= 1; ++b)
        for (int a = -1; a <= 1; ++a) {
          const uint32_t n = cw(l - 1, (x >> 1) + a, (y >> 1) + b, (z >> 1) + c3);
          if (cp[n] == C_NONE) cp[n] = C_GHOST;
        }
  });
}

// Every cell of level l outside the tree predicted from level l-1 (the
// double-hat reconstruction on the finest level, level by level).
template <typename T>
__global__ void __launch_bounds__(BLK) k3_predict_outside(const Inst<T> *__restrict__ I, T *__restrict__ F,
                                                          const uint8_t *__restrict__ code, int l) {
  for_level_cells(I, l, [&](const Inst<T> &In, uint32_t c) {
    if (code[In.loff[l] + c] >= C_INTERNAL) return;
    predict_cell(In, F, l, c);
  });
}

// ---------------------------------------------------------------- transport + collision
// MR transport (eq. AdaptiveAdvectionPhase) and collision (eq.
// AdaptiveCollision) of every complete leaf, Fc -> Fn. W / C: the 1D weights
// [n - 1][h][5] and corrections [n - 1][h][6] of the leaf's velocity sign.
template <typename T>
__device__ __forceinline__ T transport_row(const Inst<T> &In, const T *__restrict__ Fc, const uint8_t *__restrict__ cl,
                                           int h, int l, int n, int x, int y, int z, const T *__restrict__ W,
                                           const T *__restrict__ Cw) {
  const int a = h >> 1;  // axis of the velocity
  const int ea = a == 0 ? 1 : 0, eb = a == 1 ? 1 : 0, ec = a == 2 ? 1 : 0;
  const T *Fl = pop(In, Fc, l, h);
  T r[5];
#pragma unroll
  for (int k = -2; k <= 2; ++k) r[k + 2] = Fl[cw(l, x + k * ea, y + k * eb, z + k * ec)];
  T acc = T(0);
#pragma unroll
  for (int k = 0; k < 5; ++k) acc = fma(W[k], r[k], acc);
#pragma unroll
  for (int k = -1; k <= 1; k += 2) {
    const int qx = x + k * ea, qy = y + k * eb, qz = z + k * ec;
    if (cl[cw(l, qx, qy, qz)] != C_INTERNAL) continue;
    // children of the refined neighbour at level l+1, slab delta along the axis
    const int X = 2 * (qx & ((1 << l) - 1)), Y = 2 * (qy & ((1 << l) - 1)), Z = 2 * (qz & ((1 << l) - 1));
    const T *Ff = pop(In, Fc, l + 1, h);
    const T q1 = T(-0.125) * (r[k + 3] - r[k + 1]);
#pragma unroll
    for (int dl = 0; dl < 2; ++dl) {
      T s = T(0);
#pragma unroll
      for (int e2 = 0; e2 < 2; ++e2)
#pragma unroll
        for (int e1 = 0; e1 < 2; ++e1) {
          const int cx = X + (a == 0 ? dl : e1), cy = Y + (a == 1 ? dl : (a == 0 ? e1 : e2));
          const int cz = Z + (a == 2 ? dl : e2);
          s = s + Ff[(uint32_t)cx | ((uint32_t)cy << (l + 1)) | ((uint32_t)cz << (2 * (l + 1)))];
        }
      const T d = T(0.25) * s - (dl ? r[k + 2] - q1 : r[k + 2] + q1);
      acc = fma(Cw[(k + 1) * 2 + dl], d, acc);
    }
  }
  return fma((T)ldexp(1.0, -n), acc, r[2]);
}

template <typename T>
__global__ void __launch_bounds__(BLK) k3_transport_collide(Batch bt, const Inst<T> *__restrict__ I,
                                                            const T *__restrict__ Fc, T *__restrict__ Fn,
                                                            const uint8_t *__restrict__ code,
                                                            const uint32_t *__restrict__ lst,
                                                            const int *__restrict__ lvl, const T *__restrict__ W,
                                                            const T *__restrict__ C,
                                                            unsigned long long *__restrict__ cnt) {
  __shared__ unsigned done;
  if (threadIdx.x == 0) done = 0;
  __syncthreads();
  unsigned mine = 0;
  __shared__ SegLDS s;
  for_items(s, bt, I, lst, lvl, CAT_LEAF, -1, [&](const Inst<T> &In, int lv, uint32_t c) {
    int x, y, z;
    xyz(lv, c, x, y, z);
    const int n = In.jmax - lv;
    const uint8_t *cl = code + In.loff[lv];
    T f[Q];
    if (n == 0) {
#pragma unroll
      for (int h = 0; h < Q; ++h) {
        const T *Fl = pop(In, Fc, lv, h);
        f[h] = Fl[cw(lv, x - Vel<SCHEME>::ex(h), y - Vel<SCHEME>::ey(h), z - Vel<SCHEME>::ez(h))];
      }
    } else {
#pragma unroll
      for (int h = 0; h < Q; ++h) {
        const size_t r = (size_t)(n - 1) * Q + h;
        f[h] = transport_row(In, Fc, cl, h, lv, n, x, y, z, W + r * 5, C + r * 6);
      }
    }
    collide<SCHEME, T>(f, In.sc);
#pragma unroll
    for (int h = 0; h < Q; ++h) pop(In, Fn, lv, h)[c] = f[h];
    ++mine;
  });
  if (mine) atomicAdd(&done, mine);
  __syncthreads();
  if (threadIdx.x == 0 && done) atomicAdd(cnt, (unsigned long long)done);
}

}  // namespace d3
}  // namespace mrlbm
