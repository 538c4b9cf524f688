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
__device__ __forceinline__ void project_cell(const Inst<T> &In, T *__restrict__ F, int l, uint32_t c) {
  int x, y, z;
  xyz(l, c, x, y, z);
  uint32_t k[8];
#pragma unroll
  for (int sg = 0; sg < 8; ++sg) k[sg] = child(l, x, y, z, sg);
#pragma unroll
  for (int h = 0; h < Q; ++h) {
    const T *C = pop(In, (const T *)F, l + 1, h);
    T acc = C[k[0]];
#pragma unroll
    for (int sg = 1; sg < 8; ++sg) acc = acc + C[k[sg]];
    pop(In, F, l, h)[c] = T(0.125) * acc;
  }
}
template <typename T>
__global__ void __launch_bounds__(BLK) k3_project(Batch bt, const Inst<T> *__restrict__ I, T *__restrict__ F,
                                                  const uint32_t *__restrict__ lst, const int *__restrict__ lvl,
                                                  int l) {
  __shared__ SegLDS s;
  for_items(s, bt, I, lst, lvl, CAT_INTERNAL, l, [&](const Inst<T> &In, int lv, uint32_t c) { project_cell(In, F, lv, c); });
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
// Byte flags and codes are read and written eight cells at a time: level sizes
// 8^l and every level offset (sums of such sizes, jmin >= 1) are multiples of
// 8, so the 64-bit word of cells [c0, c0 + 8) is aligned and inside the level.
// Words that are all zero (most of a sparse 3D mesh) are skipped at once.
__device__ __forceinline__ uint64_t ld8(const uint8_t *p) { return *reinterpret_cast<const uint64_t *>(p); }
__device__ __forceinline__ void st8(uint8_t *p, uint64_t v) { *reinterpret_cast<uint64_t *>(p) = v; }
__device__ __forceinline__ unsigned byte_of(uint64_t w, int b) { return (unsigned)(w >> (8 * b)) & 0xffu; }
constexpr uint64_t ONES8 = 0x0101010101010101ull;

// Calls f(instance, level, c0) for every word of every level of every instance
// (blocks from binfo: CCHUNK cells of one instance and level each).
template <typename T, typename Fn>
__device__ __forceinline__ void for_all_words(const Inst<T> *__restrict__ I, const uint32_t *__restrict__ binfo,
                                              Fn &&f) {
  int i, l;
  long long base;
  chunk_block(binfo, i, l, base);
  const long long nl = 1ll << (3 * l);
#pragma unroll
  for (int k = 0; k < CCHUNK / 8 / BLK; ++k) {
    const long long c0 = base + 8ll * (threadIdx.x + k * BLK);
    if (c0 >= nl) break;
    f(I[i], l, (uint32_t)c0);
  }
}
// Calls f(instance, c0) for every word of level l of every instance that has
// it (grid.y = instance).
template <typename T, typename Fn>
__device__ __forceinline__ void for_level_words(const Inst<T> *__restrict__ I, int l, Fn &&f) {
  const Inst<T> &In = I[blockIdx.y];
  if (l < In.jmin || l > In.jmax) return;
  const long long c0 = 8ll * ((long long)blockIdx.x * BLK + threadIdx.x);
  if (c0 < (1ll << (3 * l))) f(In, (uint32_t)c0);
}

// Sets the 0/1 flag bytes fl of row (y, z) of level l (l >= 3: a row is a whole
// number of words) given by the 24-bit mask m over x0 - 8 .. x0 + 15 (x0 a
// multiple of 8, periodic): an atomic OR of 1 per byte, with no read, since
// every writer of these bytes only sets them to 1.
__device__ __forceinline__ void or_row(uint8_t *__restrict__ fl, int l, int x0, int y, int z, uint32_t m) {
#pragma unroll
  for (int seg = -1; seg <= 1; ++seg) {
    const uint32_t bits = (m >> (8 * (seg + 1))) & 0xffu;
    if (!bits) continue;
    uint64_t set = 0;
#pragma unroll
    for (int b = 0; b < 8; ++b) set |= (uint64_t)((bits >> b) & 1u) << (8 * b);
    atomicOr(reinterpret_cast<unsigned long long *>(fl + cw(l, x0 + 8 * seg, y, z)), (unsigned long long)set);
  }
}
// Bit b set where byte b of w equals v.
__device__ __forceinline__ uint32_t byte_mask(uint64_t w, unsigned v) {
  uint32_t m = 0;
  for (int b = 0; b < 8; ++b) m |= (byte_of(w, b) == v ? 1u : 0u) << b;
  return m;
}

// T_eps (eq. Thresholding): level jmin always, deeper cells of the old tree
// whose group's detail reached eps_l. Clears the new tree's membership.
template <typename T>
__global__ void __launch_bounds__(BLK) k3_keep(const Inst<T> *__restrict__ I, const uint32_t *__restrict__ binfo,
                                               const uint8_t *__restrict__ code_old, const uint8_t *__restrict__ refg,
                                               uint8_t *__restrict__ keep, uint8_t *__restrict__ tnew) {
  for_all_words(I, binfo, [&](const Inst<T> &In, int l, uint32_t c0) {
    const long long g = In.loff[l] + c0;
    uint64_t kw = 0;
    if (l == In.jmin) {
      kw = ONES8;
    } else {
      const uint64_t ow = ld8(code_old + g);
      if (ow)
        for (int b = 0; b < 8; ++b) {
          if (byte_of(ow, b) < C_INTERNAL) continue;
          int x, y, z;
          xyz(l, c0 + b, x, y, z);
          if (refg[In.loff[l - 1] + cw(l - 1, x >> 1, y >> 1, z >> 1)] & 1) kw |= 1ull << (8 * b);
        }
    }
    st8(keep + g, kw);
    st8(tnew + g, 0);
  });
}

// Ancestor closure, level l (fine to coarse): a kept cell keeps its parent's
// sibling group (the children at level l-1 of its grandparent).
template <typename T>
__device__ __forceinline__ void closure_word(const Inst<T> &In, uint8_t *__restrict__ keep, int l, uint32_t c0) {
  const uint64_t kw = ld8(keep + In.loff[l] + c0);
  if (!kw) return;
  uint8_t *kp = keep + In.loff[l - 1];
  uint32_t last = ~0u;
  for (int b = 0; b < 8; ++b) {
    if (!byte_of(kw, b)) continue;
    int x, y, z;
    xyz(l, c0 + b, x, y, z);
    const uint32_t gp = cw(l - 2, x >> 2, y >> 2, z >> 2);
    if (gp == last) continue;
    last = gp;
#pragma unroll
    for (int sg = 0; sg < 8; ++sg) kp[child(l - 2, x >> 2, y >> 2, z >> 2, sg)] = 1;
  }
}
template <typename T>
__global__ void __launch_bounds__(BLK) k3_closure(const Inst<T> *__restrict__ I, uint8_t *__restrict__ keep, int l) {
  for_level_words(I, l, [&](const Inst<T> &In, uint32_t c0) { closure_word(In, keep, l, c0); });
}

// H_eps (eq. AdditionNeigh and the refinement rule): a kept cell, its
// neighbours c - eta^h along the six velocities, and the children of a kept
// cell of a group whose detail reached 2^{mu_bar + d} eps_l; all of level jmin.
template <typename T>
__global__ void __launch_bounds__(BLK) k3_enlarge(const Inst<T> *__restrict__ I, const uint32_t *__restrict__ binfo,
                                                  const uint8_t *__restrict__ keep, const uint8_t *__restrict__ refg,
                                                  uint8_t *__restrict__ tnew) {
  for_all_words(I, binfo, [&](const Inst<T> &In, int l, uint32_t c0) {
    const long long g = In.loff[l] + c0;
    if (l == In.jmin) st8(tnew + g, ONES8);
    const uint64_t kw = ld8(keep + g);
    if (!kw) return;
    uint8_t *tl = tnew + In.loff[l];
    for (int b = 0; b < 8; ++b) {
      if (!byte_of(kw, b)) continue;
      const uint32_t c = c0 + b;
      int x, y, z;
      xyz(l, c, x, y, z);
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
    }
  });
}

// Grading G at level l (fine to coarse): a new cell completes its sibling group
// and puts the 3^3 box around its parent into level l-1. From level 4 on (level
// l-1 has rows of whole words) the eight cells of a word are handled as bit
// masks: their parents px0 .. px0 + 3 (x0 = 2 px0), the sibling rows of those
// parents and the x-dilated parent rows of the box, each one atomic OR.
template <typename T>
__device__ __forceinline__ void grade_word(const Inst<T> &In, uint8_t *__restrict__ tnew, int l, uint32_t c0) {
  const uint64_t tw = ld8(tnew + In.loff[l] + c0);
  if (!tw) return;
  uint8_t *tl = tnew + In.loff[l], *tp = tnew + In.loff[l - 1];
  int x0, y, z;
  xyz(l, c0, x0, y, z);
  if (l - 1 >= 3) {
    uint32_t P = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) P |= (byte_of(tw, 2 * k) | byte_of(tw, 2 * k + 1)) ? 1u << k : 0u;
    uint64_t S = 0;  // the siblings: both children along x of each parent
#pragma unroll
    for (int k = 0; k < 4; ++k) S |= ((P >> k) & 1u) ? 0x0101ull << (16 * k) : 0ull;
    const int py = y >> 1, pz = z >> 1;
    const int px0 = x0 >> 1, X0 = px0 & ~7;
    const uint32_t Pw = P << (8 + px0 - X0), box = Pw | (Pw << 1) | (Pw >> 1);
    uint64_t sb[3];  // the box's byte masks in the words X0 - 8, X0, X0 + 8 of a row
#pragma unroll
    for (int g = 0; g < 3; ++g) {
      const uint32_t bits = (box >> (8 * g)) & 0xffu;
      uint64_t v = 0;
#pragma unroll
      for (int b = 0; b < 8; ++b) v |= (uint64_t)((bits >> b) & 1u) << (8 * b);
      sb[g] = v;
    }
    // every word first, then an atomic OR only where a flag is still missing
    // (in a refined region most are set already, and the atomics would queue)
    uint8_t *sa[4], *ba[9][3];
    uint64_t sv[4], bv[9][3];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      sa[e] = tl + cw(l, x0, 2 * py + (e & 1), 2 * pz + (e >> 1));
      sv[e] = ld8(sa[e]);
    }
#pragma unroll
    for (int r = 0; r < 9; ++r)
#pragma unroll
      for (int g = 0; g < 3; ++g) {
        ba[r][g] = tp + cw(l - 1, X0 + 8 * (g - 1), py + r % 3 - 1, pz + r / 3 - 1);
        bv[r][g] = sb[g] ? ld8(ba[r][g]) : ~0ull;
      }
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (S & ~sv[e]) atomicOr(reinterpret_cast<unsigned long long *>(sa[e]), (unsigned long long)S);
#pragma unroll
    for (int r = 0; r < 9; ++r)
#pragma unroll
      for (int g = 0; g < 3; ++g)
        if (sb[g] & ~bv[r][g]) atomicOr(reinterpret_cast<unsigned long long *>(ba[r][g]), (unsigned long long)sb[g]);
    return;
  }
  uint32_t last = ~0u;
  for (int b = 0; b < 8; ++b) {
    if (!byte_of(tw, b)) continue;
    int x;
    xyz(l, c0 + b, x, y, z);
    const int px = x >> 1, py = y >> 1, pz = z >> 1;
    const uint32_t pc = cw(l - 1, px, py, pz);
    if (pc == last) continue;
    last = pc;
#pragma unroll
    for (int sg = 0; sg < 8; ++sg) tl[child(l - 1, px, py, pz, sg)] = 1;
    for (int c3 = -1; c3 <= 1; ++c3)
      for (int bb = -1; bb <= 1; ++bb)
        for (int a = -1; a <= 1; ++a) tp[cw(l - 1, px + a, py + bb, pz + c3)] = 1;
  }
}
template <typename T>
__global__ void __launch_bounds__(BLK) k3_grade(const Inst<T> *__restrict__ I, uint8_t *__restrict__ tnew, int l) {
  for_level_words(I, l, [&](const Inst<T> &In, uint32_t c0) { grade_word(In, tnew, l, c0); });
}

// Codes of the new tree: leaf (in the tree, no child in it, or at J),
// internal, or none; the ghost flags gm are cleared (ghost marks follow).
template <typename T>
__global__ void __launch_bounds__(BLK) k3_classify(const Inst<T> *__restrict__ I, const uint32_t *__restrict__ binfo,
                                                   const uint8_t *__restrict__ tnew, uint8_t *__restrict__ code,
                                                   uint8_t *__restrict__ gm) {
  for_all_words(I, binfo, [&](const Inst<T> &In, int l, uint32_t c0) {
    const long long g = In.loff[l] + c0;
    const uint64_t tw = ld8(tnew + g);
    uint64_t v = 0;
    if (tw)
      for (int b = 0; b < 8; ++b) {
        if (!byte_of(tw, b)) continue;
        uint64_t k = C_LEAF;
        if (l < In.jmax) {
          int x, y, z;
          xyz(l, c0 + b, x, y, z);
          if (tnew[In.loff[l + 1] + child(l, x, y, z, 0)]) k = C_INTERNAL;
        }
        v |= k << (8 * b);
      }
    st8(code + g, v);
    st8(gm + g, 0);
  });
}

// Ghost cells of a mesh: the cells outside the tree that the transport, the
// transfer and the ghost predictions read. (a) At the level of every leaf: its
// 3^3 box (the parent stencil of a child created there by the next adaptation)
// and its rows +-2 along the three axes (the transport). (b) Level by level,
// fine to coarse: the 3^3 box at level l-1 around the parent of a ghost of
// level l (its prediction stencil). The marks go to the flag bytes gm (tree
// cells included); a ghost is a cell outside the tree with its flag set, which
// k3_ghost_codes writes into the codes at the end. From level 3 on (rows of
// whole words) the boxes of a word's eight cells are dilated bit masks, one
// atomic OR per row segment; below, cell by cell.
__device__ __forceinline__ uint64_t ghost_bytes(uint64_t code, uint64_t gm) {
  return gm & ~((code >> 1) & ONES8);  // flag set and code C_NONE (tree codes have bit 1)
}
template <typename T>
__device__ __forceinline__ void ghost_leaf_word(const Inst<T> &In, const uint8_t *__restrict__ code,
                                                uint8_t *__restrict__ gm, int l, uint32_t c0) {
  const uint64_t w = ld8(code + In.loff[l] + c0);
  if (!w) return;
  const uint32_t L = byte_mask(w, C_LEAF);
  if (!L) return;
  uint8_t *gl = gm + In.loff[l];
  int x0, y, z;
  xyz(l, c0, x0, y, z);
  if (l >= 3) {
    const uint32_t Lw = L << 8, box = Lw | (Lw << 1) | (Lw >> 1);
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        or_row(gl, l, x0, y + dy, z + dz, (dy == 0 && dz == 0) ? (box | (Lw << 2) | (Lw >> 2)) : box);
    or_row(gl, l, x0, y - 2, z, Lw);
    or_row(gl, l, x0, y + 2, z, Lw);
    or_row(gl, l, x0, y, z - 2, Lw);
    or_row(gl, l, x0, y, z + 2, Lw);
    return;
  }
  for (int b = 0; b < 8; ++b) {
    if (!((L >> b) & 1u)) continue;
    int x;
    xyz(l, c0 + b, x, y, z);
    for (int c3 = -1; c3 <= 1; ++c3)
      for (int bb = -1; bb <= 1; ++bb)
        for (int a = -1; a <= 1; ++a) gl[cw(l, x + a, y + bb, z + c3)] = 1;
    gl[cw(l, x - 2, y, z)] = 1;
    gl[cw(l, x + 2, y, z)] = 1;
    gl[cw(l, x, y - 2, z)] = 1;
    gl[cw(l, x, y + 2, z)] = 1;
    gl[cw(l, x, y, z - 2)] = 1;
    gl[cw(l, x, y, z + 2)] = 1;
  }
}
template <typename T>
__global__ void __launch_bounds__(BLK) k3_ghost_leaf(const Inst<T> *__restrict__ I, const uint32_t *__restrict__ binfo,
                                                     const uint8_t *__restrict__ code, uint8_t *__restrict__ gm) {
  for_all_words(I, binfo, [&](const Inst<T> &In, int l, uint32_t c0) { ghost_leaf_word(In, code, gm, l, c0); });
}
template <typename T>
__device__ __forceinline__ void ghost_up_word(const Inst<T> &In, const uint8_t *__restrict__ code,
                                              uint8_t *__restrict__ gm, int l, uint32_t c0) {
  const long long g = In.loff[l] + c0;
  const uint64_t fw = ld8(gm + g);
  if (!fw) return;
  const uint32_t G = byte_mask(ghost_bytes(ld8(code + g), fw), 1u);
  if (!G) return;
  uint8_t *gp = gm + In.loff[l - 1];
  int x0, y, z;
  xyz(l, c0, x0, y, z);
  if (l - 1 >= 3) {  // the four parents px0 .. px0 + 3 lie in one word of level l-1
    uint32_t P = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) P |= ((G >> (2 * k)) & 3u) ? 1u << k : 0u;
    const int px0 = x0 >> 1, X0 = px0 & ~7;
    const uint32_t Pw = P << (8 + px0 - X0), box = Pw | (Pw << 1) | (Pw >> 1);
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy) or_row(gp, l - 1, X0, (y >> 1) + dy, (z >> 1) + dz, box);
    return;
  }
  uint32_t last = ~0u;
  for (int b = 0; b < 8; ++b) {
    if (!((G >> b) & 1u)) continue;
    int x;
    xyz(l, c0 + b, x, y, z);
    const uint32_t pc = cw(l - 1, x >> 1, y >> 1, z >> 1);
    if (pc == last) continue;
    last = pc;
    for (int c3 = -1; c3 <= 1; ++c3)
      for (int bb = -1; bb <= 1; ++bb)
        for (int a = -1; a <= 1; ++a) gp[cw(l - 1, (x >> 1) + a, (y >> 1) + bb, (z >> 1) + c3)] = 1;
  }
}
template <typename T>
__global__ void __launch_bounds__(BLK) k3_ghost_up(const Inst<T> *__restrict__ I, const uint8_t *__restrict__ code,
                                                   uint8_t *__restrict__ gm, int l) {
  for_level_words(I, l, [&](const Inst<T> &In, uint32_t c0) { ghost_up_word(In, code, gm, l, c0); });
}
// The ghost flags into the codes: C_GHOST where the code is C_NONE and the flag set.
template <typename T>
__global__ void __launch_bounds__(BLK) k3_ghost_codes(const Inst<T> *__restrict__ I, const uint32_t *__restrict__ binfo,
                                                      uint8_t *__restrict__ code, const uint8_t *__restrict__ gm) {
  for_all_words(I, binfo, [&](const Inst<T> &In, int l, uint32_t c0) {
    const long long g = In.loff[l] + c0;
    const uint64_t fw = ld8(gm + g);
    if (fw) {
      const uint64_t cv = ld8(code + g);
      st8(code + g, cv | ghost_bytes(cv, fw));
    }
  });
}

// ---------------------------------------------------------------- coarse levels
// The levels up to lc (at most 8^lc cells each) of a chain in one launch: one
// block of CBLK threads per instance (blockIdx.x), level after level in the
// chain's order with a block barrier between levels.
template <typename T>
__global__ void __launch_bounds__(CBLK) k3_project_coarse(const Inst<T> *__restrict__ I, T *__restrict__ F,
                                                          const uint32_t *__restrict__ lst,
                                                          const int *__restrict__ lvl, int lc) {
  const Inst<T> &In = I[blockIdx.x];
  const int *L = lvl + (blockIdx.x * NCAT + CAT_INTERNAL) * LVL_STRIDE;
  for (int l = min(lc, In.jmax - 1); l >= In.jmin; --l) {
    for (int k = L[l] + (int)threadIdx.x; k < L[l + 1]; k += CBLK) project_cell(In, F, l, lst[k] & CELL_MASK);
    __syncthreads();
  }
}
template <typename T>
__global__ void __launch_bounds__(CBLK) k3_ghost_coarse(const Inst<T> *__restrict__ I, T *__restrict__ F,
                                                        const uint32_t *__restrict__ lst, const int *__restrict__ lvl,
                                                        int lc) {
  const Inst<T> &In = I[blockIdx.x];
  const int *L = lvl + (blockIdx.x * NCAT + CAT_GHOST) * LVL_STRIDE;
  for (int l = In.jmin + 1; l <= min(lc, In.jmax); ++l) {
    for (int k = L[l] + (int)threadIdx.x; k < L[l + 1]; k += CBLK) predict_cell(In, F, l, lst[k] & CELL_MASK);
    __syncthreads();
  }
}
// kind 0: ancestor closure (levels lc .. jmin+2) of `bytes`, 1: grading (lc ..
// jmin+1) of `bytes`, 2: ghost marks (b) (lc .. jmin+1) into the flags `bytes`
// from the codes `code`; fine to coarse.
template <typename T, int KIND>
__global__ void __launch_bounds__(CBLK) k3_dense_coarse(const Inst<T> *__restrict__ I, uint8_t *__restrict__ bytes,
                                                        const uint8_t *__restrict__ code, int lc) {
  const Inst<T> &In = I[blockIdx.x];
  for (int l = min(lc, In.jmax); l >= In.jmin + (KIND == 0 ? 2 : 1); --l) {
    const int words = 1 << (3 * l - 3);
    for (int k = threadIdx.x; k < words; k += CBLK) {
      if (KIND == 0) closure_word(In, bytes, l, 8u * k);
      else if (KIND == 1) grade_word(In, bytes, l, 8u * k);
      else ghost_up_word(In, code, bytes, l, 8u * k);
    }
    __syncthreads();
  }
}

// Calls f(instance, cell) for every cell of level l of every instance that has
// it (grid.y = instance, CPT cells per thread).
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
  });
  if (blockIdx.x == 0 && threadIdx.x == 0) {  // leaf updates and launches, from the segments in LDS
    unsigned long long tot = 0;
    for (int i = 0; i < bt.B; ++i) tot += (unsigned long long)s.cnt[i];
    atomicAdd(&cnt[0], tot);
    atomicAdd(&cnt[1], 1ull);
  }
}

}  // namespace d3
}  // namespace mrlbm
