// Kernels of one MR-LBM time step (Algorithm 1 of arXiv 2103.02903) over a
// batch of independent instances.
//
// Every launch serves all instances at once. List kernels (projection, ghost
// prediction, details, transfer, transport) work on chunks of 64 list items of
// one instance; wavefront h of the block handles population h, so loads of a
// wavefront are coalesced along the list and the transport weights are uniform
// across it. Their trip counts come from list lengths the compaction left in
// device memory, so a whole step is enqueued without host synchronisation.
// Byte kernels on the dense cell codes map blocks to instances through static
// tables built at creation.
#pragma once

#include "mr_device.h"

namespace mrlbm {

constexpr int BLK = 256;
constexpr int MAXB = 256;  // instances per batch
constexpr int CHUNK = 64;  // list items per chunk (one per lane)
constexpr int CPT = 16;    // consecutive cells per thread of an all-level dense pass
constexpr int CCHUNK = BLK * CPT;
constexpr int GCHUNK = BLK * 4;  // cells per block of the ghost classification

// Mesh activity of instance i: act[ACT*i] and act[ACT*i+1] hold the finest
// tree level of the last two meshes the compaction built (the current mesh's
// first), act[ACT*i+2] the finest level the current adaptation's refinement
// reaches (0 if none). A new tree is at most as fine as the old one or its
// refinement, and the code buffer the adaptation rewrites holds the mesh before
// the current one, so above active_top every code, membership and flag byte
// the dense passes of an adaptation read or write is zero, and stays zero:
// those passes skip such levels (by induction over the steps, from a state
// where every level is active, as after set_state).
constexpr int ACT = 4;
constexpr int ACT_ALL = 64;  // an entry above every level: all levels active
template <typename T>
__device__ __forceinline__ int active_top(const int *__restrict__ act, const Inst<T> &In, int i) {
  const int a0 = act[ACT * i], a1 = act[ACT * i + 1], r = act[ACT * i + 2];
  const int a = a0 > a1 ? (a0 > r ? a0 : r) : (a1 > r ? a1 : r);
  return a < In.jmax ? a : In.jmax;
}

// ---------------------------------------------------------------- list segments
// Per-instance list segments of one category: of one level (l >= 0) or of all
// levels (l < 0), with the exclusive prefix of their chunk counts.
struct SegLDS {
  int beg[MAXB];
  int cnt[MAXB];
  int pre[MAXB + 1];
};

template <typename T>
__device__ __forceinline__ void load_segments(SegLDS &s, const Inst<T> *__restrict__ I, const int *__restrict__ lvl,
                                              int B, int cat, int l) {
  for (int i = threadIdx.x; i < B; i += blockDim.x) {
    const int *L = lvl + (i * NCAT + cat) * LVL_STRIDE;
    const int jmin = I[i].jmin, jmax = I[i].jmax;
    int b = 0, e = 0;
    if (l < 0) { b = L[jmin]; e = L[jmax + 1]; }
    else if (l >= jmin && l <= jmax) { b = L[l]; e = L[l + 1]; }
    s.beg[i] = b;
    s.cnt[i] = e - b;
  }
  __syncthreads();
  if (threadIdx.x < 64) {  // wavefront 0: scan of ceil(cnt / CHUNK), four instances per lane
    const int lane = threadIdx.x;
    int v[4], sum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = lane * 4 + k;
      v[k] = i < B ? (s.cnt[i] + CHUNK - 1) / CHUNK : 0;
      sum += v[k];
    }
    int incl = sum;
    for (int off = 1; off < 64; off <<= 1) {
      const int t = __shfl_up(incl, off, 64);
      if (lane >= off) incl += t;
    }
    int run = incl - sum;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = lane * 4 + k;
      if (i < B) s.pre[i] = run;
      run += v[k];
    }
    if (lane == 63) s.pre[B] = incl;
  }
  __syncthreads();
}

// Chunk schedule of a list kernel. The hardware deals the blocks of a launch
// round-robin to the 8 XCDs, each with its own L2. Each XCD takes a contiguous
// eighth of the chunks, walked in order, so that list neighbours, whose
// stencils overlap, are read through the same L2. `per_block` chunks per block
// and round; `sub` is this wavefront's slot among them. Grids that are not a
// multiple of 8 fall back to the plain interleaved order.
#ifndef MRLBM_XCD
#define MRLBM_XCD 1
#endif
constexpr int NXCD = 8;
struct ChunkSched {
  int ch, end, stride;
};
// The list work may occupy the first G blocks of a launch that also carries
// other work (G a multiple of 8 keeps the XCD mapping).
// b is the block's index among the G (blockIdx.x unless the launch carries
// two parts; the second starts at a multiple of 8 blocks, so b and blockIdx.x
// agree modulo 8).
__device__ __forceinline__ ChunkSched chunk_sched(int total, int per_block, int sub, int G, int b) {
  if (MRLBM_XCD && G % NXCD == 0) {
    const int x = b % NXCD, slot = b / NXCD;
    const int lo = (int)((long long)total * x / NXCD), hi = (int)((long long)total * (x + 1) / NXCD);
    return {lo + slot * per_block + sub, hi, (G / NXCD) * per_block};
  }
  return {b * per_block + sub, total, G * per_block};
}
#define MRLBM_FOR_CHUNKS_GB(var_, total, per_block, sub, G, b) \
  for (ChunkSched cs_ = chunk_sched((total), (per_block), (sub), (G), (b)); cs_.ch < cs_.end; cs_.ch += cs_.stride) \
    if (const int var_ = cs_.ch; true)
#define MRLBM_FOR_CHUNKS_G(var_, total, per_block, sub, G) \
  MRLBM_FOR_CHUNKS_GB(var_, total, per_block, sub, G, (int)blockIdx.x)
#define MRLBM_FOR_CHUNKS(var_, total, per_block, sub) MRLBM_FOR_CHUNKS_G(var_, total, per_block, sub, (int)gridDim.x)

// ---------------------------------------------------------------- reconstruction
// Projection P_nabla on the internal cells of level l (section "Projection and
// prediction operators"), children read at level l+1 of the same buffer. The
// first G blocks; wavefront h < Q takes population h.
template <int DIM, int Q, typename T>
__device__ __forceinline__ void project_level(SegLDS &s, const Batch &bt, const Inst<T> *__restrict__ I,
                                              T *__restrict__ F, const uint32_t *__restrict__ lst,
                                              const int *__restrict__ lvl, int l, int G, int b) {
  load_segments(s, I, lvl, bt.B, CAT_INTERNAL, l);
  const int h = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (h >= Q) return;
  MRLBM_FOR_CHUNKS_GB(ch, s.pre[bt.B], 1, 0, G, b) {
    const int i = upper_index(s.pre, bt.B, ch);
    const int item = (ch - s.pre[i]) * CHUNK + lane;
    if (item >= s.cnt[i]) continue;
    const uint32_t c = lst[s.beg[i] + item] & CELL_MASK;
    int x, y;
    coords<DIM>(l, c, x, y);
    F[foff(I[i], DIM, Q, l, h) + c] = project<DIM, T>(F + foff(I[i], DIM, Q, l + 1, h), l + 1, x, y);
  }
}
template <int DIM, int Q, typename T>
__global__ void __launch_bounds__(64 * Q) k_project(Batch bt, const Inst<T> *__restrict__ I, T *__restrict__ F,
                                                    const uint32_t *__restrict__ lst, const int *__restrict__ lvl,
                                                    int l) {
  __shared__ SegLDS s;
  project_level<DIM, Q, T>(s, bt, I, F, lst, lvl, l, (int)gridDim.x, (int)blockIdx.x);
}

// Projection of internal cell c of level l in the reconstruction that follows
// an adaptation. F then holds the old mesh's projections, computed at the start
// of the adaptation; since then only cells outside the old tree were written
// (old ghosts, and the transfer into cells the adaptation added). Each value
// that changed carries a mark byte: the new leaves outside the old tree (set by
// the compaction) and, level by level, the internal cells with a marked child.
// An unmarked internal cell with unmarked children belonged to the old mesh
// with the same children, so its old projection is the exact result and it is
// skipped. A parent consumes (zeroes) its children's marks; a stray mark only
// costs a recomputation.
template <int DIM, int Q, typename T>
__device__ __forceinline__ void project_marked(const Inst<T> &In, T *__restrict__ F, uint8_t *__restrict__ mark,
                                               int l, uint32_t c) {
  int x, y;
  coords<DIM>(l, c, x, y);
  uint8_t *mc = mark + In.loff[l + 1];
  const long long r0 = DIM == 1 ? 2ll * x : cidx<2>(l + 1, 2 * x, 2 * y);
  const long long r1 = DIM == 1 ? r0 : cidx<2>(l + 1, 2 * x, 2 * y + 1);
  if (!(mc[r0] | mc[r0 + 1] | mc[r1] | mc[r1 + 1])) return;
  T v[Q];
#pragma unroll
  for (int h = 0; h < Q; ++h) v[h] = project<DIM, T>(F + foff(In, DIM, Q, l + 1, h), l + 1, x, y);
#pragma unroll
  for (int h = 0; h < Q; ++h) F[foff(In, DIM, Q, l, h) + c] = v[h];
  mc[r0] = 0;
  mc[r0 + 1] = 0;
  if (DIM == 2) {
    mc[r1] = 0;
    mc[r1 + 1] = 0;
  }
  if (l > In.jmin) mark[In.loff[l] + c] = 1;
}
// project_marked on the internal cells of level l, one cell (all populations)
// per thread.
template <int DIM, int Q, typename T>
__global__ void __launch_bounds__(BLK) k_project_marked(Batch bt, const Inst<T> *__restrict__ I, T *__restrict__ F,
                                                        const uint32_t *__restrict__ lst, const int *__restrict__ lvl,
                                                        int l, uint8_t *__restrict__ mark) {
  constexpr int WPB = BLK / 64;
  __shared__ SegLDS s;
  load_segments(s, I, lvl, bt.B, CAT_INTERNAL, l);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  MRLBM_FOR_CHUNKS(ch, s.pre[bt.B], WPB, wave) {
    const int i = upper_index(s.pre, bt.B, ch);
    const int item = (ch - s.pre[i]) * CHUNK + lane;
    if (item >= s.cnt[i]) continue;
    project_marked<DIM, Q, T>(I[i], F, mark, l, lst[s.beg[i] + item] & CELL_MASK);
  }
}

// Zero-detail prediction P_delta on the ghost cells of level l, from level l-1.
// The first G blocks; wavefront h < Q takes population h.
template <int DIM, int Q, typename T, int GAM>
__device__ __forceinline__ void ghost_level(SegLDS &s, const Batch &bt, const Inst<T> *__restrict__ I,
                                            T *__restrict__ F, const uint32_t *__restrict__ lst,
                                            const int *__restrict__ lvl, int l, int G, int b) {
  load_segments(s, I, lvl, bt.B, CAT_GHOST, l);
  const int h = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (h >= Q) return;
  MRLBM_FOR_CHUNKS_GB(ch, s.pre[bt.B], 1, 0, G, b) {
    const int i = upper_index(s.pre, bt.B, ch);
    const int item = (ch - s.pre[i]) * CHUNK + lane;
    if (item >= s.cnt[i]) continue;
    const uint32_t c = lst[s.beg[i] + item] & CELL_MASK;
    int x, y;
    coords<DIM>(l, c, x, y);
    F[foff(I[i], DIM, Q, l, h) + c] =
        predict<DIM, T>(F + foff(I[i], DIM, Q, l - 1, h), l, x, y, I[i].walls, gamma_k<GAM>(I[i]));
  }
}
template <int DIM, int Q, typename T, int GAM>
__global__ void __launch_bounds__(64 * Q) k_ghost(Batch bt, const Inst<T> *__restrict__ I, T *__restrict__ F,
                                                  const uint32_t *__restrict__ lst, const int *__restrict__ lvl, int l) {
  __shared__ SegLDS s;
  ghost_level<DIM, Q, T, GAM>(s, bt, I, F, lst, lvl, l, (int)gridDim.x, (int)blockIdx.x);
}

// ---------------------------------------------------------------- paired links
// Two consecutive links of a per-level chain (the second reads what the first
// writes) in one launch: the first takes blocks 0..G0-1, the second the next
// G1. The finest links of the chains are often empty, and a launch costs about
// as much as a nearly empty level; sharing one saves it. The order between the
// links is needed only when both have work (both sides tell from the list
// lengths, which the compaction summarises per mesh in ne[cat][level]): then
// every block of the first publishes its writes (device-scope release) and
// counts itself in sync[0], and every block of the second waits for the count
// and acquires. Blocks are dispatched in increasing order on each XCD, so a
// waiting block never holds back one it waits for.
//
// sync[] (device memory of the context): [0] first-link blocks counted and not
// yet consumed (read as a signed int), [1] second-link blocks that have left,
// [2] the spin budget of one wait, [3] a sticky flag. The last block of the
// second link consumes the launch's G0 counts by subtraction, not by a reset,
// so a first-link block that counts itself late (after a wait gave up) still
// leaves the counter balanced for the next launch. A wait that exhausts its
// budget sets sync[3], which the host reports as MRLBM_ERR_SYNC; the step's
// results are then invalid, but every block still runs to its end.
__device__ __forceinline__ void pair_wait(unsigned *__restrict__ sync, unsigned G0) {
  if (threadIdx.x == 0) {
    const unsigned budget = __hip_atomic_load(sync + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (unsigned spin = 0;; ++spin) {
      if ((int)__hip_atomic_load(sync, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= (int)G0) break;
      if (spin >= budget) {
        atomicOr(sync + 3, 1u);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __threadfence();
  }
  __syncthreads();
}
__device__ __forceinline__ void pair_signal(unsigned *__restrict__ sync) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    atomicAdd(sync, 1u);
  }
}
__device__ __forceinline__ void pair_leave(unsigned *__restrict__ sync, unsigned G0, unsigned G1) {
  __syncthreads();
  if (threadIdx.x == 0 && atomicAdd(sync + 1, 1u) == G1 - 1u) {  // every block has passed its wait
    atomicSub(sync, G0);
    __hip_atomic_store(sync + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}
// KIND 0: projections (levels l0 then l0-1 = l1), 2: marked projections, 1:
// ghost predictions (levels l0 then l0+1 = l1).
template <int DIM, int Q, typename T, int KIND, int GAM>
__global__ void __launch_bounds__(64 * Q) k_pair(Batch bt, const Inst<T> *__restrict__ I, T *__restrict__ F,
                                                 const uint32_t *__restrict__ lst, const int *__restrict__ lvl,
                                                 int l0, int l1, int G0, int G1, unsigned *__restrict__ sync,
                                                 uint8_t *__restrict__ mark, const int *__restrict__ ne) {
  __shared__ SegLDS s;
  const int cat = KIND == 1 ? CAT_GHOST : CAT_INTERNAL;
  const bool second = (int)blockIdx.x >= G0;
  const bool ordered = ne[cat * LVL_STRIDE + l0] && ne[cat * LVL_STRIDE + l1];
  if (second && ordered) pair_wait(sync, (unsigned)G0);
  const int l = second ? l1 : l0, G = second ? G1 : G0, b = second ? (int)blockIdx.x - G0 : (int)blockIdx.x;
  if constexpr (KIND == 0) {
    project_level<DIM, Q, T>(s, bt, I, F, lst, lvl, l, G, b);
  } else if constexpr (KIND == 1) {
    ghost_level<DIM, Q, T, GAM>(s, bt, I, F, lst, lvl, l, G, b);
  } else {  // one internal cell (all populations) per thread, Q chunks per block
    load_segments(s, I, lvl, bt.B, CAT_INTERNAL, l);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    MRLBM_FOR_CHUNKS_GB(ch, s.pre[bt.B], Q, wave, G, b) {
      const int i = upper_index(s.pre, bt.B, ch);
      const int item = (ch - s.pre[i]) * CHUNK + lane;
      if (item >= s.cnt[i]) continue;
      project_marked<DIM, Q, T>(I[i], F, mark, l, lst[s.beg[i] + item] & CELL_MASK);
    }
  }
  if (ordered) {
    if (second) pair_leave(sync, (unsigned)G0, (unsigned)G1);
    else pair_signal(sync);
  }
}

// ---------------------------------------------------------------- mesh adaptation
// The sibling metric of one population's details d = f(child) - prediction,
// children in the order (0,0), (1,0), (0,1), (1,1): the max of |d| (metric 0),
// or the square of the l2 form of the footnote in section "Mesh coarsening",
// 2^{-d} (((d00^2 + d10^2) + d01^2) + d11^2) (metric 1).
template <int DIM, typename T>
__device__ __forceinline__ T sibling_metric(const ParentStencil<DIM, T> &st, const T *__restrict__ C, int l, int px,
                                            int py, int metric) {
  T m = T(0);
  for (int dy = 0; dy < (DIM == 2 ? 2 : 1); ++dy)
    for (int dx = 0; dx < 2; ++dx) {
      const T d = C[cidx<DIM>(l, 2 * px + dx, 2 * py + dy)] - st.child(dx, dy);
      if (metric) {
        m = m + d * d;
      } else {
        const T a = d < T(0) ? -d : d;
        m = a > m ? a : m;
      }
    }
  return metric ? (T)ldexp(m, -DIM) : m;
}

// Details and the sibling metric over all populations (section "Mesh
// coarsening"), per internal cell p (level l-1) of the old tree (MET: the
// batch's metric, 0 max or 1 l2, or 2 for each instance its own): keep the
// children (T_eps, eq. Thresholding) if the metric reaches eps_l, flag the group
// for refinement (H_eps) if it reaches 2^{mu_bar + d} eps_l (both squared for
// the l2 metric).
template <int DIM, int Q, typename T, int GAM, int MET>
__global__ void __launch_bounds__(64 * Q) k_details(Batch bt, const Inst<T> *__restrict__ I, const T *__restrict__ F,
                                                    const uint32_t *__restrict__ lst, const int *__restrict__ lvl,
                                                    uint8_t *__restrict__ keep, uint8_t *__restrict__ refg,
                                                    int *__restrict__ act) {
  __shared__ SegLDS s;
  __shared__ T dm[Q][64];
  load_segments(s, I, lvl, bt.B, CAT_INTERNAL, -1);
  const int h = threadIdx.x >> 6, lane = threadIdx.x & 63;
  MRLBM_FOR_CHUNKS(ch, s.pre[bt.B], 1, 0) {
    const int i = upper_index(s.pre, bt.B, ch);
    const int item = (ch - s.pre[i]) * CHUNK + lane;
    const bool valid = item < s.cnt[i];
    uint32_t e = 0;
    T dmax = T(0);
    if (valid) {
      e = lst[s.beg[i] + item];
      const int lp = (int)(e >> LEVEL_SHIFT), l = lp + 1;
      int px, py;
      coords<DIM>(lp, e & CELL_MASK, px, py);
      ParentStencil<DIM, T> st;
      st.load(F + foff(I[i], DIM, Q, lp, h), lp, px, py, I[i].walls, gamma_k<GAM>(I[i]));
      dmax = sibling_metric<DIM, T>(st, F + foff(I[i], DIM, Q, l, h), l, px, py, MET == 2 ? I[i].metric : MET);
    }
    dm[h][lane] = dmax;
    __syncthreads();
    if (h == 0 && valid) {
      T D = dm[0][lane];
#pragma unroll
      for (int k = 1; k < Q; ++k) D = dm[k][lane] > D ? dm[k][lane] : D;
      const int lp = (int)(e >> LEVEL_SHIFT), l = lp + 1;
      const uint32_t p = e & CELL_MASK;
      int px, py;
      coords<DIM>(lp, p, px, py);
      if (D >= I[i].eps_l[l]) {
        uint8_t *k = keep + I[i].loff[l];
        for (int dy = 0; dy < (DIM == 2 ? 2 : 1); ++dy)
          for (int dx = 0; dx < 2; ++dx) k[cidx<DIM>(l, 2 * px + dx, 2 * py + dy)] = 1;
      }
      if (l > I[i].jmin && l < I[i].jmax && D >= I[i].ref_l[l]) {
        refg[I[i].loff[lp] + p] = 1;
        // its grandchildren join the tree: recorded when finer than the mesh
        if (l + 1 > act[ACT * i]) atomicMax(act + ACT * i + 2, l + 1);
      }
    }
    __syncthreads();
  }
}

// The same per internal parent, one thread per parent and all populations in
// that thread: no block barriers, and the loads of every population can be in
// flight together. Same arithmetic and decisions as k_details.
template <int DIM, int Q, typename T, int GAM, int MET>
__global__ void __launch_bounds__(BLK) k_details_leaf(Batch bt, const Inst<T> *__restrict__ I,
                                                      const T *__restrict__ F, const uint32_t *__restrict__ lst,
                                                      const int *__restrict__ lvl, uint8_t *__restrict__ keep,
                                                      uint8_t *__restrict__ refg, int *__restrict__ act) {
  constexpr int WPB = BLK / 64;
  __shared__ SegLDS s;
  load_segments(s, I, lvl, bt.B, CAT_INTERNAL, -1);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  MRLBM_FOR_CHUNKS(ch, s.pre[bt.B], WPB, wave) {
    const int i = upper_index(s.pre, bt.B, ch);
    const int item = (ch - s.pre[i]) * CHUNK + lane;
    if (item >= s.cnt[i]) continue;
    const Inst<T> &In = I[i];
    const uint32_t e = lst[s.beg[i] + item];
    const int lp = (int)(e >> LEVEL_SHIFT), l = lp + 1;
    const uint32_t p = e & CELL_MASK;
    int px, py;
    coords<DIM>(lp, p, px, py);
    T D = T(0);
#pragma unroll
    for (int h = 0; h < Q; ++h) {
      ParentStencil<DIM, T> st;
      st.load(F + foff(In, DIM, Q, lp, h), lp, px, py, In.walls, gamma_k<GAM>(In));
      const T dmax = sibling_metric<DIM, T>(st, F + foff(In, DIM, Q, l, h), l, px, py, MET == 2 ? In.metric : MET);
      D = h == 0 ? dmax : (dmax > D ? dmax : D);
    }
    if (D >= In.eps_l[l]) {
      uint8_t *k = keep + In.loff[l];
      for (int dy = 0; dy < (DIM == 2 ? 2 : 1); ++dy)
        for (int dx = 0; dx < 2; ++dx) k[cidx<DIM>(l, 2 * px + dx, 2 * py + dy)] = 1;
    }
    if (l > In.jmin && l < In.jmax && D >= In.ref_l[l]) {
      refg[In.loff[lp] + p] = 1;
      // its grandchildren join the tree: recorded when finer than the mesh
      if (l + 1 > act[ACT * i]) atomicMax(act + ACT * i + 2, l + 1);
    }
  }
}

// Block -> (instance, first cell) of a dense pass over one level per instance:
// one static info word per block, instance | (chunk << 8).
__device__ __forceinline__ long long dense_block(const uint32_t *__restrict__ info, int &i) {
  const uint32_t w = info[blockIdx.x];
  i = (int)(w & 0xffu);
  return (long long)(w >> 8) * BLK + threadIdx.x;
}

// Block of an all-level dense pass: CCHUNK cells of one (instance, level), from
// one static info word instance | (level << 8) | (chunk << 13).
__device__ __forceinline__ void chunk_block(const uint32_t *__restrict__ binfo, int &i, int &l, long long &base) {
  const uint32_t w = binfo[blockIdx.x];
  i = (int)(w & 0xffu);
  l = (int)((w >> 8) & 0x1fu);
  base = (long long)(w >> 13) * CCHUNK;
}


// ---------------------------------------------------------------- 16-cell runs
// Sixteen consecutive byte flags or codes of one level as four little-endian
// words. Runs start at multiples of 16 cells; `vec` (uniform per block) says
// that the level is 16-byte aligned and holds at least 16 cells, so a run is
// one 16-byte access. Otherwise bytes at or beyond nl read as 0.
struct Run16 {
  uint32_t w[4];
};
__device__ __forceinline__ Run16 ld16(const uint8_t *__restrict__ p, long long c0, long long nl, bool vec) {
  Run16 r;
  if (vec) {
    const uint4 v = *reinterpret_cast<const uint4 *>(p + c0);
    r.w[0] = v.x; r.w[1] = v.y; r.w[2] = v.z; r.w[3] = v.w;
  } else if (c0 + 16 <= nl && (((uintptr_t)(p + c0)) & 7u) == 0) {  // two 8-byte halves (3D levels)
    const uint2 a = *reinterpret_cast<const uint2 *>(p + c0), b = *reinterpret_cast<const uint2 *>(p + c0 + 8);
    r.w[0] = a.x; r.w[1] = a.y; r.w[2] = b.x; r.w[3] = b.y;
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) r.w[k] = 0;
    for (int t = 0; t < 16; ++t)
      if (c0 + t < nl) r.w[t >> 2] |= (uint32_t)p[c0 + t] << (8 * (t & 3));
  }
  return r;
}
__device__ __forceinline__ void st16(uint8_t *__restrict__ p, long long c0, long long nl, bool vec, const Run16 &r) {
  if (vec) {
    *reinterpret_cast<uint4 *>(p + c0) = make_uint4(r.w[0], r.w[1], r.w[2], r.w[3]);
  } else {
    for (int t = 0; t < 16; ++t)
      if (c0 + t < nl) p[c0 + t] = (uint8_t)(r.w[t >> 2] >> (8 * (t & 3)));
  }
}
// out[t] = in[t + 1], in[16] = next (a byte).
__device__ __forceinline__ Run16 run_next(const Run16 &a, uint32_t next) {
  Run16 r;
  r.w[0] = (a.w[0] >> 8) | (a.w[1] << 24);
  r.w[1] = (a.w[1] >> 8) | (a.w[2] << 24);
  r.w[2] = (a.w[2] >> 8) | (a.w[3] << 24);
  r.w[3] = (a.w[3] >> 8) | (next << 24);
  return r;
}
// out[t] = in[t - 1], in[-1] = prev (a byte).
__device__ __forceinline__ Run16 run_prev(const Run16 &a, uint32_t prev) {
  Run16 r;
  r.w[0] = (a.w[0] << 8) | prev;
  r.w[1] = (a.w[1] << 8) | (a.w[0] >> 24);
  r.w[2] = (a.w[2] << 8) | (a.w[1] >> 24);
  r.w[3] = (a.w[3] << 8) | (a.w[2] >> 24);
  return r;
}
// Bytes 0, 2, 4, 6 of the eight bytes (lo, hi) packed into one word.
__device__ __forceinline__ uint32_t even_bytes(uint32_t lo, uint32_t hi) {
  return (lo & 0xffu) | ((lo >> 8) & 0xff00u) | ((hi & 0xffu) << 16) | ((hi << 8) & 0xff000000u);
}
__device__ __forceinline__ bool level_vec(const uint8_t *p, long long nl) {
  return nl >= 16 && (((uintptr_t)p) & 15u) == 0;
}

// Ancestor closure of the thresholded set: the group of the parent of every kept
// cell of level l is kept. One thread per cell g of level l-2 (its 4^d
// grandchildren are read).
template <int DIM, typename T>
__device__ __forceinline__ bool ancestor_any(const Inst<T> &In, const uint8_t *__restrict__ keep, int l,
                                             long long cell) {
  const int lg = l - 2;
  const uint8_t *kl = keep + In.loff[l];
  int x, y;
  coords<DIM>(lg, (uint32_t)cell, x, y);
  bool any = false;
  if ((((uintptr_t)kl) & 3u) == 0) {  // each grandchild row is one aligned 4-byte word
    for (int b = 0; b < (DIM == 2 ? 4 : 1); ++b)
      any |= *reinterpret_cast<const uint32_t *>(kl + cidx<DIM>(l, 4 * x, 4 * y + b)) != 0;
  } else if (DIM == 1) {
    for (int a = 0; a < 4; ++a) any |= kl[4 * x + a] != 0;
  } else {
    for (int b = 0; b < 4; ++b)
      for (int a = 0; a < 4; ++a) any |= kl[cidx<2>(l, 4 * x + a, 4 * y + b)] != 0;
  }
  return any;
}
template <int DIM, typename T>
__device__ __forceinline__ void ancestor_mark(const Inst<T> &In, uint8_t *__restrict__ keep, int l, long long cell) {
  uint8_t *kp = keep + In.loff[l - 1];
  int x, y;
  coords<DIM>(l - 2, (uint32_t)cell, x, y);
  for (int dy = 0; dy < (DIM == 2 ? 2 : 1); ++dy)
    for (int dx = 0; dx < 2; ++dx) kp[cidx<DIM>(l - 1, 2 * x + dx, 2 * y + dy)] = 1;
}
template <int DIM, typename T>
__device__ __forceinline__ void ancestor_cell(const Inst<T> &In, uint8_t *__restrict__ keep, int l, long long cell) {
  if (ancestor_any<DIM, T>(In, keep, l, cell)) ancestor_mark<DIM, T>(In, keep, l, cell);
}
template <int DIM, typename T>
__global__ void __launch_bounds__(BLK) k_ancestor(Batch bt, const Inst<T> *__restrict__ I, uint8_t *__restrict__ keep,
                                                  const uint32_t *__restrict__ info, int l,
                                                  const int *__restrict__ act) {
  int i;
  const long long cell = dense_block(info, i);
  if (cell >= ncells_d(DIM, l - 2) || l > active_top(act, I[i], i)) return;
  ancestor_cell<DIM, T>(I[i], keep, l, cell);
}

// H_eps (section "Construction of the time adaptive mesh"): a cell of level l is
// in the enlarged set if it is kept, if it is k - eta^h for a kept k (eq.
// AdditionNeigh), or if its parent belongs to a group flagged for refinement.
// Level jmin is always complete. Each thread takes 16 consecutive cells of a
// row: the shifted runs of the rows y + eta_y, ORed (rows of at least 16
// cells), else cell by cell.
template <int DIM, int SCHEME, typename T, bool WALLS>
__global__ void __launch_bounds__(BLK) k_enlarge(Batch bt, const Inst<T> *__restrict__ I,
                                                 const uint32_t *__restrict__ binfo, const uint8_t *__restrict__ keep,
                                                 const uint8_t *__restrict__ refg, uint8_t *__restrict__ tnew,
                                                 const int *__restrict__ act) {
  using V = Vel<SCHEME>;
  int i, l;
  long long base;
  chunk_block(binfo, i, l, base);
  if (l > active_top(act, I[i], i)) return;
  const Inst<T> &In = I[i];
  const long long nl = ncells_d(DIM, l);
  const long long c0 = base + CPT * threadIdx.x;
  if (c0 >= nl) return;
  const uint8_t *kl = keep + In.loff[l];
  const uint8_t *rg = l >= In.jmin + 2 ? refg + In.loff[l - 2] : nullptr;
  uint8_t *tl = tnew + In.loff[l];
  const bool vec = level_vec(kl, nl) && level_vec(tl, nl) && l >= 4;
  Run16 v;
  if (l == In.jmin) {
#pragma unroll
    for (int k = 0; k < 4; ++k) v.w[k] = 0x01010101u;
  } else if (vec) {  // rows (2D) or the level (1D) hold at least 16 cells
    int x0, y;
    coords<DIM>(l, (uint32_t)c0, x0, y);
    v = ld16(kl + cidx<DIM>(l, 0, y), x0, nl, true);  // the kept cells themselves
    const int N = 1 << l;
    const bool wx = WALLS && (In.walls & 1), wy = WALLS && DIM == 2 && (In.walls & 2);
#pragma unroll
    for (int h = 0; h < V::Q; ++h) {
      const int ex = V::ex(h), ey = V::ey(h);
      if (ex == 0 && ey == 0) continue;
      if (wy && (y + ey < 0 || y + ey >= N)) continue;  // beyond a wall: no cell
      const uint8_t *row = kl + cidx<DIM>(l, 0, wrapl(y + ey, l));
      const Run16 a = ld16(row, x0, nl, true);
      // the cell beyond the run: byte 0 of the word after it, or byte 3 of the word
      // before (none beyond a wall)
      const Run16 t =
          ex == 0 ? a
          : ex > 0 ? run_next(a, wx && x0 + 16 >= N ? 0u
                                     : *reinterpret_cast<const uint32_t *>(row + wrapl(x0 + 16, l)) & 0xffu)
                   : run_prev(a, wx && x0 == 0 ? 0u : *reinterpret_cast<const uint32_t *>(row + wrapl(x0 - 4, l)) >> 24);
#pragma unroll
      for (int k = 0; k < 4; ++k) v.w[k] |= t.w[k];
    }
    if (rg) {  // 16 cells have 4 grandparents (x >> 2), one 4-byte word when aligned
      const uint8_t *g = rg + cidx<DIM>(l - 2, x0 >> 2, y >> 2);
      const uint32_t gw = (((uintptr_t)g) & 3u) == 0 ? *reinterpret_cast<const uint32_t *>(g)
                                                     : (uint32_t)g[0] | (uint32_t)g[1] << 8 |
                                                           (uint32_t)g[2] << 16 | (uint32_t)g[3] << 24;
#pragma unroll
      for (int k = 0; k < 4; ++k) v.w[k] |= ((gw >> (8 * k)) & 0xffu) * 0x01010101u;
    }
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) v.w[k] = 0;
    for (int t = 0; t < 16 && c0 + t < nl; ++t) {
      const long long c = c0 + t;
      int x, y;
      coords<DIM>(l, (uint32_t)c, x, y);
      uint32_t b = kl[c];
      const int N = 1 << l;
      for (int h = 0; h < V::Q; ++h) {
        const int sx = x + V::ex(h), sy = y + V::ey(h);
        if (WALLS && (((In.walls & 1) && (sx < 0 || sx >= N)) || (DIM == 2 && (In.walls & 2) && (sy < 0 || sy >= N))))
          continue;
        b |= kl[cidx<DIM>(l, wrapl(sx, l), wrapl(sy, l))];
      }
      if (rg) b |= rg[cidx<DIM>(l - 2, x >> 2, y >> 2)];
      v.w[t >> 2] |= (b ? 1u : 0u) << (8 * (t & 3));
    }
  }
  st16(tl, c0, nl, vec, v);
}

// Grading G, level l: every sibling group of level l with one member gets all
// of them, and every cell of level l-1 whose 3^d box holds a parent of a level-l
// tree cell joins the tree. One thread per cell of level l-1.
template <int DIM, typename T, bool WALLS, int GAM>
__device__ __forceinline__ void grade_cell(const Inst<T> &In, uint8_t *__restrict__ tnew, int l, long long cell) {
  const int lp = l - 1;
  uint8_t *tl = tnew + In.loff[l];
  uint8_t *tp = tnew + In.loff[lp];
  int x, y;
  coords<DIM>(lp, (uint32_t)cell, x, y);
  bool own = false, box = false;
  // beyond a wall there is no parent: the box is clipped there
  const int np = 1 << lp;
  const bool wx = WALLS && (In.walls & 1), wy = WALLS && DIM == 2 && (In.walls & 2);
  const int g = gamma_k<GAM>(In);
  if (g == 1 && (((uintptr_t)tl) & 3u) == 0) {
    // children columns 2x-2 .. 2x+3 of a row: two aligned words (rows of level
    // l >= 2 hold a multiple of 4 cells); pairs -1, 0, +1 at bytes sh .. sh+5
    const int wa = wrapl(2 * x - 2, l) & ~3, wb = wrapl(wa + 4, l), sh = 8 * ((2 * x - 2) & 3);
    unsigned long long keep6 = 0xffffffffffffull;
    if (WALLS) keep6 &= (wx && x == 0 ? ~0xffffull : ~0ull) & (wx && x == np - 1 ? ~0xffff00000000ull : ~0ull);
    for (int b = (DIM == 2 ? -1 : 0); b <= (DIM == 2 ? 1 : 0); ++b) {
      if (WALLS && wy && (y + b < 0 || y + b >= np)) continue;
      for (int dy = 0; dy < (DIM == 2 ? 2 : 1); ++dy) {
        const uint8_t *row = tl + cidx<DIM>(l, 0, DIM == 2 ? wrapl(2 * (y + b) + dy, l) : 0);
        const unsigned long long v = ((unsigned long long)*reinterpret_cast<const uint32_t *>(row + wb) << 32 |
                                      *reinterpret_cast<const uint32_t *>(row + wa)) >> sh;
        box |= (v & keep6) != 0;
        if (b == 0) own |= ((v >> 16) & 0xffffu) != 0;
      }
    }
  } else {
    // box of half-width gamma around the cell (a parent of level l-1)
    for (int b = (DIM == 2 ? -g : 0); b <= (DIM == 2 ? g : 0); ++b)
      for (int a = -g; a <= g; ++a) {
        if (WALLS && ((wx && (x + a < 0 || x + a >= np)) || (wy && (y + b < 0 || y + b >= np)))) continue;
        const int px = wrapl(x + a, lp), py = DIM == 2 ? wrapl(y + b, lp) : 0;
        bool any = false;
        for (int dy = 0; dy < (DIM == 2 ? 2 : 1); ++dy)
          for (int dx = 0; dx < 2; ++dx) any |= tl[cidx<DIM>(l, 2 * px + dx, 2 * py + dy)] != 0;
        box |= any;
        if (a == 0 && b == 0) own = any;
      }
  }
  if (own)
    for (int dy = 0; dy < (DIM == 2 ? 2 : 1); ++dy)
      for (int dx = 0; dx < 2; ++dx) tl[cidx<DIM>(l, 2 * x + dx, 2 * y + dy)] = 1;
  if (box) tp[cell] = 1;
}

// ---------------------------------------------------------------- coarse levels
// The coarse levels of an instance (up to level lc, chosen by the host) are
// walked by one block of CBLK threads per instance, level after level with
// block barriers, in a single launch (a per-level launch costs a few
// microseconds whatever its work). Each level runs the same per-cell
// operations as the per-level kernels; the finer levels keep one launch per
// level.
constexpr int CBLK = 1024;

template <int DIM, typename T>
__device__ void ghost_run4(const Inst<T> &In, uint8_t *__restrict__ code, int l, long long c0);
template <int DIM, typename T>
__device__ void ghost_run16(const Inst<T> &In, uint8_t *__restrict__ code, int l, long long c0);

// Ghost classification of levels min(lc, jmax) .. jmin+1, finest first; bit L
// of v16 selects the 16-cell form for level L.
template <int DIM, typename T>
__global__ void __launch_bounds__(CBLK) k_classify_ghost_coarse(const Inst<T> *__restrict__ I,
                                                                uint8_t *__restrict__ code, int lc,
                                                                unsigned long long v16) {
  const Inst<T> &In = I[blockIdx.x];
  for (int l = lc < In.jmax ? lc : In.jmax; l > In.jmin; --l) {
    const long long nl = ncells_d(DIM, l);
    if ((v16 >> l) & 1ull) {
      for (long long c0 = (long long)threadIdx.x * CPT; c0 < nl; c0 += (long long)CBLK * CPT)
        ghost_run16<DIM, T>(In, code, l, c0);
    } else {
      for (long long c0 = (long long)threadIdx.x * 4; c0 < nl; c0 += (long long)CBLK * 4)
        ghost_run4<DIM, T>(In, code, l, c0);
    }
    __syncthreads();
  }
}

// Ancestor closure for l = min(lc + 2, jmax) .. jmin+2 (cells of level l-2).
template <int DIM, typename T>
__global__ void __launch_bounds__(CBLK) k_ancestor_coarse(const Inst<T> *__restrict__ I, uint8_t *__restrict__ keep,
                                                          int lc) {
  const Inst<T> &In = I[blockIdx.x];
  for (int l = lc + 2 < In.jmax ? lc + 2 : In.jmax; l >= In.jmin + 2; --l) {
    const long long n = ncells_d(DIM, l - 2);
    for (long long cell = threadIdx.x; cell < n; cell += CBLK) ancestor_cell<DIM, T>(In, keep, l, cell);
    __syncthreads();
  }
}

// Ghost predictions of levels jmin+1 .. min(lc, jmax) of instance i, coarsest
// first, by the whole block.
template <int DIM, int Q, typename T, int GAM>
__device__ __forceinline__ void ghost_coarse_walk(const Inst<T> *__restrict__ I, T *__restrict__ F,
                                                  const uint32_t *__restrict__ lst, const int *__restrict__ lvl,
                                                  int lc, int i) {
  const int nt = (int)blockDim.x;
  const Inst<T> &In = I[i];
  const int *L = lvl + (i * NCAT + CAT_GHOST) * LVL_STRIDE;
  for (int l = In.jmin + 1; l <= (lc < In.jmax ? lc : In.jmax); ++l) {
    const int b = L[l], n = L[l + 1] - b;
    if constexpr (sizeof(T) == 4) {
      for (int item = threadIdx.x; item < n; item += nt) {  // all populations per thread, loads before stores
        const uint32_t c = lst[b + item] & CELL_MASK;
        int x, y;
        coords<DIM>(l, c, x, y);
        T v[Q];
#pragma unroll
        for (int h = 0; h < Q; ++h)
          v[h] = predict<DIM, T>(F + foff(In, DIM, Q, l - 1, h), l, x, y, In.walls, gamma_k<GAM>(In));
#pragma unroll
        for (int h = 0; h < Q; ++h) F[foff(In, DIM, Q, l, h) + c] = v[h];
      }
    } else {  // (double: the nine populations' stencils would not fit 128 VGPRs)
      for (int k = threadIdx.x; k < n * Q; k += nt) {  // population-major: lanes on consecutive items
        const int h = k / n, item = k - h * n;
        const uint32_t c = lst[b + item] & CELL_MASK;
        int x, y;
        coords<DIM>(l, c, x, y);
        F[foff(In, DIM, Q, l, h) + c] =
            predict<DIM, T>(F + foff(In, DIM, Q, l - 1, h), l, x, y, In.walls, gamma_k<GAM>(In));
      }
    }
    __syncthreads();
  }
}
// Projection of the internal cells of levels min(lc, jmax-1) .. jmin (with
// mark, only the marked ones: project_marked); with lg, then the ghost
// predictions of levels jmin+1 .. min(lc, jmax) (same block, after the
// projections they read).
template <int DIM, int Q, typename T, int GAM>
__global__ void __launch_bounds__(CBLK) k_project_coarse(const Inst<T> *__restrict__ I, T *__restrict__ F,
                                                         const uint32_t *__restrict__ lst, const int *__restrict__ lvl,
                                                         int lc, const uint32_t *__restrict__ lg,
                                                         uint8_t *__restrict__ mark) {
  const int i = blockIdx.x;
  const Inst<T> &In = I[i];
  const int *L = lvl + (i * NCAT + CAT_INTERNAL) * LVL_STRIDE;
  for (int l = lc < In.jmax - 1 ? lc : In.jmax - 1; l >= In.jmin; --l) {
    const int b = L[l], n = L[l + 1] - b;
    for (int item = threadIdx.x; item < n; item += CBLK) {  // all populations per thread, loads before stores
      const uint32_t c = lst[b + item] & CELL_MASK;
      if (mark) {
        project_marked<DIM, Q, T>(In, F, mark, l, c);
        continue;
      }
      int x, y;
      coords<DIM>(l, c, x, y);
      T v[Q];
#pragma unroll
      for (int h = 0; h < Q; ++h) v[h] = project<DIM, T>(F + foff(In, DIM, Q, l + 1, h), l + 1, x, y);
#pragma unroll
      for (int h = 0; h < Q; ++h) F[foff(In, DIM, Q, l, h) + c] = v[h];
    }
    __syncthreads();
  }
  if (lg) ghost_coarse_walk<DIM, Q, T, GAM>(I, F, lg, lvl, lc, i);
}

// The coarse ancestor closure (blocks 0..B-1) beside the coarse link of the
// old mesh's ghost predictions (blocks B..2B-1), which reads only the old
// mesh's reconstruction: two walks of one block per instance in one launch.
template <int DIM, int Q, typename T, int GAM>
__global__ void __launch_bounds__(CBLK) k_ancestor_ghost_coarse(const Inst<T> *__restrict__ I,
                                                                uint8_t *__restrict__ keep, int lc, int B,
                                                                T *__restrict__ F, const uint32_t *__restrict__ lst,
                                                                const int *__restrict__ lvl) {
  if ((int)blockIdx.x >= B) {
    ghost_coarse_walk<DIM, Q, T, GAM>(I, F, lst, lvl, lc, (int)blockIdx.x - B);
    return;
  }
  const Inst<T> &In = I[blockIdx.x];
  for (int l = lc + 2 < In.jmax ? lc + 2 : In.jmax; l >= In.jmin + 2; --l) {
    const long long n = ncells_d(DIM, l - 2);
    for (long long cell = threadIdx.x; cell < n; cell += CBLK) ancestor_cell<DIM, T>(In, keep, l, cell);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- fused launches
// Two independent chains of a step share launches: each launch runs one link of
// each, in disjoint blocks that touch disjoint data. Blocks hold wavefronts for
// the Q populations of the list work and at least BLK threads for the dense work.
template <int Q>
constexpr int fused_block() { return 64 * Q > BLK ? 64 * Q : BLK; }

// Grading beside the ghost predictions of the old mesh. Grading (blocks G..):
// of level lg, one cell of level lg-1 per thread (block table ginfo), or with
// GC the coarse levels min(lc, jmax) .. jmin+1, one block per instance.
// Ghosts (the first G blocks): of level lh, or with HC the coarse levels
// jmin+1 .. min(lc, jmax), one block per instance. The first writes the
// membership array, the second the values.
template <int DIM, int Q, typename T, bool GC, bool HC, bool WALLS, int GAM>
__global__ void __launch_bounds__(fused_block<Q>())
    k_grade_ghost(Batch bt, const Inst<T> *__restrict__ I, uint8_t *__restrict__ tnew,
                  const uint32_t *__restrict__ ginfo, int lg, T *__restrict__ F, const uint32_t *__restrict__ lst,
                  const int *__restrict__ lvl, int lh, int G, int lc, const int *__restrict__ act) {
  if ((int)blockIdx.x >= G) {
    if (GC) {
      const Inst<T> &In = I[blockIdx.x - G];
      for (int l = lc < In.jmax ? lc : In.jmax; l > In.jmin; --l) {
        const long long n = ncells_d(DIM, l - 1);
        for (long long cell = threadIdx.x; cell < n; cell += blockDim.x) grade_cell<DIM, T, WALLS, GAM>(In, tnew, l, cell);
        __syncthreads();
      }
      return;
    }
    const uint32_t w = ginfo[blockIdx.x - G];
    const int i = (int)(w & 0xffu);
    const long long cell = (long long)(w >> 8) * fused_block<Q>() + threadIdx.x;
    if (cell < ncells_d(DIM, lg - 1) && lg <= active_top(act, I[i], i)) grade_cell<DIM, T, WALLS, GAM>(I[i], tnew, lg, cell);
    return;
  }
  if (HC) {
    ghost_coarse_walk<DIM, Q, T, GAM>(I, F, lst, lvl, lc, (int)blockIdx.x);
    return;
  }
  __shared__ SegLDS s;
  ghost_level<DIM, Q, T, GAM>(s, bt, I, F, lst, lvl, lh, G, (int)blockIdx.x);
}

// Codes of the tree cells of a 0/1 membership array: leaf, or internal when
// its first child is in the tree. Sixteen consecutive cells per thread; their
// first children are the even bytes of 32 cells of the finer row. The same
// cells of the two flag arrays `clear0`, `clear1` (indexed like the codes:
// the keep and refine flags) are zeroed, ready for the next adaptation, where
// the run holds a tree cell: a kept cell belongs to the new tree, and so does
// a cell flagged for refinement (its grandchildren join the tree, and with
// them their ancestors), so flags outside the tree are already zero.
template <int DIM, typename T>
__global__ void __launch_bounds__(BLK) k_classify_tree(Batch bt, const Inst<T> *__restrict__ I,
                                                       const uint32_t *__restrict__ binfo,
                                                       const uint8_t *__restrict__ tnew, uint8_t *__restrict__ code,
                                                       uint8_t *__restrict__ clear0, uint8_t *__restrict__ clear1,
                                                       const int *__restrict__ act) {
  int i, l;
  long long base;
  chunk_block(binfo, i, l, base);
  if (l > active_top(act, I[i], i)) return;
  const Inst<T> &In = I[i];
  const long long nl = ncells_d(DIM, l);
  const long long c0 = base + CPT * threadIdx.x;
  if (c0 >= nl) return;
  const uint8_t *tl = tnew + In.loff[l];
  const uint8_t *tf = l < In.jmax ? tnew + In.loff[l + 1] : nullptr;
  uint8_t *cl = code + In.loff[l];
  const bool vec = level_vec(tl, nl) && level_vec(cl, nl) && (!tf || level_vec(tf, 2 * nl)) && l >= 4;
  const Run16 t = ld16(tl, c0, nl, vec);
  uint32_t ch[4] = {0, 0, 0, 0};
  if (tf) {
    if (vec) {
      int x0, y;
      coords<DIM>(l, (uint32_t)c0, x0, y);
      const uint8_t *row = tf + cidx<DIM>(l + 1, 2 * x0, 2 * y);
      const Run16 a = ld16(row, 0, 16, true), b = ld16(row, 16, 16, true);
      ch[0] = even_bytes(a.w[0], a.w[1]);
      ch[1] = even_bytes(a.w[2], a.w[3]);
      ch[2] = even_bytes(b.w[0], b.w[1]);
      ch[3] = even_bytes(b.w[2], b.w[3]);
    } else {
      for (int k = 0; k < 16 && c0 + k < nl; ++k) {
        int x, y;
        coords<DIM>(l, (uint32_t)(c0 + k), x, y);
        ch[k >> 2] |= (uint32_t)tf[cidx<DIM>(l + 1, 2 * x, 2 * y)] << (8 * (k & 3));
      }
    }
  }
  // per byte (0/1 flags): in tree -> bit 1; in tree without a first child -> bit 0
  Run16 v;
#pragma unroll
  for (int k = 0; k < 4; ++k) v.w[k] = (t.w[k] << 1) | (t.w[k] & ~ch[k]);
  st16(cl, c0, nl, vec, v);
  if (t.w[0] | t.w[1] | t.w[2] | t.w[3]) {
    const Run16 z = {{0, 0, 0, 0}};
    uint8_t *k0 = clear0 + In.loff[l], *k1 = clear1 + In.loff[l];
    st16(k0, c0, nl, level_vec(k0, nl) && l >= 4, z);
    st16(k1, c0, nl, level_vec(k1, nl) && l >= 4, z);
  }
}

// Four consecutive codes starting at p (byte loads if p is not 4-byte aligned).
__device__ __forceinline__ uint32_t load4(const uint8_t *__restrict__ p) {
  if (((uintptr_t)p & 3u) == 0) return *reinterpret_cast<const uint32_t *>(p);
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}
// Bit j set where byte j of w equals v.
__device__ __forceinline__ uint32_t byte_eq_mask(uint32_t w, uint32_t v) {
  uint32_t m = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) m |= (((w >> (8 * j)) & 0xffu) == v ? 1u : 0u) << j;
  return m;
}

// Ghost cells of level l (run from the finest level down): a cell outside the
// tree is a ghost if a leaf of its own level lies in its 5^d box (transport and
// transfer stencils), or if it lies in the 3^d parent box of a ghost of level
// l+1 (prediction of that ghost). Each thread classifies 4 consecutive cells of
// a row (level l >= 2) from aligned 4-cell words of the rows around them.
template <int DIM, typename T>
__device__ __forceinline__ void ghost_run4(const Inst<T> &In, uint8_t *__restrict__ code, int l, long long c0) {
  uint8_t *cl = code + In.loff[l];
  const uint32_t own = load4(cl + c0);
  if (byte_eq_mask(own, C_NONE) == 0) return;
  int x0, y;
  coords<DIM>(l, (uint32_t)c0, x0, y);
  const int nw = (1 << l) >> 2;  // words per row of level l
  const int k = x0 >> 2;
  // leaves of level l: columns x0-4 .. x0+7 (three words) of rows y-2 .. y+2
  uint32_t leafm = 0;
  for (int b = (DIM == 2 ? -2 : 0); b <= (DIM == 2 ? 2 : 0); ++b) {
    const uint8_t *row = cl + (DIM == 2 ? ((long long)wrapl(y + b, l) << l) : 0);
#pragma unroll
    for (int j = 0; j < 3; ++j) leafm |= byte_eq_mask(load4(row + 4 * ((k - 1 + j + nw) % nw)), C_LEAF) << (4 * j);
  }
  // ghosts of level l+1: columns 2x0-4 .. 2x0+11 (four words) of rows 2y-2 .. 2y+3
  uint32_t ghostm = 0;
  if (l < In.jmax) {
    const uint8_t *cf = code + In.loff[l + 1];
    const int lf = l + 1, nwf = 2 * nw;
    for (int b = (DIM == 2 ? -2 : 0); b <= (DIM == 2 ? 3 : 0); ++b) {
      const uint8_t *row = cf + (DIM == 2 ? ((long long)wrapl(2 * y + b, lf) << lf) : 0);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        ghostm |= byte_eq_mask(load4(row + 4 * ((2 * k - 1 + j + nwf) % nwf)), C_GHOST) << (4 * j);
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if (((own >> (8 * t)) & 0xffu) != C_NONE) continue;
    // cell x0+t: leaf columns x0+t-2 .. x0+t+2 -> bits t+2 .. t+6; ghost columns
    // 2(x0+t)-2 .. 2(x0+t)+3 -> bits 2t+2 .. 2t+7
    const bool need = ((leafm >> (t + 2)) & 0x1fu) || ((ghostm >> (2 * t + 2)) & 0x3fu);
    if (need) cl[c0 + t] = C_GHOST;
  }
}
template <int DIM, typename T>
__global__ void __launch_bounds__(BLK) k_classify_ghost(Batch bt, const Inst<T> *__restrict__ I,
                                                        uint8_t *__restrict__ code, const uint32_t *__restrict__ info,
                                                        int l, const int *__restrict__ act) {
  const uint32_t w = info[blockIdx.x];
  const int i = (int)(w & 0xffu);
  const long long c0 = ((long long)(w >> 8) * BLK + threadIdx.x) * 4;
  if (c0 >= ncells_d(DIM, l) || l > active_top(act, I[i], i)) return;
  ghost_run4<DIM, T>(I[i], code, l, c0);
}

// The same classification for a prediction of half-width gamma > 1 (a leaf of
// level l within 2 gamma, or a ghost of level l+1 whose parent lies within
// gamma), for a tile of TX x TY cells of level l per block, through LDS: the leaf flags of the tile with a halo of R = 2 gamma cells,
// dilated by R along x and then along y, and the ghost flags of level l+1 under
// the parents within gamma of the tile, folded to their parents and dilated by
// gamma; a cell outside the tree whose dilated flags hold is a ghost. Boxes
// wrap periodically (the superset noted above with walls). info[block] =
// instance | tile << 8 (tiles row-major over the level).
constexpr int GT_X = 64, GT_Y = 16, GT_R = 6;  // tile size and the largest 2 gamma
template <int DIM, typename T>
__global__ void __launch_bounds__(BLK) k_classify_ghost_tile(Batch bt, const Inst<T> *__restrict__ I,
                                                             uint8_t *__restrict__ code,
                                                             const uint32_t *__restrict__ info, int l,
                                                             const int *__restrict__ act) {
  constexpr int TX = DIM == 2 ? GT_X : GT_X * GT_Y, TY = DIM == 2 ? GT_Y : 1;
  constexpr int HX = TX + 2 * GT_R, HY = DIM == 2 ? TY + 2 * GT_R : 1;            // leaf flags with halo
  constexpr int CX = 2 * (TX + GT_R), CY = DIM == 2 ? 2 * (TY + GT_R) : 1;        // children under the parents
  constexpr int PX = TX + GT_R, PY = DIM == 2 ? TY + GT_R : 1;                    // those parents
  __shared__ uint8_t lf[HY][HX], hx[HY][TX], cf[CY][CX], pf[PY][PX], px_[PY][TX];
  const uint32_t w = info[blockIdx.x];
  const int i = (int)(w & 0xffu);
  const Inst<T> &In = I[i];
  if (l > active_top(act, In, i)) return;  // (uniform over the block)
  const int N = 1 << l, g = In.gamma, R = 2 * g;
  const int ntx = (N + TX - 1) / TX, tile = (int)(w >> 8);
  const int x0 = (tile % ntx) * TX, y0 = DIM == 2 ? (tile / ntx) * TY : 0;
  uint8_t *cl = code + In.loff[l];
  const bool finer = l < In.jmax;
  const uint8_t *cfl = finer ? code + In.loff[l + 1] : nullptr;
  const int RY = DIM == 2 ? TY + 2 * R : 1;  // rows of the leaf flags
  // leaf flags of rows y0-R .. y0+TY-1+R, columns x0-R .. x0+TX-1+R
  for (int k = threadIdx.x; k < RY * (TX + 2 * R); k += BLK) {
    const int r = k / (TX + 2 * R), q = k - r * (TX + 2 * R);
    const int x = wrapl(x0 - R + q, l), y = DIM == 2 ? wrapl(y0 - R + r, l) : 0;
    lf[r][q] = cl[cidx<DIM>(l, x, y)] == C_LEAF;
  }
  // ghost flags of level l+1 under the parents x0-g .. x0+TX-1+g (rows alike)
  if (finer)
    for (int k = threadIdx.x; k < (DIM == 2 ? 2 * (TY + 2 * g) : 1) * 2 * (TX + 2 * g); k += BLK) {
      const int w2 = 2 * (TX + 2 * g), r = k / w2, q = k - r * w2;
      const int x = wrapl(2 * (x0 - g) + q, l + 1), y = DIM == 2 ? wrapl(2 * (y0 - g) + r, l + 1) : 0;
      cf[r][q] = cfl[cidx<DIM>(l + 1, x, y)] == C_GHOST;
    }
  __syncthreads();
  // dilation of the leaf flags along x, rows of the halo
  for (int k = threadIdx.x; k < RY * TX; k += BLK) {
    const int r = k / TX, q = k - r * TX;
    uint8_t v = 0;
    for (int a = 0; a <= 2 * R; ++a) v |= lf[r][q + a];
    hx[r][q] = v;
  }
  // parent flags: some child is a ghost
  if (finer)
    for (int k = threadIdx.x; k < (DIM == 2 ? TY + 2 * g : 1) * (TX + 2 * g); k += BLK) {
      const int r = k / (TX + 2 * g), q = k - r * (TX + 2 * g);
      uint8_t v = cf[DIM == 2 ? 2 * r : 0][2 * q] | cf[DIM == 2 ? 2 * r : 0][2 * q + 1];
      if (DIM == 2) v |= cf[2 * r + 1][2 * q] | cf[2 * r + 1][2 * q + 1];
      pf[r][q] = v;
    }
  __syncthreads();
  if (finer)  // dilation of the parent flags along x by gamma
    for (int k = threadIdx.x; k < (DIM == 2 ? TY + 2 * g : 1) * TX; k += BLK) {
      const int r = k / TX, q = k - r * TX;
      uint8_t v = 0;
      for (int a = 0; a <= 2 * g; ++a) v |= pf[r][q + a];
      px_[r][q] = v;
    }
  __syncthreads();
  // the tile's cells: dilation along y, then the classification
  for (int k = threadIdx.x; k < TY * TX; k += BLK) {
    const int r = k / TX, q = k - r * TX;
    const int x = x0 + q, y = y0 + r;
    if (x >= N || (DIM == 2 && y >= N)) continue;
    uint8_t v = 0;
    for (int b = 0; b <= (DIM == 2 ? 2 * R : 0); ++b) v |= hx[r + b][q];
    if (finer)
      for (int b = 0; b <= (DIM == 2 ? 2 * g : 0); ++b) v |= px_[r + b][q];
    const long long c = cidx<DIM>(l, x, y);
    if (v && cl[c] == C_NONE) cl[c] = C_GHOST;
  }
}

// Byte flags (0/1) of the codes equal to C_LEAF, C_GHOST and C_NONE in a word.
__device__ __forceinline__ uint32_t leaf_flags(uint32_t w) { return w & (w >> 1) & 0x01010101u; }
__device__ __forceinline__ uint32_t ghost_flags(uint32_t w) { return w & ~(w >> 1) & 0x01010101u; }
__device__ __forceinline__ uint32_t none_flags(uint32_t w) { return ~(w | (w >> 1)) & 0x01010101u; }
__device__ __forceinline__ uint32_t internal_flags(uint32_t w) { return (w >> 1) & ~w & 0x01010101u; }

// Same classification as k_classify_ghost for 16 consecutive cells of a row
// per thread (levels whose rows hold at least 16 cells and whose code arrays
// are 16-byte aligned). Leaves of level l in the 5-wide window of each cell:
// the OR of the leaf flags of rows y-2..y+2, dilated by two bytes each way.
// Ghosts of level l+1 in columns 2x-2..2x+3 of rows 2y-2..2y+3: the OR of
// those six rows, folded into column pairs (pair t covers columns 2t, 2t+1),
// dilated by one pair each way.
template <int DIM, typename T>
__device__ __forceinline__ void ghost_run16(const Inst<T> &In, uint8_t *__restrict__ code, int l, long long c0) {
  const long long nl = ncells_d(DIM, l);
  uint8_t *cl = code + In.loff[l];
  const Run16 own = ld16(cl, c0, nl, true);
  Run16 none;
#pragma unroll
  for (int k = 0; k < 4; ++k) none.w[k] = none_flags(own.w[k]);
  if (!(none.w[0] | none.w[1] | none.w[2] | none.w[3])) return;
  int x0, y;
  coords<DIM>(l, (uint32_t)c0, x0, y);
  {
    // Necessary condition: a ghost of level l has an internal cell of level l-1
    // within one cell of its parent. (A leaf at distance <= 2 has an internal
    // parent within one cell of the ghost's parent; a ghost of level l+1 that
    // needs it has, by induction, an internal cell of level l within one cell
    // of its parent, and that cell's parent is internal.) The parents of the
    // run are columns x0/2 .. x0/2+7 of level l-1: test columns x0/2-1 ..
    // x0/2+8 of rows y/2-1 .. y/2+1 from four aligned words per row.
    const int lp = l - 1;
    const uint8_t *cp = code + In.loff[lp];
    if ((((uintptr_t)cp) & 3u) == 0) {
      const int px = x0 >> 1;  // a multiple of 8; rows of level l-1 hold at least 8 cells
      uint32_t any = 0;
      for (int b = (DIM == 2 ? -1 : 0); b <= (DIM == 2 ? 1 : 0); ++b) {
        const uint8_t *row = cp + cidx<DIM>(lp, 0, DIM == 2 ? wrapl((y >> 1) + b, lp) : 0);
        any |= internal_flags(*reinterpret_cast<const uint32_t *>(row + wrapl(px - 4, lp))) & 0x01000000u;
        any |= internal_flags(*reinterpret_cast<const uint32_t *>(row + px));
        any |= internal_flags(*reinterpret_cast<const uint32_t *>(row + px + 4));
        any |= internal_flags(*reinterpret_cast<const uint32_t *>(row + wrapl(px + 8, lp))) & 0x1u;
      }
      if (!any) return;
    }
  }
  // leaves of level l: OR of the rows, edge bytes x0-2, x0-1, x0+16, x0+17
  Run16 lf = {{0, 0, 0, 0}};
  uint32_t em2 = 0, em1 = 0, ep0 = 0, ep1 = 0;
  for (int b = (DIM == 2 ? -2 : 0); b <= (DIM == 2 ? 2 : 0); ++b) {
    const uint8_t *row = cl + cidx<DIM>(l, 0, wrapl(y + b, l));
    const Run16 a = ld16(row, x0, nl, true);
#pragma unroll
    for (int k = 0; k < 4; ++k) lf.w[k] |= leaf_flags(a.w[k]);
    // the 4-cell words left and right of the run (rows hold a multiple of 16 cells)
    const uint32_t wl = leaf_flags(*reinterpret_cast<const uint32_t *>(row + wrapl(x0 - 4, l)));
    const uint32_t wr = leaf_flags(*reinterpret_cast<const uint32_t *>(row + wrapl(x0 + 16, l)));
    em2 |= (wl >> 16) & 0xffu;
    em1 |= wl >> 24;
    ep0 |= wr & 0xffu;
    ep1 |= (wr >> 8) & 0xffu;
  }
  const Run16 n1 = run_next(lf, ep0), n2 = run_next(n1, ep1);
  const Run16 p1 = run_prev(lf, em1), p2 = run_prev(p1, em2);
  Run16 need;
#pragma unroll
  for (int k = 0; k < 4; ++k) need.w[k] = lf.w[k] | n1.w[k] | n2.w[k] | p1.w[k] | p2.w[k];
  if (l < In.jmax) {  // ghosts of level l+1
    const int lf1 = l + 1;
    const uint8_t *cf = code + In.loff[lf1];
    Run16 ga = {{0, 0, 0, 0}}, gb = {{0, 0, 0, 0}};
    uint32_t pm = 0, pp = 0;
    for (int b = (DIM == 2 ? -2 : 0); b <= (DIM == 2 ? 3 : 0); ++b) {
      const uint8_t *row = cf + cidx<DIM>(lf1, 0, wrapl(2 * y + b, lf1));
      const Run16 a = ld16(row, 2 * x0, 2 * nl, true), c = ld16(row, 2 * x0 + 16, 2 * nl, true);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        ga.w[k] |= ghost_flags(a.w[k]);
        gb.w[k] |= ghost_flags(c.w[k]);
      }
      const uint32_t wl = ghost_flags(*reinterpret_cast<const uint32_t *>(row + wrapl(2 * x0 - 4, lf1)));
      const uint32_t wr = ghost_flags(*reinterpret_cast<const uint32_t *>(row + wrapl(2 * x0 + 32, lf1)));
      pm |= ((wl >> 16) | (wl >> 24)) & 0xffu;  // columns 2x0-2, 2x0-1
      pp |= (wr | (wr >> 8)) & 0xffu;           // columns 2x0+32, 2x0+33
    }
    Run16 pr;  // pair flags of the 16 cells
    pr.w[0] = even_bytes(ga.w[0] | (ga.w[0] >> 8), ga.w[1] | (ga.w[1] >> 8));
    pr.w[1] = even_bytes(ga.w[2] | (ga.w[2] >> 8), ga.w[3] | (ga.w[3] >> 8));
    pr.w[2] = even_bytes(gb.w[0] | (gb.w[0] >> 8), gb.w[1] | (gb.w[1] >> 8));
    pr.w[3] = even_bytes(gb.w[2] | (gb.w[2] >> 8), gb.w[3] | (gb.w[3] >> 8));
    const Run16 pn = run_next(pr, pp), pq = run_prev(pr, pm);
#pragma unroll
    for (int k = 0; k < 4; ++k) need.w[k] |= pr.w[k] | pn.w[k] | pq.w[k];
  }
  Run16 out;
  bool changed = false;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t g = need.w[k] & none.w[k];  // NONE (0) -> GHOST (1)
    out.w[k] = own.w[k] | g;
    changed |= g != 0;
  }
  if (changed) st16(cl, c0, nl, true, out);
}
template <int DIM, typename T>
__global__ void __launch_bounds__(BLK) k_classify_ghost16(Batch bt, const Inst<T> *__restrict__ I,
                                                          uint8_t *__restrict__ code,
                                                          const uint32_t *__restrict__ info, int l,
                                                          const int *__restrict__ act) {
  const uint32_t wi = info[blockIdx.x];
  const int i = (int)(wi & 0xffu);
  const long long c0 = ((long long)(wi >> 8) * BLK + threadIdx.x) * CPT;
  if (c0 >= ncells_d(DIM, l) || l > active_top(act, I[i], i)) return;
  ghost_run16<DIM, T>(I[i], code, l, c0);
}

// The same pairing for the ancestor closure: levels l0 then l0-1 (blocks
// from the dense tables info0, info1), ordered when flag is nonzero (the
// finest link has kept cells).
template <int DIM, typename T>
__global__ void __launch_bounds__(BLK) k_ancestor_pair(Batch bt, const Inst<T> *__restrict__ I,
                                                       uint8_t *__restrict__ keep, const uint32_t *__restrict__ info0,
                                                       const uint32_t *__restrict__ info1, int l0, int l1, int G0,
                                                       int G1, const int *__restrict__ act,
                                                       const int *__restrict__ flag, unsigned *__restrict__ sync) {
  const bool second = (int)blockIdx.x >= G0;
  const bool ordered = *flag != 0;
  if (second && ordered) pair_wait(sync, (unsigned)G0);
  const uint32_t w = second ? info1[blockIdx.x - G0] : info0[blockIdx.x];
  const int i = (int)(w & 0xffu), l = second ? l1 : l0;
  const long long cell = (long long)(w >> 8) * BLK + threadIdx.x;
  if (l <= active_top(act, I[i], i) && cell < ncells_d(DIM, l - 2)) ancestor_cell<DIM, T>(I[i], keep, l, cell);
  if (ordered) {
    if (second) pair_leave(sync, (unsigned)G0, (unsigned)G1);
    else pair_signal(sync);
  }
}

// Codes of the initial full finest mesh of instance i: internal below jmax,
// leaf on jmax.
template <typename T>
__global__ void __launch_bounds__(BLK) k_full_tree(const Inst<T> *__restrict__ I, int i, uint8_t *__restrict__ code) {
  const Inst<T> &In = I[i];
  const long long n = In.total;
  for (long long k = blockIdx.x * (long long)BLK + threadIdx.x; k < n; k += (long long)gridDim.x * BLK) {
    const long long gc = In.cbase + k;
    code[gc] = gc >= In.loff[In.jmax] ? C_LEAF : C_INTERNAL;
  }
}

// Plain 16-byte copy (reference kernel for bandwidth and counter calibration).
__global__ void __launch_bounds__(BLK) k_copy_u4(uint4 *__restrict__ dst, const uint4 *__restrict__ src, long long n) {
  for (long long i = blockIdx.x * (long long)BLK + threadIdx.x; i < n; i += (long long)gridDim.x * BLK) dst[i] = src[i];
}

__global__ void __launch_bounds__(BLK) k_fill_u32(uint32_t *__restrict__ p, long long n, uint32_t v) {
  for (long long i = blockIdx.x * (long long)BLK + threadIdx.x; i < n; i += (long long)gridDim.x * BLK) p[i] = v;
}

// ---------------------------------------------------------------- compaction
// Lists of leaves, internal cells and ghosts in (instance, level, cell) order:
// per-block counts, one exclusive scan per instance, then a scatter with
// wavefront ballots.
__device__ __forceinline__ int cat_of(uint8_t v) {
  return v == C_LEAF ? CAT_LEAF : v == C_INTERNAL ? CAT_INTERNAL : v == C_GHOST ? CAT_GHOST : -1;
}


// Category counts (leaf, internal, ghost) of four codes in a word: leaf = 3,
// internal = 2, ghost = 1.
__device__ __forceinline__ void count_codes(uint32_t w, int *n) {
  const uint32_t lo = w & 0x01010101u, hi = (w >> 1) & 0x01010101u;
  n[CAT_LEAF] += __popc(lo & hi);
  n[CAT_INTERNAL] += __popc(hi & ~lo);
  n[CAT_GHOST] += __popc(lo & ~hi);
}

template <int DIM, typename T>
__global__ void __launch_bounds__(BLK) k_compact_count(Batch bt, const Inst<T> *__restrict__ I,
                                                       const uint32_t *__restrict__ binfo, const uint8_t *__restrict__ code,
                                                       int *__restrict__ bcnt, int nblocks, const int *__restrict__ act,
                                                       int *__restrict__ ne) {
  __shared__ int wsum[NCAT][BLK / 64];
  if (blockIdx.x == 0)  // the nonempty flags of this mesh's lists, set by the scan that follows
    for (int t = threadIdx.x; t < NCAT * LVL_STRIDE; t += blockDim.x) ne[t] = 0;
  int i, l;
  long long base;
  chunk_block(binfo, i, l, base);
  if (l > active_top(act, I[i], i)) {  // uniform: an inactive level holds no codes
    if (threadIdx.x < NCAT) bcnt[threadIdx.x * nblocks + blockIdx.x] = 0;
    return;
  }
  const long long nl = ncells_d(DIM, l);
  const uint8_t *cl = code + I[i].loff[l];
  const long long c0 = base + CPT * threadIdx.x;
  int n[NCAT] = {0, 0, 0};
  if (c0 < nl) {
    const Run16 r = ld16(cl, c0, nl, level_vec(cl, nl));
#pragma unroll
    for (int k = 0; k < 4; ++k) count_codes(r.w[k], n);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NCAT; ++k) {
    int v = n[k];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) wsum[k][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < NCAT) {
    int v = 0;
    for (int w = 0; w < BLK / 64; ++w) v += wsum[threadIdx.x][w];
    bcnt[threadIdx.x * nblocks + blockIdx.x] = v;
  }
}

// One block per instance: exclusive scan of its block counts (list positions
// start at the instance's first cell), then its per-level list offsets.
// Wavefront scans by shuffles, then a scan of the wavefront totals.
template <typename T>
__global__ void __launch_bounds__(1024) k_compact_scan(Batch bt, const Inst<T> *__restrict__ I,
                                                       const int *__restrict__ cbp, const int *__restrict__ bcnt,
                                                       int *__restrict__ boff, int *__restrict__ lvl, int nblocks,
                                                       int *__restrict__ act, int *__restrict__ ne) {
  __shared__ int wtot[NCAT][16];
  __shared__ int carry_s[NCAT];
  const int i = blockIdx.x;
  const Inst<T> &In = I[i];
  const int b0 = cbp[i], b1 = cbp[i + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int carry = (int)In.cbase;  // the same start for the three categories
  int car[NCAT] = {carry, carry, carry};
  for (int base = b0; base < b1; base += 1024) {  // the three categories side by side
    const int b = base + threadIdx.x;
    int v[NCAT], incl[NCAT];
#pragma unroll
    for (int k = 0; k < NCAT; ++k) {
      v[k] = b < b1 ? bcnt[k * nblocks + b] : 0;
      incl[k] = v[k];
    }
#pragma unroll
    for (int k = 0; k < NCAT; ++k)
      for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(incl[k], off, 64);
        if (lane >= off) incl[k] += t;
      }
    if (lane == 63)
#pragma unroll
      for (int k = 0; k < NCAT; ++k) wtot[k][wave] = incl[k];
    __syncthreads();
    if (wave < NCAT) {  // wavefront k scans the wavefront totals of category k
      const int k = wave;
      int wv = lane < 16 ? wtot[k][lane] : 0, wi = wv;
      for (int off = 1; off < 16; off <<= 1) {
        const int t = __shfl_up(wi, off, 64);
        if (lane >= off) wi += t;
      }
      if (lane < 16) wtot[k][lane] = wi - wv;  // exclusive prefix of the wavefront totals
      if (lane == 15) carry_s[k] = wi;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NCAT; ++k) {
      if (b < b1) boff[k * nblocks + b] = car[k] + wtot[k][wave] + incl[k] - v[k];
      car[k] += carry_s[k];
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < NCAT * LVL_STRIDE; t += blockDim.x) {
    const int k = t / LVL_STRIDE, l = t - k * LVL_STRIDE;
    int v;
    if (l < In.jmin) v = (int)In.cbase;
    else if (l > In.jmax) v = car[k];
    else v = boff[k * nblocks + In.bstart[l]];
    lvl[(i * NCAT + k) * LVL_STRIDE + l] = v;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < NCAT * LVL_STRIDE - 1; t += blockDim.x) {  // lists with items at (category, level)
    const int *L = lvl + (i * NCAT + t / LVL_STRIDE) * LVL_STRIDE + t % LVL_STRIDE;
    if (t % LVL_STRIDE < LVL_STRIDE - 1 && L[1] > L[0]) ne[t] = 1;
  }
  if (threadIdx.x == 0) {  // activity: this mesh's finest tree level becomes the newest entry
    const int *L = lvl + (i * NCAT + CAT_LEAF) * LVL_STRIDE;
    int fin = In.jmin;
    for (int l = In.jmin; l <= In.jmax; ++l)
      if (L[l + 1] > L[l]) fin = l;
    act[ACT * i + 1] = act[ACT * i];
    act[ACT * i] = fin;
    act[ACT * i + 2] = 0;
  }
}

// With F (the adaptation: code holds the new mesh, code_old the old one), the
// same pass also performs the transfer to the new leaves in place (Algorithm
// 1): a run with leaves reads the same 16 old codes, and its leaves that were
// outside the old mesh are predicted from level l-1; every other new leaf
// already holds its value in F (see the adaptation).
template <int DIM, int Q, typename T, int GAM>
__global__ void __launch_bounds__(BLK) k_compact_scatter(Batch bt, const Inst<T> *__restrict__ I,
                                                         const uint32_t *__restrict__ binfo, const uint8_t *__restrict__ code,
                                                         const int *__restrict__ boff, uint32_t *__restrict__ lists,
                                                         int nblocks, const uint8_t *__restrict__ code_old,
                                                         T *__restrict__ F, uint8_t *__restrict__ mark,
                                                         const int *__restrict__ act) {
  __shared__ int wsum[NCAT][BLK / 64];
  int i, l;
  long long base;
  chunk_block(binfo, i, l, base);
  if (l > active_top(act, I[i], i)) return;  // uniform: no codes, no counts
  const long long nl = ncells_d(DIM, l);
  const uint8_t *cl = code + I[i].loff[l];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long c0 = base + CPT * threadIdx.x;
  const bool vec = level_vec(cl, nl);
  Run16 r = {{0, 0, 0, 0}};
  if (c0 < nl) r = ld16(cl, c0, nl, vec);
  int n[NCAT] = {0, 0, 0}, incl[NCAT];
#pragma unroll
  for (int k = 0; k < 4; ++k) count_codes(r.w[k], n);
#pragma unroll
  for (int k = 0; k < NCAT; ++k) {  // inclusive scan over the wavefront
    int v = n[k];
    for (int off = 1; off < 64; off <<= 1) {
      const int u = __shfl_up(v, off, 64);
      if (lane >= off) v += u;
    }
    incl[k] = v;
    if (lane == 63) wsum[k][wave] = v;
  }
  __syncthreads();
  // The block's cells of each category, in cell order, gathered in LDS (as
  // offsets in the block), then written out as one contiguous, coalesced range
  // per category.
  __shared__ uint16_t ent[NCAT][CCHUNK];
  int tot[NCAT];
#pragma unroll
  for (int k = 0; k < NCAT; ++k) {
    int before = 0, all = 0;
    for (int ww = 0; ww < BLK / 64; ++ww) {
      if (ww < wave) before += wsum[k][ww];
      all += wsum[k][ww];
    }
    tot[k] = all;
    incl[k] = before + incl[k] - n[k];  // first slot of this thread
  }
  if (r.w[0] | r.w[1] | r.w[2] | r.w[3]) {
    for (int t = 0; t < 16; ++t) {
      const int k = cat_of((uint8_t)(r.w[t >> 2] >> (8 * (t & 3))));
      if (k >= 0) ent[k][incl[k]++] = (uint16_t)(CPT * threadIdx.x + t);
    }
  }
  __syncthreads();
  const uint32_t tag = (uint32_t)l << LEVEL_SHIFT;
#pragma unroll
  for (int k = 0; k < NCAT; ++k) {
    if (!tot[k]) continue;
    uint32_t *out = lists + (size_t)k * bt.ctotal + boff[k * nblocks + blockIdx.x];
    for (int j = threadIdx.x; j < tot[k]; j += BLK) out[j] = tag | (uint32_t)(base + ent[k][j]);
  }
  if (DIM == 3 || !F) return;  // uniform: the adaptation's transfer follows (3D: a kernel of its own)
  // The cells of the block created by the adaptation (new leaves outside the
  // old mesh) are gathered in LDS and predicted one per thread. New leaves
  // outside the old tree (these and former ghosts) get a mark for the
  // reconstruction that follows (project_marked).
  uint16_t *xq = ent[0];  // free again after the barrier below
  __shared__ int xtot[BLK / 64 + 1];
  uint32_t created[4] = {0, 0, 0, 0};
  if (n[CAT_LEAF]) {
    const uint8_t *co = code_old + I[i].loff[l];
    const Run16 o = ld16(co, c0, nl, level_vec(co, nl));
    Run16 fresh;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      created[k] = leaf_flags(r.w[k]) & none_flags(o.w[k]);
      fresh.w[k] = leaf_flags(r.w[k]) & ~(o.w[k] >> 1) & 0x01010101u;
    }
    if (fresh.w[0] | fresh.w[1] | fresh.w[2] | fresh.w[3]) {
      uint8_t *ml = mark + I[i].loff[l];
      st16(ml, c0, nl, level_vec(ml, nl), fresh);
    }
  }
  const int nc = __popc(created[0]) + __popc(created[1]) + __popc(created[2]) + __popc(created[3]);
  int inc = nc;
  for (int off = 1; off < 64; off <<= 1) {
    const int u = __shfl_up(inc, off, 64);
    if (lane >= off) inc += u;
  }
  if (lane == 63) xtot[wave] = inc;
  __syncthreads();
  int before = 0, total = 0;
  for (int ww = 0; ww < BLK / 64; ++ww) {
    if (ww < wave) before += xtot[ww];
    total += xtot[ww];
  }
  if (total == 0) return;  // uniform
  int at = before + inc - nc;
  for (int t = 0; t < 16; ++t)
    if ((created[t >> 2] >> (8 * (t & 3))) & 1u) xq[at++] = (uint16_t)(CPT * threadIdx.x + t);
  __syncthreads();
  const Inst<T> &In = I[i];
  for (int k = threadIdx.x; k < total; k += BLK) {
    const long long c = base + xq[k];
    int x, y;
    coords<DIM>(l, (uint32_t)c, x, y);
    for (int h = 0; h < Q; ++h)
      F[foff(In, DIM, Q, l, h) + c] =
          predict<DIM, T>(F + foff(In, DIM, Q, l - 1, h), l, x, y, In.walls, gamma_k<GAM>(In));
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
//
// Neighbours refined one level further (bit k of nbr over the 3^d - 1
// neighbours, x fastest): their children's details weighted by Cw, added to acc.
template <int DIM, typename T>
__device__ __forceinline__ T detail_correction(T acc, int l, int x, int y, const T *__restrict__ Fl,
                                               const T *__restrict__ Ff, const T *__restrict__ Cw, unsigned nbr) {
  for (int b = (DIM == 2 ? -1 : 0), bit = 0; b <= (DIM == 2 ? 1 : 0); ++b)
    for (int a = -1; a <= 1; ++a) {
      if (a == 0 && b == 0) continue;
      const int k = bit++;
      if (!(nbr & (1u << k))) continue;
      const int px = wrapl(x + a, l), py = DIM == 2 ? wrapl(y + b, l) : 0;
      ParentStencil<DIM, T> st;
      st.load(Fl, l, px, py, 0);  // leaves of the periodic paths only (walls: transport_wall)
      for (int dy = 0; dy < (DIM == 2 ? 2 : 1); ++dy)
        for (int dx = 0; dx < 2; ++dx) {
          const T d = Ff[cidx<DIM>(l + 1, 2 * px + dx, 2 * py + dy)] - st.child(dx, dy);
          const int y1 = 2 * a + dx + 2, y2 = DIM == 2 ? 2 * b + dy + 2 : 0;
          acc = fma(Cw[y2 * 6 + y1], d, acc);
        }
    }
  return acc;
}

// Neighbours (bits as in refined_neighbours) whose children's details enter the
// transport of velocity (ex, ey): the sums of an axis velocity collapse onto the
// leaf's row or column (the children of a cell average to the cell along the
// other axis), so only the two neighbours along the axis carry nonzero
// correction weights; the others are skipped (their terms would add 0).
//
// For a leaf one level above the finest (n = 1) the sets E and A lie within
// one finest cell of the leaf's faces, and only the upwind neighbours (offsets
// a in {0, -ex}, b in {0, -ey}) carry weights.
template <int DIM>
__host__ __device__ constexpr unsigned correction_mask(int ex, int ey) {
  return DIM == 1 ? 0x3u : (ey == 0 && ex != 0) ? 0x18u : (ex == 0 && ey != 0) ? 0x42u : 0xffu;
}
template <int DIM>
__host__ __device__ constexpr unsigned upwind_mask(int ex, int ey) {
  unsigned m = 0;
  for (int b = (DIM == 2 ? -1 : 0), bit = 0; b <= (DIM == 2 ? 1 : 0); ++b)
    for (int a = -1; a <= 1; ++a) {
      if (a == 0 && b == 0) continue;
      if ((a == 0 || a == -ex) && (b == 0 || b == -ey)) m |= 1u << bit;
      ++bit;
    }
  return m;
}
template <int DIM>
__host__ __device__ constexpr unsigned correction_mask(int ex, int ey, int n) {
  return correction_mask<DIM>(ex, ey) & (n == 1 ? upwind_mask<DIM>(ex, ey) : 0xffu);
}

// Population h of the leaf (l, c): Fl / Ff point at population h of levels l and
// l+1, cl at the codes of level l, W / Cw at the weights of (n, h).
template <int DIM, int SCHEME, typename T>
__device__ __forceinline__ T transport_pop(int h, int l, int J, uint32_t c, int x, int y, const T *__restrict__ Fl,
                                           const T *__restrict__ Ff, const uint8_t *__restrict__ cl,
                                           const T *__restrict__ W, const T *__restrict__ Cw, unsigned nbr) {
  using V = Vel<SCHEME>;
  const int ex = V::ex(h), ey = V::ey(h);
  const int n = J - l;
  if (ex == 0 && ey == 0) return Fl[c];
  if (n == 0) return Fl[cidx<DIM>(J, wrapl(x - ex, J), wrapl(y - ey, J))];
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
  if (nbr & correction_mask<DIM>(ex, ey, n))
    acc = detail_correction<DIM, T>(acc, l, x, y, Fl, Ff, Cw, nbr & correction_mask<DIM>(ex, ey, n));
  return fma((T)ldexp(1.0, -DIM * n), acc, Fl[c]);
}

// Bit k (over the 3^d - 1 neighbours, x fastest) set if that neighbour of (x, y)
// at level l is an internal cell.
template <int DIM>
__device__ __forceinline__ unsigned refined_neighbours(const uint8_t *__restrict__ cl, int l, int x, int y) {
  unsigned nbr = 0;
  if (l >= 2 && (((uintptr_t)cl) & 3u) == 0) {  // columns x-1..x+1 of each row from two aligned words
    const int wa = wrapl(x - 1, l) & ~3, wb = wrapl(wa + 4, l), sh = 8 * ((x - 1) & 3);
    for (int b = (DIM == 2 ? -1 : 0), bit = 0; b <= (DIM == 2 ? 1 : 0); ++b) {
      const uint8_t *row = cl + cidx<DIM>(l, 0, DIM == 2 ? wrapl(y + b, l) : 0);
      const unsigned long long v = ((unsigned long long)*reinterpret_cast<const uint32_t *>(row + wb) << 32 |
                                    *reinterpret_cast<const uint32_t *>(row + wa)) >> sh;
      for (int a = -1; a <= 1; ++a) {
        if (a == 0 && b == 0) continue;
        if (((v >> (8 * (a + 1))) & 0xffu) == C_INTERNAL) nbr |= 1u << bit;
        ++bit;
      }
    }
    return nbr;
  }
  for (int b = (DIM == 2 ? -1 : 0), bit = 0; b <= (DIM == 2 ? 1 : 0); ++b)
    for (int a = -1; a <= 1; ++a) {
      if (a == 0 && b == 0) continue;
      if (cl[cidx<DIM>(l, wrapl(x + a, l), DIM == 2 ? wrapl(y + b, l) : 0)] == C_INTERNAL) nbr |= 1u << bit;
      ++bit;
    }
  return nbr;
}

// ---------------------------------------------------------------- walls, wide stencils
// Tables of the general transport path, per n - 1 and wall case wc = cx + 3 cy
// (per axis 0: the leaf touches no wall of that axis, 1: the lower one, 2: the
// upper one): W over the leaf-level box of half-width R = 2 gamma ((2R+1)^d
// entries) and C over the children offsets -R .. R+1 from 2k ((2R+2)^d), as
// for the periodic leaves but with the finest cells of E beyond the walls left
// out, and the number of those cells beyond the x wall and (x inside) beyond
// the y wall. Those cells take the side's condition evaluated on the leaf
// itself (section "Boundary conditions", eq. AdvectionOnBoundary, direct
// evaluation). Case 0 holds the periodic tables of the batch's gamma.
template <typename T>
struct WallTabs {
  const T *W;  // [nmax][9][q][(2R+1)^d]
  const T *C;  // [nmax][9][q][(2R+2)^d]
  const T *N;  // [nmax][9][q][2]
};

template <int SCHEME>
__host__ __device__ constexpr int opposite_vel(int h) {
  for (int k = 0; k < Vel<SCHEME>::Q; ++k)
    if (Vel<SCHEME>::ex(k) == -Vel<SCHEME>::ex(h) && Vel<SCHEME>::ey(k) == -Vel<SCHEME>::ey(h)) return k;
  return h;
}

// Population h entering a leaf from beyond a wall of `kind` (eq.
// refBoundaryConditions), evaluated on the leaf: its own value of h (copy) or
// of the opposite velocity (bounce back; anti bounce back with the sign changed).
template <int SCHEME, typename T>
__device__ __forceinline__ T wall_value(int kind, int h, const T *__restrict__ Fl0, long long nl, uint32_t c) {
  const T v = Fl0[(long long)(kind == 1 ? h : opposite_vel<SCHEME>(h)) * nl + c];
  return kind == 3 ? -v : v;
}

// A leaf whose transport box (half-width 2 gamma) reaches beyond a wall: the
// box is read with reflection, which reproduces the reconstruction of the
// mirrored problem.
template <int DIM, typename T>
__device__ __forceinline__ bool near_wall(const Inst<T> &In, int l, int x, int y) {
  const int n = 1 << l, R = 2 * In.gamma;
  return ((In.walls & 1) && (x < R || x > n - 1 - R)) || (DIM == 2 && (In.walls & 2) && (y < R || y > n - 1 - R));
}

// Population h of a leaf by the general path (walls at any position, or a
// prediction of half-width gamma > 1): the sums of transport_pop over the box
// of half-width R = 2 gamma with every index reflected at a wall, detail
// corrections from the neighbours within gamma that are refined one level
// further (beyond a wall mirrored: a refined mirrored neighbour contributes the
// details of the mirrored children), the tables of the leaf's wall case, and
// the incoming values from beyond the walls. Fl0 / Ff0 point at population 0 of
// levels l and l+1, cl at the codes of level l.
template <int DIM, int SCHEME, typename T, int G, int H>
__device__ __attribute__((noinline)) T transport_wall_gh(const Inst<T> &In, int l, uint32_t c, int x, int y,
                                                         const T *__restrict__ Fl0, const T *__restrict__ Ff0,
                                                         const uint8_t *__restrict__ cl, WallTabs<T> wt) {
  using V = Vel<SCHEME>;
  constexpr int Q = V::Q, h = H;
  constexpr int ex = V::ex(H), ey = V::ey(H);
  const int J = In.jmax, n = J - l, N = 1 << l;
  const bool wx = In.walls & 1, wy = DIM == 2 && (In.walls & 2);
  const long long nl = ncells_d(DIM, l), nf = ncells_d(DIM, l + 1);
  const T *Fl = Fl0 + (long long)h * nl;
  if (ex == 0 && ey == 0) return Fl[c];
  if (n == 0) {  // the plain shift, or the condition of the wall the source lies beyond
    const int sx = x - ex, sy = y - ey;
    int side = -1;
    if (wx && (sx < 0 || sx >= N)) side = sx < 0 ? 0 : 1;
    else if (wy && (sy < 0 || sy >= N)) side = sy < 0 ? 2 : 3;
    if (side >= 0) return wall_value<SCHEME, T>(In.bck[side], h, Fl0, nl, c);
    return Fl[cidx<DIM>(l, wrapl(sx, l), wrapl(sy, l))];
  }
  const int cx = wx ? (x == 0 ? 1 : (x == N - 1 ? 2 : 0)) : 0;
  const int cy = wy ? (y == 0 ? 1 : (y == N - 1 ? 2 : 0)) : 0;
  constexpr int g = G, R = 2 * g, WW = 2 * R + 1, CW = 2 * R + 2;
  constexpr int WSg = DIM == 2 ? WW * WW : WW, CSg = DIM == 2 ? CW * CW : CW;
  const int wc = cx + 3 * cy, nn = n - 1;
  const T *W = wt.W + (((long long)nn * 9 + wc) * Q + h) * WSg;
  const T *Cw = wt.C + (((long long)nn * 9 + wc) * Q + h) * CSg;
  T acc = T(0);
  // an axis velocity's weights vanish off its own row (column): the sums over
  // the other rows of the leaf's cells of a unit impulse's reconstruction
  constexpr int b0 = DIM == 2 && ey != 0 ? -R : 0, b1 = DIM == 2 && ey != 0 ? R : 0;
  constexpr int a0 = ex != 0 ? -R : 0, a1 = ex != 0 ? R : 0;
  // (the rows unrolled for gamma = 1 only: the wider boxes would not fit the registers)
#pragma unroll(G == 1 ? 5 : 1)
  for (int b = b0; b <= b1; ++b) {
    const long long row = DIM == 2 ? ((long long)axl(y + b, l, wy) << l) : 0;
#pragma unroll
    for (int a = a0; a <= a1; ++a)
      acc = fma(W[DIM == 2 ? (b + R) * WW + a + R : a + R], Fl[row + axl(x + a, l, wx)], acc);
  }
  // neighbours refined one level further, mirrored beyond a wall
  const T *Ff = Ff0 + (long long)h * nf;
  for (int b = (DIM == 2 ? -g : 0); b <= (DIM == 2 ? g : 0); ++b)
#pragma unroll 1
    for (int a = -g; a <= g; ++a) {
      if (a == 0 && b == 0) continue;
      const int vx = x + a, vy = y + b;
      const bool mx = wx && (vx < 0 || vx >= N), my = wy && (vy < 0 || vy >= N);
      const int px = axl(vx, l, wx), py = DIM == 2 ? axl(vy, l, wy) : 0;
      if (cl[cidx<DIM>(l, px, py)] != C_INTERNAL) continue;
      ParentStencil<DIM, T> st;
      st.load(Fl, l, px, py, In.walls, G);
      for (int dy = 0; dy < (DIM == 2 ? 2 : 1); ++dy)
        for (int dx = 0; dx < 2; ++dx) {
          const int rx = mx ? 1 - dx : dx, ry = my ? 1 - dy : dy;  // the real child the virtual one mirrors
          const T d = Ff[cidx<DIM>(l + 1, 2 * px + rx, 2 * py + ry)] - st.child(rx, ry);
          const int y1 = 2 * a + dx + R, y2 = DIM == 2 ? 2 * b + dy + R : 0;
          acc = fma(Cw[y2 * CW + y1], d, acc);
        }
    }
  if (wc) {  // the finest cells of E beyond the walls
    const T *Nw = wt.N + (((long long)nn * 9 + wc) * Q + h) * 2;
    if (cx && Nw[0] != T(0)) acc = fma(Nw[0], wall_value<SCHEME, T>(In.bck[cx - 1], h, Fl0, nl, c), acc);
    if (cy && Nw[1] != T(0)) acc = fma(Nw[1], wall_value<SCHEME, T>(In.bck[1 + cy], h, Fl0, nl, c), acc);
  }
  return fma((T)ldexp(1.0, -DIM * n), acc, Fl[c]);
}

// transport_wall_gh for the instance's gamma and a run-time population h.
template <int DIM, int SCHEME, typename T, int G, int H>
__device__ __forceinline__ T transport_wall_h(int h, const Inst<T> &In, int l, uint32_t c, int x, int y, const T *Fl0,
                                              const T *Ff0, const uint8_t *cl, WallTabs<T> wt) {
  if constexpr (H + 1 < Vel<SCHEME>::Q)
    if (h != H) return transport_wall_h<DIM, SCHEME, T, G, H + 1>(h, In, l, c, x, y, Fl0, Ff0, cl, wt);
  return transport_wall_gh<DIM, SCHEME, T, G, H>(In, l, c, x, y, Fl0, Ff0, cl, wt);
}
template <int DIM, int SCHEME, typename T, int G>
__device__ __forceinline__ T transport_wall(const Inst<T> &In, int h, int l, uint32_t c, int x, int y,
                                            const T *__restrict__ Fl0, const T *__restrict__ Ff0,
                                            const uint8_t *__restrict__ cl, WallTabs<T> wt) {
  return transport_wall_h<DIM, SCHEME, T, G, 0>(h, In, l, c, x, y, Fl0, Ff0, cl, wt);
}

// One leaf of an instance with walls, every population by transport_wall, then
// the tape, the collision and the store as in leaf_update.
template <int DIM, int SCHEME, typename T, int G>
__device__ __attribute__((noinline)) void leaf_update_wall(const Inst<T> &In, int l, uint32_t c,
                                                           const T *__restrict__ Fs, T *__restrict__ Fo,
                                                           const uint8_t *__restrict__ code, WallTabs<T> wt,
                                                           T *__restrict__ tape) {
  constexpr int Q = Vel<SCHEME>::Q;
  int x, y;
  coords<DIM>(l, c, x, y);
  const long long ol = (long long)Q * In.loff[l], nl = ncells_d(DIM, l);
  const T *Ff0 = l < In.jmax ? Fs + (long long)Q * In.loff[l + 1] : Fs;
  T f[Q];
#pragma unroll
  for (int h = 0; h < Q; ++h)
    f[h] = transport_wall<DIM, SCHEME, T, G>(In, h, l, c, x, y, Fs + ol, Ff0, code + In.loff[l], wt);
  if (tape)
#pragma unroll
    for (int h = 0; h < Q; ++h) tape[ol + h * nl + c] = f[h];
  collide<SCHEME, T>(f, In.sc);
#pragma unroll
  for (int h = 0; h < Q; ++h) Fo[ol + h * nl + c] = f[h];
}

// ParentStencil::load_wide for a half-width G known at compile time and a
// periodic neighbourhood (the same operations in the same order).
template <int DIM, typename T, int G>
__device__ __forceinline__ void parent_stencil_g(ParentStencil<DIM, T> &st, const T *__restrict__ P, int lp, int px,
                                                 int py) {
  auto at = [&](int a, int b) -> T {
    return DIM == 1 ? P[wrapl(px + a, lp)] : P[cidx<2>(lp, wrapl(px + a, lp), wrapl(py + b, lp))];
  };
  st.c = at(0, 0);
  st.qx = T(table1(G, 1)) * (at(1, 0) - at(-1, 0));
#pragma unroll
  for (int a = 2; a <= G; ++a) st.qx = st.qx + T(table1(G, a)) * (at(a, 0) - at(-a, 0));
  if (DIM == 1) {
    st.qy = T(0);
    st.qxy = T(0);
    return;
  }
  st.qy = T(table1(G, 1)) * (at(0, 1) - at(0, -1));
#pragma unroll
  for (int b = 2; b <= G; ++b) st.qy = st.qy + T(table1(G, b)) * (at(0, b) - at(0, -b));
  auto term = [&](int a, int b) -> T {
    return T(table1(G, a) * table1(G, b)) * (((at(a, b) - at(-a, b)) - at(a, -b)) + at(-a, -b));
  };
  st.qxy = term(1, 1);
#pragma unroll
  for (int b = 1; b <= G; ++b)
#pragma unroll
    for (int a = (b == 1 ? 2 : 1); a <= G; ++a) st.qxy = st.qxy + term(a, b);
}

// Neighbours of (x, y) within G (periodic) that are internal cells, as bits
// (b + G)(2G + 1) + (a + G) of offset (a, b): their codes are loaded together,
// once per leaf.
template <int DIM, int G>
__device__ __forceinline__ unsigned long long refined_within_g(const uint8_t *__restrict__ cl, int l, int x, int y) {
  constexpr int S = 2 * G + 1;
  unsigned long long m = 0;
#pragma unroll
  for (int b = (DIM == 2 ? -G : 0); b <= (DIM == 2 ? G : 0); ++b)
#pragma unroll
    for (int a = -G; a <= G; ++a)
      if ((a != 0 || b != 0) && cl[cidx<DIM>(l, wrapl(x + a, l), DIM == 2 ? wrapl(y + b, l) : 0)] == C_INTERNAL)
        m |= 1ull << ((b + G) * S + (a + G));
  return m;
}

// transport_wall for a leaf whose transport box stays inside the domain (a
// periodic instance, or a leaf farther than 2 G cells from every wall), with
// the prediction half-width G and the population H as compile-time constants:
// no reflection, the tables of wall case 0, the refined neighbours given as
// bits (refined_within_g); the same operations in the same order.
template <int DIM, int SCHEME, typename T, int G, int H>
__device__ __attribute__((noinline)) T transport_inner_g(const Inst<T> &In, int l, uint32_t c, int x, int y,
                                                         const T *__restrict__ Fl0, const T *__restrict__ Ff0,
                                                         unsigned long long nbm, WallTabs<T> wt) {
  using V = Vel<SCHEME>;
  constexpr int Q = V::Q, R = 2 * G, WW = 2 * R + 1, CW = 2 * R + 2, h = H;
  constexpr int WSg = DIM == 2 ? WW * WW : WW, CSg = DIM == 2 ? CW * CW : CW;
  constexpr int ex = V::ex(H), ey = V::ey(H);
  const int n = In.jmax - l;
  const long long nl = ncells_d(DIM, l), nf = ncells_d(DIM, l + 1);
  const T *Fl = Fl0 + (long long)h * nl;
  if (ex == 0 && ey == 0) return Fl[c];
  if (n == 0) return Fl[cidx<DIM>(l, wrapl(x - ex, l), wrapl(y - ey, l))];
  const T *W = wt.W + ((long long)(n - 1) * 9 * Q + h) * WSg;
  const T *Cw = wt.C + ((long long)(n - 1) * 9 * Q + h) * CSg;
  T acc = T(0);
  constexpr int b0 = DIM == 2 && ey != 0 ? -R : 0, b1 = DIM == 2 && ey != 0 ? R : 0;
  constexpr int a0 = ex != 0 ? -R : 0, a1 = ex != 0 ? R : 0;
#pragma unroll
  for (int b = b0; b <= b1; ++b) {
    const long long row = DIM == 2 ? ((long long)wrapl(y + b, l) << l) : 0;
#pragma unroll
    for (int a = a0; a <= a1; ++a)
      acc = fma(W[DIM == 2 ? (b + R) * WW + a + R : a + R], Fl[row + wrapl(x + a, l)], acc);
  }
  const T *Ff = Ff0 + (long long)h * nf;
  for (int b = (DIM == 2 ? -G : 0); b <= (DIM == 2 ? G : 0); ++b)
#pragma unroll 1
    for (int a = -G; a <= G; ++a) {
      if (!((nbm >> ((b + G) * (2 * G + 1) + (a + G))) & 1ull)) continue;
      const int px = wrapl(x + a, l), py = DIM == 2 ? wrapl(y + b, l) : 0;
      ParentStencil<DIM, T> st;
      parent_stencil_g<DIM, T, G>(st, Fl, l, px, py);
#pragma unroll
      for (int dy = 0; dy < (DIM == 2 ? 2 : 1); ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
          const T d = Ff[cidx<DIM>(l + 1, 2 * px + dx, 2 * py + dy)] - st.child(dx, dy);
          const int y1 = 2 * a + dx + R, y2 = DIM == 2 ? 2 * b + dy + R : 0;
          acc = fma(Cw[y2 * CW + y1], d, acc);
        }
    }
  return fma((T)ldexp(1.0, -DIM * n), acc, Fl[c]);
}

// Every population H of a leaf by transport_inner_g (f[H]), and population h
// (a run-time index) by a chain of tests.
template <int DIM, int SCHEME, typename T, int G, int H>
__device__ __forceinline__ void inner_all(T *f, const Inst<T> &In, int l, uint32_t c, int x, int y, const T *Fl0,
                                          const T *Ff0, unsigned long long nbm, WallTabs<T> wt) {
  if constexpr (H < Vel<SCHEME>::Q) {
    f[H] = transport_inner_g<DIM, SCHEME, T, G, H>(In, l, c, x, y, Fl0, Ff0, nbm, wt);
    inner_all<DIM, SCHEME, T, G, H + 1>(f, In, l, c, x, y, Fl0, Ff0, nbm, wt);
  }
}
template <int DIM, int SCHEME, typename T, int G, int H>
__device__ __forceinline__ T inner_one(int h, const Inst<T> &In, int l, uint32_t c, int x, int y, const T *Fl0,
                                       const T *Ff0, unsigned long long nbm, WallTabs<T> wt) {
  if constexpr (H + 1 < Vel<SCHEME>::Q)
    if (h != H) return inner_one<DIM, SCHEME, T, G, H + 1>(h, In, l, c, x, y, Fl0, Ff0, nbm, wt);
  return transport_inner_g<DIM, SCHEME, T, G, H>(In, l, c, x, y, Fl0, Ff0, nbm, wt);
}

// One leaf by transport_inner_g, then the tape, the collision and the store.
template <int DIM, int SCHEME, typename T, int G>
__device__ __forceinline__ void leaf_update_inner_g(const Inst<T> &In, int l, uint32_t c,
                                                    const T *__restrict__ Fs, T *__restrict__ Fo,
                                                    const uint8_t *__restrict__ code, WallTabs<T> wt,
                                                    T *__restrict__ tape) {
  constexpr int Q = Vel<SCHEME>::Q;
  int x, y;
  coords<DIM>(l, c, x, y);
  const long long ol = (long long)Q * In.loff[l], nl = ncells_d(DIM, l);
  const T *Ff0 = l < In.jmax ? Fs + (long long)Q * In.loff[l + 1] : Fs;
  const unsigned long long nbm = l < In.jmax ? refined_within_g<DIM, G>(code + In.loff[l], l, x, y) : 0ull;
  T f[Q];
  inner_all<DIM, SCHEME, T, G, 0>(f, In, l, c, x, y, Fs + ol, Ff0, nbm, wt);
  if (tape)
#pragma unroll
    for (int h = 0; h < Q; ++h) tape[ol + h * nl + c] = f[h];
  collide<SCHEME, T>(f, In.sc);
#pragma unroll
  for (int h = 0; h < Q; ++h) Fo[ol + h * nl + c] = f[h];
}

// Variant for small leaf sets: wavefront h transports population h of 64 leaves
// (nine times the parallelism), the collision of each leaf then runs in
// wavefront 0 through LDS.
template <int DIM, int SCHEME, typename T, int MODE>
__global__ void __launch_bounds__(64 * Vel<SCHEME>::Q)
    k_transport_collide_pop(Batch bt, const Inst<T> *__restrict__ I, const T *__restrict__ Fs, T *__restrict__ Fo,
                            const uint8_t *__restrict__ code, const uint32_t *__restrict__ leaves,
                            const int *__restrict__ lvl, const T *__restrict__ Wt, const T *__restrict__ Ct,
                            WallTabs<T> wt, unsigned long long *__restrict__ counters, T *__restrict__ tape) {
  using V = Vel<SCHEME>;
  constexpr int Q = V::Q;
  constexpr int WS = DIM == 2 ? 25 : 5, CS = DIM == 2 ? 36 : 6;
  __shared__ SegLDS s;
  __shared__ T fl[Q][64];
  __shared__ long long sloff[LVL_STRIDE];
  __shared__ int sjmax;
  load_segments(s, I, lvl, bt.B, CAT_LEAF, -1);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    unsigned long long tot = 0;
    for (int i = 0; i < bt.B; ++i) tot += (unsigned long long)s.cnt[i];
    atomicAdd(&counters[0], tot);
    atomicAdd(&counters[1], 1ull);
  }
  const int h = threadIdx.x >> 6, lane = threadIdx.x & 63;
  MRLBM_FOR_CHUNKS(ch, s.pre[bt.B], 1, 0) {
    const int i = upper_index(s.pre, bt.B, ch);
    const int item = (ch - s.pre[i]) * CHUNK + lane;
    const bool valid = item < s.cnt[i];
    const uint32_t e = valid ? leaves[s.beg[i] + item] : 0u;
    if (threadIdx.x < LVL_STRIDE) sloff[threadIdx.x] = I[i].loff[threadIdx.x];
    if (threadIdx.x == 0) sjmax = I[i].jmax;
    __syncthreads();
    const int l = (int)(e >> LEVEL_SHIFT);
    const uint32_t c = e & CELL_MASK;
    // MODE 1: the leaves near a wall belong to k_transport_wall_band; MODE =
    // gamma > 1: they take the general path, the others the path of that gamma
    bool todo = valid, wall = false;
    if (MODE != 0 && valid && I[i].walls) {
      int x, y;
      coords<DIM>(l, c, x, y);
      wall = near_wall<DIM>(I[i], l, x, y);
      if (MODE == 1) todo = !wall;
    }
    if (todo) {
      int x, y;
      coords<DIM>(l, c, x, y);
      const int J = sjmax, n = J - l;
      const uint8_t *cl = code + sloff[l];
      const unsigned nbr = n > 0 ? refined_neighbours<DIM>(cl, l, x, y) : 0u;
      const T *Fl = Fs + (long long)Q * sloff[l] + (long long)h * ncells_d(DIM, l);
      const T *Ff = n > 0 ? Fs + (long long)Q * sloff[l + 1] + (long long)h * ncells_d(DIM, l + 1) : Fl;
      const int nn = n > 0 ? n - 1 : 0;
      if constexpr (MODE >= 2) {
        if (wall)
          fl[h][lane] = transport_wall<DIM, SCHEME, T, MODE>(I[i], h, l, c, x, y, Fs + (long long)Q * sloff[l],
                                                       n > 0 ? Fs + (long long)Q * sloff[l + 1] : Fs, cl, wt);
        else
          fl[h][lane] = inner_one<DIM, SCHEME, T, MODE, 0>(
              h, I[i], l, c, x, y, Fs + (long long)Q * sloff[l], n > 0 ? Fs + (long long)Q * sloff[l + 1] : Fs,
              n > 0 ? refined_within_g<DIM, MODE>(cl, l, x, y) : 0ull, wt);
      } else {
        fl[h][lane] = transport_pop<DIM, SCHEME, T>(h, l, J, c, x, y, Fl, Ff, cl, Wt + ((long long)nn * Q + h) * WS,
                                                    Ct + ((long long)nn * Q + h) * CS, nbr);
      }
      if (tape) tape[(long long)Q * sloff[l] + (long long)h * ncells_d(DIM, l) + c] = fl[h][lane];
    }
    __syncthreads();
    if (h == 0 && todo) {
      T g[Q];
#pragma unroll
      for (int k = 0; k < Q; ++k) g[k] = fl[k][lane];
      collide<SCHEME, T>(g, I[i].sc);
#pragma unroll
      for (int k = 0; k < Q; ++k) fl[k][lane] = g[k];
    }
    __syncthreads();
    if (todo) Fo[(long long)Q * sloff[l] + (long long)h * ncells_d(DIM, l) + c] = fl[h][lane];
    __syncthreads();
  }
}

// One leaf of the per-leaf variant: transport of every population, optional
// tape of the pre-collision values, collision, store.
template <int DIM, int SCHEME, typename T>
__device__ __forceinline__ void leaf_update(const Inst<T> &In, int l, uint32_t c, const T *__restrict__ Fs,
                                            T *__restrict__ Fo, const uint8_t *__restrict__ code,
                                            const T *__restrict__ Wt, const T *__restrict__ Ct, T *__restrict__ tape) {
  using V = Vel<SCHEME>;
  constexpr int Q = V::Q;
  constexpr int WS = DIM == 2 ? 25 : 5, CS = DIM == 2 ? 36 : 6;
  int x, y;
  coords<DIM>(l, c, x, y);
  const int J = In.jmax, n = J - l;
  const long long ol = (long long)Q * In.loff[l], nl = ncells_d(DIM, l);
  const uint8_t *cl = code + In.loff[l];
  const unsigned nbr = n > 0 ? refined_neighbours<DIM>(cl, l, x, y) : 0u;
  const long long of = n > 0 ? (long long)Q * In.loff[l + 1] : ol, nf = ncells_d(DIM, l + 1);
  const int nn = n > 0 ? n - 1 : 0;
  T f[Q];
#pragma unroll
  for (int h = 0; h < Q; ++h) {
    // The stencil offsets of every population are the same; computed once they
    // would stay live across all nine (too many registers for 4 waves per SIMD).
    // Hiding the coordinates behind an empty asm makes each population
    // recompute its offsets right before its loads.
    int xh = x, yh = y;
    asm volatile("" : "+v"(xh), "+v"(yh));
    f[h] = transport_pop<DIM, SCHEME, T>(h, l, J, c, xh, yh, Fs + ol + h * nl, Fs + of + h * nf, cl,
                                         Wt + ((long long)nn * Q + h) * WS, Ct + ((long long)nn * Q + h) * CS, nbr);
  }
  if (tape)
#pragma unroll
    for (int h = 0; h < Q; ++h) tape[ol + h * nl + c] = f[h];
  collide<SCHEME, T>(f, In.sc);
#pragma unroll
  for (int h = 0; h < Q; ++h) Fo[ol + h * nl + c] = f[h];
}

// The detail correction as a call: it concerns few leaves, and inlined its
// addressing would compete for registers with the stencil loads of every leaf.
template <int DIM, typename T>
__device__ __attribute__((noinline)) T detail_correction_call(T acc, int l, int x, int y, const T *__restrict__ Fl,
                                                              const T *__restrict__ Ff, const T *__restrict__ Cw,
                                                              unsigned nbr) {
  return detail_correction<DIM, T>(acc, l, x, y, Fl, Ff, Cw, nbr);
}

// Buffer resource of n values at a wavefront-uniform base (raw buffer, no
// stride; the third word is the CDNA data-format word), and a load at a 32-bit
// byte offset from it: one scalar descriptor per array and one VGPR per
// address. Offsets at or beyond n values would read 0; every offset used here
// is a wrapped cell index of the array's level.
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t pop_rsrc(const T *base, long long n) {
  return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, (int)(n * (long long)sizeof(T)), 0x00020000);
}
template <typename T>
__device__ __forceinline__ T ld_off(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
template <typename T>
using const_ptr = const __attribute__((address_space(4))) T *;

// Row buffers of one wavefront: 68 columns (64 leaves and two on each side)
// per staged row; one row for each x-axis velocity and five for each diagonal
// one, at consecutive slots in population order.
constexpr int ROWBUF = 68;
template <int SCHEME>
__host__ __device__ constexpr int row_slot(int h) {
  int r = 0;
  for (int k = 0; k < h; ++k)
    if (Vel<SCHEME>::ex(k) != 0) r += Vel<SCHEME>::ey(k) == 0 ? 1 : 5;
  return r;
}
template <int SCHEME>
__host__ __device__ constexpr int row_slots() { return row_slot<SCHEME>(Vel<SCHEME>::Q); }

// Order LDS accesses of the lanes of one wavefront: the compiler may not move
// memory operations across it, and the LDS executes a wavefront's operations
// in order.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
}

// leaf_update for a wavefront whose leaves all lie on level l of instance In
// (l, In uniform): the population arrays of level l are uniform buffers, the
// 5^d stencil is a sum of a row and a column byte offset computed once per
// leaf, and the weights of (n, h) are uniform scalar loads. With `row` (2D,
// uniform: the 64 leaves are the consecutive cells x0..x0+63 of one row, lane
// k at x0 + k, above the finest level), the rows of the stencils of the x-axis
// and diagonal velocities are staged once per wavefront in `rowbuf` (68
// columns each, coalesced) and the 5 or 25 values of each leaf are read from
// there. Same operations in the same order as transport_pop.
template <int DIM, int SCHEME, typename T>
__device__ __forceinline__ void leaf_update_level(const Inst<T> &In, int l, uint32_t c, const T *__restrict__ Fs,
                                                  T *__restrict__ Fo, const uint8_t *__restrict__ code,
                                                  const T *__restrict__ Wt, const T *__restrict__ Ct,
                                                  T *__restrict__ tape, bool row, T (*rowbuf)[ROWBUF]) {
  using V = Vel<SCHEME>;
  constexpr int Q = V::Q;
  constexpr int WS = DIM == 2 ? 25 : 5, CS = DIM == 2 ? 36 : 6;
  int x, y;
  coords<DIM>(l, c, x, y);
  const int J = In.jmax, n = J - l;
  const long long nl = ncells_d(DIM, l);
  const T *Fl0 = Fs + (long long)Q * In.loff[l];
  T f[Q];
  if (n == 0) {
#pragma unroll
    for (int h = 0; h < Q; ++h) {
      const uint32_t cs = (uint32_t)cidx<DIM>(l, wrapl(x - V::ex(h), l), wrapl(y - V::ey(h), l));
      f[h] = ld_off<T>(pop_rsrc(Fl0 + h * nl, nl), cs * (uint32_t)sizeof(T));
    }
  } else {
    const uint8_t *cl = code + In.loff[l];
    const unsigned nbr = refined_neighbours<DIM>(cl, l, x, y);
    const T *Ff0 = Fs + (long long)Q * In.loff[l + 1];
    const long long nf = ncells_d(DIM, l + 1);
    const int nn = n - 1;
    const T scale = (T)ldexp(1.0, -DIM * n);
    uint32_t rowb[5], colb[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      rowb[k] = DIM == 2 ? ((uint32_t)wrapl(y + k - 2, l) << l) * (uint32_t)sizeof(T) : 0u;
      colb[k] = (uint32_t)wrapl(x + k - 2, l) * (uint32_t)sizeof(T);
    }
    const uint32_t own = c * (uint32_t)sizeof(T);
    // Stencil sums of every population first, with no call in between, so that
    // the loads of several populations can be in flight together; then the
    // detail corrections (leaves next to finer cells only), then the update.
    T acc[Q], fc[Q];
    const int lane = threadIdx.x & 63;
    if (DIM == 2 && row) {
      // Stage the stencil rows of every x-axis and diagonal velocity at once:
      // all loads first (one memory latency for the chunk), then the LDS writes.
      const uint32_t cst0 = (uint32_t)wrapl(x - 2, l) * (uint32_t)sizeof(T);   // column x0 - 2 + lane
      const uint32_t cst1 = (uint32_t)wrapl(x + 62, l) * (uint32_t)sizeof(T);  // x0 + 62 + lane (lanes 0..3)
      constexpr int NR = row_slots<SCHEME>();
      T v0[NR], v1[NR];
#pragma unroll
      for (int h = 0; h < Q; ++h) {
        if (V::ex(h) == 0) continue;
        const __amdgpu_buffer_rsrc_t base = pop_rsrc(Fl0 + h * nl, nl);
        const int rs = row_slot<SCHEME>(h);
        const int b0 = V::ey(h) == 0 ? 2 : 0, b1 = V::ey(h) == 0 ? 2 : 4;
#pragma unroll
        for (int b = b0; b <= b1; ++b) {
          v0[rs + b - b0] = ld_off<T>(base, rowb[b] + cst0);
          v1[rs + b - b0] = lane < 4 ? ld_off<T>(base, rowb[b] + cst1) : T(0);
        }
      }
      wave_lds_sync();  // the previous chunk's reads of the buffer come first
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        rowbuf[r][lane] = v0[r];
        if (lane < 4) rowbuf[r][64 + lane] = v1[r];
      }
      wave_lds_sync();
    }
#pragma unroll
    for (int h = 0; h < Q; ++h) {
      const int ex = V::ex(h), ey = V::ey(h);
      const __amdgpu_buffer_rsrc_t base = pop_rsrc(Fl0 + h * nl, nl);
      const_ptr<T> W = (const_ptr<T>)(Wt + ((long long)nn * Q + h) * WS);
      if (DIM == 2 && row && ex != 0) {
        // from the staged rows: row y at slot rs (x-axis velocity) or rows
        // y-2 .. y+2 at slots rs .. rs+4 (diagonal)
        const int rs = row_slot<SCHEME>(h);
        fc[h] = rowbuf[ey == 0 ? rs : rs + 2][lane + 2];
        T a_h = T(0);
        if (ey == 0) {
#pragma unroll
          for (int a = 0; a < 5; ++a) a_h = fma(W[10 + a], rowbuf[rs][lane + a], a_h);
        } else {
#pragma unroll
          for (int b = 0; b < 5; ++b)
#pragma unroll
            for (int a = 0; a < 5; ++a) a_h = fma(W[b * 5 + a], rowbuf[rs + b][lane + a], a_h);
        }
        acc[h] = a_h;
        continue;
      }
      fc[h] = ld_off<T>(base, own);
      T a_h = T(0);
      if (ex == 0 && ey == 0) {
      } else if (DIM == 1) {
#pragma unroll
        for (int a = 0; a < 5; ++a) a_h = fma(W[a], ld_off<T>(base, colb[a]), a_h);
      } else if (ey == 0) {
#pragma unroll
        for (int a = 0; a < 5; ++a) a_h = fma(W[10 + a], ld_off<T>(base, rowb[2] + colb[a]), a_h);
      } else if (ex == 0) {
#pragma unroll
        for (int b = 0; b < 5; ++b) a_h = fma(W[b * 5 + 2], ld_off<T>(base, rowb[b] + colb[2]), a_h);
      } else {
#pragma unroll
        for (int b = 0; b < 5; ++b)
#pragma unroll
          for (int a = 0; a < 5; ++a) a_h = fma(W[b * 5 + a], ld_off<T>(base, rowb[b] + colb[a]), a_h);
      }
      acc[h] = a_h;
    }
    if (nbr) {
#pragma unroll
      for (int h = 0; h < Q; ++h) {
        const unsigned m = nbr & correction_mask<DIM>(V::ex(h), V::ey(h), n);
        if ((V::ex(h) != 0 || V::ey(h) != 0) && m)
          acc[h] = detail_correction_call<DIM, T>(acc[h], l, x, y, Fl0 + h * nl, Ff0 + h * nf,
                                                  Ct + ((long long)nn * Q + h) * CS, m);
      }
    }
#pragma unroll
    for (int h = 0; h < Q; ++h) f[h] = (V::ex(h) == 0 && V::ey(h) == 0) ? fc[h] : fma(scale, acc[h], fc[h]);
  }
  const long long ol = (long long)Q * In.loff[l];
  if (tape)
#pragma unroll
    for (int h = 0; h < Q; ++h) tape[ol + h * nl + c] = f[h];
  collide<SCHEME, T>(f, In.sc);
#pragma unroll
  for (int h = 0; h < Q; ++h) Fo[ol + h * nl + c] = f[h];
}

// Variant for large leaf sets: one thread per leaf, all populations in
// registers, no barriers; every wavefront takes a chunk of 64 leaves. Register
// budget for 4 waves per SIMD (latency hiding of the stencil loads). A chunk
// whose leaves share one level (all but those that straddle a level boundary)
// takes leaf_update_level, in row mode when its leaves are one row segment.
template <int DIM, int SCHEME, typename T, int MODE>
__global__ void __launch_bounds__(BLK) __attribute__((amdgpu_waves_per_eu(MODE >= 2 ? 2 : (sizeof(T) == 4 ? 5 : 4))))
    k_transport_collide_leaf(Batch bt, const Inst<T> *__restrict__ I, const T *__restrict__ Fs, T *__restrict__ Fo,
                             const uint8_t *__restrict__ code, const uint32_t *__restrict__ leaves,
                             const int *__restrict__ lvl, const T *__restrict__ Wt, const T *__restrict__ Ct,
                             WallTabs<T> wt, unsigned long long *__restrict__ counters, T *__restrict__ tape) {
  constexpr int WPB = BLK / 64;
  __shared__ SegLDS s;
  __shared__ T rowbuf[WPB][DIM == 2 ? row_slots<SCHEME>() : 1][ROWBUF];
  load_segments(s, I, lvl, bt.B, CAT_LEAF, -1);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    unsigned long long tot = 0;
    for (int i = 0; i < bt.B; ++i) tot += (unsigned long long)s.cnt[i];
    atomicAdd(&counters[0], tot);
    atomicAdd(&counters[1], 1ull);
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  MRLBM_FOR_CHUNKS(ch, s.pre[bt.B], WPB, wave) {
    const int i = __builtin_amdgcn_readfirstlane(upper_index(s.pre, bt.B, ch));
    const int item = (ch - s.pre[i]) * CHUNK + lane;
    const bool valid = item < s.cnt[i];  // lane 0 always is
    const uint32_t e = valid ? leaves[s.beg[i] + item] : 0u;
    const int l = (int)(e >> LEVEL_SHIFT);
    const uint32_t c = e & CELL_MASK;
    const int l0 = __builtin_amdgcn_readfirstlane(l);
    const bool one_level = __ballot(valid && l != l0) == 0;
    // MODE 0: periodic, gamma = 1; 1 (gamma = 1 with walls): leaves whose
    // transport box reaches beyond a wall are left to k_transport_wall_band;
    // MODE = gamma > 1: those leaves take the general path here, the others
    // the path of that gamma
    bool wall = false;
    if constexpr (MODE != 0) {
      int x, y;
      coords<DIM>(l, c, x, y);
      wall = valid && I[i].walls && near_wall<DIM>(I[i], l, x, y);
    }
    // row mode: 64 consecutive cells of one row of a level above the finest
    const uint32_t c0 = __builtin_amdgcn_readfirstlane(c);
    const bool row = DIM == 2 && one_level && l0 < I[i].jmax && __ballot(valid && c == c0 + (uint32_t)lane) == ~0ull &&
                     (c0 & ((1u << l0) - 1)) + 63u < (1u << l0) && __ballot(wall) == 0;
    if (!valid) continue;
    const Inst<T> &In = I[i];
    if (MODE == 1 && wall) continue;  // k_transport_wall_band takes the leaves near a wall
    if constexpr (MODE >= 2) {
      if (wall)
        leaf_update_wall<DIM, SCHEME, T, MODE>(In, l, c, Fs, Fo, code, wt, tape);
      else
        leaf_update_inner_g<DIM, SCHEME, T, MODE>(In, l, c, Fs, Fo, code, wt, tape);
    } else if (one_level)
      leaf_update_level<DIM, SCHEME, T>(In, l0, c, Fs, Fo, code, Wt, Ct, tape, row, rowbuf[wave]);
    else
      leaf_update<DIM, SCHEME, T>(In, l, c, Fs, Fo, code, Wt, Ct, tape);
  }
}

// The leaves whose transport box reaches beyond a wall (batches with gamma = 1
// and walls; the transport kernels leave them out), by the general path. Each
// block takes 64 cells of the wall band of one level of one instance: the rows
// within R = 2 gamma of a y wall, then the columns within R of an x wall in the
// other rows (every cell when the level is at most 2R wide). Wavefront h
// transports population h of the band cells that are complete leaves; the
// collision then runs in wavefront 0 through LDS, as in the per-population
// transport kernel. info[block] = instance | level << 8 | chunk << 13.
constexpr int WBAND_CHUNK = 64;
template <int DIM, int SCHEME, typename T>
__global__ void __launch_bounds__(64 * Vel<SCHEME>::Q)
    k_transport_wall_band(const Inst<T> *__restrict__ I, const T *__restrict__ Fs, T *__restrict__ Fo,
                          const uint8_t *__restrict__ code, const uint32_t *__restrict__ info, WallTabs<T> wt,
                          T *__restrict__ tape) {
  constexpr int Q = Vel<SCHEME>::Q;
  __shared__ T fl[Q][64];
  const uint32_t w = info[blockIdx.x];
  const int i = (int)(w & 0xffu), l = (int)((w >> 8) & 0x1fu);
  const int h = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long long k = (long long)(w >> 13) * WBAND_CHUNK + lane;
  const Inst<T> &In = I[i];
  const int N = 1 << l, R = 2 * In.gamma;
  const bool wx = In.walls & 1, wy = DIM == 2 && (In.walls & 2);
  const int rows = wy ? min(2 * R, N) : 0;                   // rows of the y band
  const int cols = wx ? min(2 * R, N) : 0;                   // columns of the x band
  const long long ny = DIM == 2 ? (long long)(N - rows) : 1;  // rows left to the x band
  int x = 0, y = 0;
  bool in = true;
  if (k < (long long)rows * N) {
    const int r = (int)(k / N);
    x = (int)(k - (long long)r * N);
    y = r < R ? r : N - rows + r;
  } else {
    const long long kk = k - (long long)rows * N;
    in = kk < ny * cols;
    const int r = in ? (int)(kk / cols) : 0, cc = in ? (int)(kk - (long long)r * cols) : 0;
    y = DIM == 2 ? (wy ? R : 0) + r : 0;
    x = cc < R ? cc : N - cols + cc;
  }
  const uint32_t c = (uint32_t)cidx<DIM>(l, x, y);
  const bool leaf = in && code[In.loff[l] + c] == C_LEAF;
  const long long ol = (long long)Q * In.loff[l], nl = ncells_d(DIM, l);
  if (leaf) {
    const T *Ff0 = l < In.jmax ? Fs + (long long)Q * In.loff[l + 1] : Fs;
    fl[h][lane] = transport_wall<DIM, SCHEME, T, 1>(In, h, l, c, x, y, Fs + ol, Ff0, code + In.loff[l], wt);
    if (tape) tape[ol + h * nl + c] = fl[h][lane];
  }
  __syncthreads();
  if (h == 0 && leaf) {
    T g[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) g[q] = fl[q][lane];
    collide<SCHEME, T>(g, In.sc);
#pragma unroll
    for (int q = 0; q < Q; ++q) fl[q][lane] = g[q];
  }
  __syncthreads();
  if (leaf) Fo[ol + h * nl + c] = fl[h][lane];
}

// ---------------------------------------------------------------- init / diagnostics
template <int DIM, int SCHEME, typename T>
__global__ void __launch_bounds__(BLK) k_init_equilibrium(const Inst<T> *__restrict__ I, int i, T *__restrict__ F,
                                                          const T *__restrict__ mom) {
  using V = Vel<SCHEME>;
  const Inst<T> &In = I[i];
  const long long n = ncells_d(DIM, In.jmax);
  for (long long c = blockIdx.x * (long long)BLK + threadIdx.x; c < n; c += (long long)gridDim.x * BLK) {
    T mc[V::NC], f[V::Q];
    for (int k = 0; k < V::NC; ++k) mc[k] = mom[k * n + c];
    equilibrium_populations<SCHEME, T>(mc, f, In.sc);
    for (int h = 0; h < V::Q; ++h) F[foff(In, DIM, V::Q, In.jmax, h) + c] = f[h];
  }
}

constexpr int RED_BLOCKS = 64;

// Compensated summation (Neumaier's variant of Kahan's): s + c carries the
// rounding error of every addition into s. Needs unfused, unreassociated
// double arithmetic (the library is built with -ffp-contract=off).
__device__ __forceinline__ void neumaier_add(double &s, double &c, double t) {
  const double u = s + t;
  c += fabs(s) >= fabs(t) ? (s - u) + t : (t - u) + s;
  s = u;
}

// Mass partial sums of instance blockIdx.y (fixed grid and order, so the result
// is reproducible) and its non-finite flag bad[i].
template <int DIM, int Q, typename T>
__global__ void __launch_bounds__(BLK) k_mass_partial(Batch bt, const Inst<T> *__restrict__ I, const T *__restrict__ F,
                                                      const uint32_t *__restrict__ leaves, const int *__restrict__ lvl,
                                                      double *__restrict__ part, int *__restrict__ bad) {
  __shared__ double red_s[BLK], red_c[BLK];
  const int i = blockIdx.y;
  const Inst<T> &In = I[i];
  const int *L = lvl + (i * NCAT + CAT_LEAF) * LVL_STRIDE;
  const int beg = L[In.jmin], n = L[In.jmax + 1] - beg;
  double acc = 0.0, comp = 0.0;
  int nonfinite = 0;
  for (int k = blockIdx.x * BLK + threadIdx.x; k < n; k += gridDim.x * BLK) {
    const uint32_t e = leaves[beg + k];
    const int l = (int)(e >> LEVEL_SHIFT);
    const uint32_t c = e & CELL_MASK;
    for (int h = 0; h < Q; ++h) {
      const double v = (double)F[foff(In, DIM, Q, l, h) + c];
      nonfinite |= !isfinite(v);
      neumaier_add(acc, comp, ldexp(v, DIM * (In.jmax - l)));  // the volume factor is exact
    }
  }
  red_s[threadIdx.x] = acc;
  red_c[threadIdx.x] = comp;
  __syncthreads();
  for (int off = BLK / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      double s2 = red_s[threadIdx.x], c2 = red_c[threadIdx.x] + red_c[threadIdx.x + off];
      neumaier_add(s2, c2, red_s[threadIdx.x + off]);
      red_s[threadIdx.x] = s2;
      red_c[threadIdx.x] = c2;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * (i * RED_BLOCKS + blockIdx.x)] = red_s[0];
    part[2 * (i * RED_BLOCKS + blockIdx.x) + 1] = red_c[0];
  }
  if (nonfinite) atomicOr(bad + i, 1);
}

template <int DIM, int Q, typename T>
__global__ void __launch_bounds__(BLK) k_export(const Inst<T> *__restrict__ I, int i, const T *__restrict__ F,
                                                const uint32_t *__restrict__ leaves, const int *__restrict__ lvl,
                                                uint32_t *__restrict__ cells, T *__restrict__ vals) {
  const Inst<T> &In = I[i];
  const int *L = lvl + (i * NCAT + CAT_LEAF) * LVL_STRIDE;
  const int beg = L[In.jmin], n = L[In.jmax + 1] - beg;
  for (int k = blockIdx.x * BLK + threadIdx.x; k < n; k += gridDim.x * BLK) {
    const uint32_t e = leaves[beg + k];
    const int l = (int)(e >> LEVEL_SHIFT);
    const uint32_t c = e & CELL_MASK;
    if (cells) cells[k] = e;
    if (vals)
      for (int h = 0; h < Q; ++h) vals[(long long)k * Q + h] = F[foff(In, DIM, Q, l, h) + c];
  }
}

// Moments m = M f of every complete leaf of instance i, [leaf][k] in the order
// (level, cell) of the leaf list (the moment bases of the collision: section
// "Lattice Boltzmann schemes on volumes", and the D2Q9 matrix of the
// incompressible Navier-Stokes section).
template <int DIM, int SCHEME, typename T>
__global__ void __launch_bounds__(BLK) k_moments(const Inst<T> *__restrict__ I, int i, const T *__restrict__ F,
                                                 const uint32_t *__restrict__ leaves, const int *__restrict__ lvl,
                                                 T *__restrict__ out) {
  constexpr int Q = Vel<SCHEME>::Q;
  const Inst<T> &In = I[i];
  const int *L = lvl + (i * NCAT + CAT_LEAF) * LVL_STRIDE;
  const int beg = L[In.jmin], n = L[In.jmax + 1] - beg;
  for (int k = blockIdx.x * BLK + threadIdx.x; k < n; k += gridDim.x * BLK) {
    const uint32_t e = leaves[beg + k];
    const int l = (int)(e >> LEVEL_SHIFT);
    const uint32_t c = e & CELL_MASK;
    T f[Q], m[Q];
#pragma unroll
    for (int h = 0; h < Q; ++h) f[h] = F[foff(In, DIM, Q, l, h) + c];
    moments<SCHEME, T>(f, m, In.sc.lam);
#pragma unroll
    for (int h = 0; h < Q; ++h) out[(long long)k * Q + h] = m[h];
  }
}

// Reconstruction of level l of instance i on every cell outside the complete
// tree (ghost or not): the zero-detail prediction from level l-1, which holds
// the reconstruction of that level. Applied for l = jmin+1 .. J in order after
// the reconstruction of the tree, it gives the double-hat reconstruction on
// the finest level (section "Mesh coarsening"). Ghosts get the value they
// already hold (same expression); values of tree cells are not touched.
template <int DIM, int Q, typename T, int GAM>
__global__ void __launch_bounds__(BLK) k_predict_outside(const Inst<T> *__restrict__ I, int i, T *__restrict__ F,
                                                         const uint8_t *__restrict__ code, int l) {
  const Inst<T> &In = I[i];
  const long long n = ncells_d(DIM, l);
  const uint8_t *cl = code + In.loff[l];
  for (long long c = blockIdx.x * (long long)BLK + threadIdx.x; c < n; c += (long long)gridDim.x * BLK) {
    if (cl[c] >= C_INTERNAL) continue;
    int x, y;
    coords<DIM>(l, (uint32_t)c, x, y);
#pragma unroll
    for (int h = 0; h < Q; ++h)
      F[foff(In, DIM, Q, l, h) + c] =
          predict<DIM, T>(F + foff(In, DIM, Q, l - 1, h), l, x, y, In.walls, gamma_k<GAM>(In));
  }
}

}  // namespace mrlbm
