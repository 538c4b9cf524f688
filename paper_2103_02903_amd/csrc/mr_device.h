// Device-side building blocks of the MR-LBM step: level geometry, the gamma = 1
// projection / prediction operators, and the collision of each scheme.
//
// Storage is dense-addressed per level: level l owns N_l^d slots (N_l = 2^l) per
// population, laid out [level][h][cell] with cell = x + (y << l). Only cells of
// the complete tree, ghost cells and leaves are ever read or written, so the
// traffic is proportional to the number of leaves while every neighbour lookup
// is a plain address computation (no hashing, no rank tables).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mrlbm {

constexpr int MAXLEV = 32;
constexpr int LEVEL_SHIFT = 26;                      // list entry = (level << 26) | cell
constexpr uint32_t CELL_MASK = (1u << LEVEL_SHIFT) - 1;
constexpr int LVL_STRIDE = MAXLEV + 2;               // per-category stride of level offsets

// Cell codes of a mesh.
enum : uint8_t { C_NONE = 0, C_GHOST = 1, C_INTERNAL = 2, C_LEAF = 3 };
// List categories produced by the compaction.
enum { CAT_LEAF = 0, CAT_INTERNAL = 1, CAT_GHOST = 2, NCAT = 3 };

template <typename T>
struct SchemeC {
  T lam, inv_lam, eq;  // lattice velocity, its inverse, V (D1Q2), alpha (D1Q3) or gamma_gas (Euler)
  T s[16];
  T vel[3];            // D3Q6: the advection velocity (V_x, V_y, V_z)
};

// One simulation of a batch. Per-cell arrays (codes, flags, lists) of all
// instances are concatenated; instance i owns cells [cbase, cbase + total) and
// the list slots with the same indices in every category. Populations are laid
// out [instance][level][h][cell].
template <typename T>
struct Inst {
  int jmin, jmax;
  long long cbase, total;
  long long loff[MAXLEV + 2];  // absolute first cell of level l; loff[jmax + 1] = cbase + total
  int bstart[MAXLEV + 2];      // absolute first compaction block of level l; bstart[jmax + 1] = end
  T eps_l[MAXLEV + 2];         // eps_l = 2^{d (l - J)} eps, indexed by the level of the children
  T ref_l[MAXLEV + 2];         // 2^{mu_bar + d} eps_l
  SchemeC<T> sc;
  // Boundaries (section "Boundary conditions"): bit 0 walls on the x axis, bit
  // 1 on the y axis (else periodic); kind of each side x-, x+, y-, y+ (1 copy,
  // 2 bounce back, 3 anti bounce back, 0 periodic).
  int walls;
  int bck[4];
  // Prediction stencil half-width gamma (1..3, Table 1; the same for the whole
  // batch) and the sibling metric of the details: 0 the max norm, 1 the l2
  // form 2^{-d/2} (sum d^2)^{1/2}, kept squared (eps_l and ref_l are then the
  // squared thresholds).
  int gamma;
  int metric;
};

// Batch-wide constants (passed by value).
struct Batch {
  int B, dim, q, jmin, maxJ;
  long long ctotal;  // cells of all instances
};

__device__ __forceinline__ long long ncells_d(int dim, int l) { return 1ll << (dim * l); }
template <typename T>
__device__ __forceinline__ long long foff(const Inst<T> &I, int dim, int q, int l, int h) {
  return (long long)q * I.loff[l] + (long long)h * ncells_d(dim, l);
}
__device__ __forceinline__ int wrapl(int x, int l) { return x & ((1 << l) - 1); }
// Index x (|overflow| <= N_l) of level l along an axis as the MR operators read
// it: periodic wrap, or with a wall even reflection (cell -1 reads cell 0, cell
// N_l reads cell N_l - 1). The prediction stencil is symmetric, so reflection
// commutes with it: the reconstruction near a wall is that of the mirrored
// periodic problem.
__device__ __forceinline__ int axl(int x, int l, bool wall) {
  if (!wall) return wrapl(x, l);
  const int n = 1 << l;
  return x < 0 ? -1 - x : (x >= n ? 2 * n - 1 - x : x);
}
// The same for a neighbour at distance 1 (x in [-1, N_l]), where reflection is
// a clamp: no branch, one select.
__device__ __forceinline__ int axl1(int x, int l, bool wall) {
  const int w = wrapl(x, l), c = min(max(x, 0), (1 << l) - 1);
  return wall ? c : w;
}
template <int DIM>
__device__ __forceinline__ long long cidx(int l, int x, int y) {
  return DIM == 1 ? (long long)x : (long long)x + ((long long)y << l);
}
template <int DIM>
__device__ __forceinline__ void coords(int l, uint32_t c, int &x, int &y) {
  if (DIM == 1) { x = (int)c; y = 0; }
  else { x = (int)(c & ((1u << l) - 1)); y = (int)(c >> l); }
}
// Largest i in [0, n) with a[i] <= v (a non-decreasing, a[0] <= v).
template <typename I>
__device__ __forceinline__ int upper_index(const I *a, int n, long long v) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((long long)a[mid] <= v) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------- MR operators
// Table 1: the coefficients c_1 .. c_gamma of the prediction of half-width
// gamma (exact dyadic rationals, exact in float as well).
__host__ __device__ constexpr double table1(int g, int a) {
  return g == 1 ? -0.125
         : g == 2 ? (a == 1 ? -22.0 / 128 : 3.0 / 128)
                  : (a == 1 ? -201.0 / 1024 : (a == 2 ? 11.0 / 256 : -5.0 / 1024));
}

// Prediction (gamma = 1, c_1 = -1/8): with P the data of level l-1 around the
// parent (px, py) of a child,
//   1D: child = P(p) + s_x Qx,                      Qx = c_1 (P(p+1) - P(p-1)),
//   2D: child = ((P(p) + s_x Qx) + s_y Qy) + s_x s_y Qxy,
//       Qxy = c_1^2 (((P(+,+) - P(-,+)) - P(+,-)) + P(-,-)),
// with s = +1 for the lower child and -1 for the upper one along each axis
// (tensor product of the 1D operator). The evaluation order is part of the
// contract: details decide the mesh, which must not depend on rounding order.
// `walls` (Inst::walls) selects reflection instead of wrap per axis. With
// gamma > 1 (Table 1): Qx = c_1 (P(+1) - P(-1)), then + c_a (P(+a) - P(-a)) for
// a = 2..gamma; Qy alike; Qxy the sum of c_a c_b (((P(+a,+b) - P(-a,+b)) -
// P(+a,-b)) + P(-a,-b)) starting with (a, b) = (1, 1), then b = 1, a = 2..gamma,
// then b = 2..gamma, a = 1..gamma.
template <int DIM, typename T>
struct ParentStencil {
  T c, qx, qy, qxy;
  __device__ __noinline__ void load_wide(const T *__restrict__ P, int lp, int px, int py, int walls, int g) {
    const bool wx = walls & 1, wy = walls & 2;
    auto at = [&](int a, int b) -> T {
      return DIM == 1 ? P[axl(px + a, lp, wx)] : P[cidx<2>(lp, axl(px + a, lp, wx), axl(py + b, lp, wy))];
    };
    c = at(0, 0);
    qx = T(table1(g, 1)) * (at(1, 0) - at(-1, 0));
    for (int a = 2; a <= g; ++a) qx = qx + T(table1(g, a)) * (at(a, 0) - at(-a, 0));
    if (DIM == 1) {
      qy = T(0);
      qxy = T(0);
      return;
    }
    qy = T(table1(g, 1)) * (at(0, 1) - at(0, -1));
    for (int b = 2; b <= g; ++b) qy = qy + T(table1(g, b)) * (at(0, b) - at(0, -b));
    auto term = [&](int a, int b) -> T {
      return T(table1(g, a) * table1(g, b)) * (((at(a, b) - at(-a, b)) - at(a, -b)) + at(-a, -b));
    };
    qxy = term(1, 1);
    for (int b = 1; b <= g; ++b)
      for (int a = (b == 1 ? 2 : 1); a <= g; ++a) qxy = qxy + term(a, b);
  }
  __device__ __forceinline__ void load(const T *__restrict__ P, int lp, int px, int py, int walls, int g = 1) {
    if (g > 1) {
      load_wide(P, lp, px, py, walls, g);
      return;
    }
    const T c1 = T(-0.125);
    const bool wx = walls & 1, wy = walls & 2;
    if (DIM == 1) {
      c = P[px];
      qx = c1 * (P[axl1(px + 1, lp, wx)] - P[axl1(px - 1, lp, wx)]);
      qy = T(0);
      qxy = T(0);
    } else {
      const int xm = axl1(px - 1, lp, wx), xp = axl1(px + 1, lp, wx);
      const int ym = axl1(py - 1, lp, wy), yp = axl1(py + 1, lp, wy);
      c = P[cidx<2>(lp, px, py)];
      qx = c1 * (P[cidx<2>(lp, xp, py)] - P[cidx<2>(lp, xm, py)]);
      qy = c1 * (P[cidx<2>(lp, px, yp)] - P[cidx<2>(lp, px, ym)]);
      qxy = T(0.015625) * (((P[cidx<2>(lp, xp, yp)] - P[cidx<2>(lp, xm, yp)]) - P[cidx<2>(lp, xp, ym)]) +
                           P[cidx<2>(lp, xm, ym)]);
    }
  }
  // child offset (dx, dy) in {0, 1}^d
  __device__ __forceinline__ T child(int dx, int dy) const {
    const T sx = dx ? T(-1) : T(1);
    if (DIM == 1) return c + sx * qx;
    const T sy = dy ? T(-1) : T(1);
    return ((c + sx * qx) + sy * qy) + (sx * sy) * qxy;
  }
};

// The prediction half-width of an instance as a kernel sees it: GAM = 1 for the
// kernels of batches with gamma = 1 (a constant: the wide stencil code is left
// out of them), GAM = 0 for the others (the instance's value).
template <int GAM, typename T>
__device__ __forceinline__ int gamma_k(const Inst<T> &In) {
  return GAM == 1 ? 1 : In.gamma;
}

template <int DIM, typename T>
__device__ __forceinline__ T predict(const T *__restrict__ P, int l, int cx, int cy, int walls, int g) {
  ParentStencil<DIM, T> s;
  s.load(P, l - 1, cx >> 1, cy >> 1, walls, g);
  return s.child(cx & 1, cy & 1);
}

// Projection: average of the 2^d children, 1D 0.5 (a0 + a1),
// 2D 0.25 (((a00 + a10) + a01) + a11) with x fastest.
template <int DIM, typename T>
__device__ __forceinline__ T project(const T *__restrict__ C, int lc, int px, int py) {
  if (DIM == 1) return T(0.5) * (C[2 * px] + C[2 * px + 1]);
  const long long r0 = cidx<2>(lc, 2 * px, 2 * py), r1 = cidx<2>(lc, 2 * px, 2 * py + 1);
  return T(0.25) * (((C[r0] + C[r0 + 1]) + C[r1]) + C[r1 + 1]);
}

// ---------------------------------------------------------------- schemes
template <int SCHEME>
struct Vel;
template <>
struct Vel<1> {  // D1Q2
  static constexpr int Q = 2, DIM = 1, NC = 1;
  __host__ __device__ static constexpr int ex(int h) { return h == 0 ? 1 : -1; }
  __host__ __device__ static constexpr int ey(int) { return 0; }
};
template <>
struct Vel<2> {  // D1Q3
  static constexpr int Q = 3, DIM = 1, NC = 1;
  __host__ __device__ static constexpr int ex(int h) { return h == 0 ? 0 : (h == 1 ? 1 : -1); }
  __host__ __device__ static constexpr int ey(int) { return 0; }
};
template <>
struct Vel<4> {  // Euler system: four D2Q4 schemes, population 4 i + k is velocity k of variable i
  static constexpr int Q = 16, DIM = 2, NC = 4;
  __host__ __device__ static constexpr int ex(int h) { return (h & 3) == 0 ? 1 : ((h & 3) == 2 ? -1 : 0); }
  __host__ __device__ static constexpr int ey(int h) { return (h & 3) == 1 ? 1 : ((h & 3) == 3 ? -1 : 0); }
};
template <>
struct Vel<5> {  // D3Q6: lambda cos(pi h) along x (h = 0, 1), y (2, 3) and z (4, 5)
  static constexpr int Q = 6, DIM = 3, NC = 1;
  __host__ __device__ static constexpr int ex(int h) { return h == 0 ? 1 : (h == 1 ? -1 : 0); }
  __host__ __device__ static constexpr int ey(int h) { return h == 2 ? 1 : (h == 3 ? -1 : 0); }
  __host__ __device__ static constexpr int ez(int h) { return h == 4 ? 1 : (h == 5 ? -1 : 0); }
};
template <>
struct Vel<3> {  // D2Q9: rest, four axis velocities, four diagonals
  static constexpr int Q = 9, DIM = 2, NC = 3;
  __host__ __device__ static constexpr int ex(int h) {
    return h == 1 || h == 5 || h == 8 ? 1 : (h == 3 || h == 6 || h == 7 ? -1 : 0);
  }
  __host__ __device__ static constexpr int ey(int h) {
    return h == 2 || h == 5 || h == 6 ? 1 : (h == 4 || h == 7 || h == 8 ? -1 : 0);
  }
};

// D2Q9 moments m = M f (Lallemand-Luo basis, rows scaled by powers of lambda).
template <typename T>
__device__ __forceinline__ void d2q9_moments(const T *f, T *m, T L) {
  const T L2 = L * L, L3 = L2 * L, L4 = L2 * L2;
  const T sa = f[1] + f[2] + f[3] + f[4], sd = f[5] + f[6] + f[7] + f[8];
  m[0] = f[0] + sa + sd;
  m[1] = L * (f[1] - f[3] + f[5] - f[6] - f[7] + f[8]);
  m[2] = L * (f[2] - f[4] + f[5] + f[6] - f[7] - f[8]);
  m[3] = L2 * (T(-4) * f[0] - sa + T(2) * sd);
  m[4] = L3 * (T(-2) * f[1] + T(2) * f[3] + f[5] - f[6] - f[7] + f[8]);
  m[5] = L3 * (T(-2) * f[2] + T(2) * f[4] + f[5] + f[6] - f[7] - f[8]);
  m[6] = L4 * (T(4) * f[0] - T(2) * sa + sd);
  m[7] = L2 * (f[1] - f[2] + f[3] - f[4]);
  m[8] = L2 * (f[5] - f[6] + f[7] - f[8]);
}

// Lallemand-Luo equilibrium of the non-conserved moments 3..8, c_s^2 = lambda^2 / 3.
template <typename T>
__device__ __forceinline__ void d2q9_equilibrium(T rho, T qx, T qy, T L, T *e) {
  const T cs2 = (L * L) / T(3), irho = T(1) / rho, q2 = qx * qx + qy * qy;
  e[3] = T(3) * (T(-2) * cs2 * rho + q2 * irho);
  e[4] = T(-3) * cs2 * qx;
  e[5] = T(-3) * cs2 * qy;
  e[6] = T(9) * (cs2 * cs2 * rho - cs2 * q2 * irho);
  e[7] = (qx * qx - qy * qy) * irho;
  e[8] = qx * qy * irho;
}

// f = M^{-1} m. The rows of M are orthogonal, so M^{-1} = M^T diag(1 / |row|^2).
template <typename T>
__device__ __forceinline__ void d2q9_populations(const T *m, T *f, T il) {
  const T il2 = il * il, il3 = il2 * il, il4 = il2 * il2;
  const T a0 = m[0] * T(1.0 / 9.0), a1 = m[1] * il * T(1.0 / 6.0), a2 = m[2] * il * T(1.0 / 6.0);
  const T a3 = m[3] * il2 * T(1.0 / 36.0), a4 = m[4] * il3 * T(1.0 / 12.0), a5 = m[5] * il3 * T(1.0 / 12.0);
  const T a6 = m[6] * il4 * T(1.0 / 36.0), a7 = m[7] * il2 * T(0.25), a8 = m[8] * il2 * T(0.25);
  f[0] = a0 - T(4) * a3 + T(4) * a6;
  f[1] = a0 + a1 - a3 - T(2) * a4 - T(2) * a6 + a7;
  f[2] = a0 + a2 - a3 - T(2) * a5 - T(2) * a6 - a7;
  f[3] = a0 - a1 - a3 + T(2) * a4 - T(2) * a6 + a7;
  f[4] = a0 - a2 - a3 + T(2) * a5 - T(2) * a6 - a7;
  f[5] = a0 + a1 + a2 + T(2) * a3 + a4 + a5 + a6 + a8;
  f[6] = a0 - a1 + a2 + T(2) * a3 - a4 + a5 + a6 - a8;
  f[7] = a0 - a1 - a2 + T(2) * a3 - a4 - a5 + a6 + a8;
  f[8] = a0 + a1 - a2 + T(2) * a3 + a4 - a5 + a6 - a8;
}

// Vectorial D2Q4 scheme of the Euler system (section "Systems of hyperbolic
// conservation laws"): variable i (rho, rho u, rho v, E) has its own D2Q4 scheme
// with moments m0 = sum f, m1 = lambda (f0 - f2), m2 = lambda (f1 - f3),
// m3 = lambda^2 (f0 - f1 + f2 - f3), relaxed towards (u_i, Phi_x,i(u),
// Phi_y,i(u), 0); the fluxes couple the four. M^{-1} in the closed form of the
// orthogonal rows: f0 = m0/4 + m1/(2 lambda) + m3/(4 lambda^2), f2 with -m1,
// f1 = m0/4 + m2/(2 lambda) - m3/(4 lambda^2), f3 with -m2.
template <typename T>
__device__ __forceinline__ void euler_fluxes(const T *u, T gam, T *fx, T *fy) {
  const T rho = u[0], mx = u[1], my = u[2], E = u[3];
  const T ir = T(1) / rho, vx = mx * ir, vy = my * ir;
  const T p = (gam - T(1)) * (E - T(0.5) * rho * (vx * vx + vy * vy));
  fx[0] = mx;
  fx[1] = mx * vx + p;
  fx[2] = mx * vy;
  fx[3] = vx * (E + p);
  fy[0] = my;
  fy[1] = my * vx;
  fy[2] = my * vy + p;
  fy[3] = vy * (E + p);
}
template <typename T>
__device__ __forceinline__ void d2q4_populations(T m0, T m1, T m2, T m3, T il, T *f) {
  const T a = T(0.25) * m0, b = T(0.5) * il * m1, c = T(0.5) * il * m2, d = T(0.25) * (il * il) * m3;
  f[0] = (a + b) + d;
  f[1] = (a + c) - d;
  f[2] = (a - b) + d;
  f[3] = (a - c) - d;
}

// D3Q6 (section "Three dimensional advection equation"): with a = f0 + f1,
// b = f2 + f3, c = f4 + f5 the moments are m0 = a + b + c, m1..m3 = lambda
// (f0 - f1, f2 - f3, f4 - f5), m4 = lambda^2 (a - b), m5 = lambda^2 (a - c);
// M^{-1}: a = (m0 + (m4 + m5) / lambda^2) / 3, b = a - m4 / lambda^2,
// c = a - m5 / lambda^2, f0 = (a + m1 / lambda) / 2, f1 = (a - m1 / lambda) / 2,
// and alike along y and z.
template <typename T>
__device__ __forceinline__ void d3q6_moments(const T *f, T *m, T L) {
  const T a = f[0] + f[1], b = f[2] + f[3], c = f[4] + f[5];
  m[0] = (a + b) + c;
  m[1] = L * (f[0] - f[1]);
  m[2] = L * (f[2] - f[3]);
  m[3] = L * (f[4] - f[5]);
  m[4] = (L * L) * (a - b);
  m[5] = (L * L) * (a - c);
}
template <typename T>
__device__ __forceinline__ void d3q6_populations(const T *m, T *f, T il) {
  const T il2 = il * il, d4 = m[4] * il2, d5 = m[5] * il2;
  const T a = (m[0] + (d4 + d5)) * T(1.0 / 3.0), b = a - d4, c = a - d5;
  const T u = m[1] * il, v = m[2] * il, w = m[3] * il;
  f[0] = T(0.5) * (a + u);
  f[1] = T(0.5) * (a - u);
  f[2] = T(0.5) * (b + v);
  f[3] = T(0.5) * (b - v);
  f[4] = T(0.5) * (c + w);
  f[5] = T(0.5) * (c - w);
}

// Collision in moment space: f^* = M^{-1} (m + S (m_eq(m) - m)), m = M f; the
// conserved moments (s = 0) are passed through untouched.
template <int SCHEME, typename T>
__device__ __forceinline__ void collide(T *f, const SchemeC<T> &sc) {
  if constexpr (SCHEME == 5) {  // m_eq = (u, V_x u, V_y u, V_z u, 0, 0)
    T m[6];
    d3q6_moments(f, m, sc.lam);
    m[1] = m[1] + sc.s[1] * (sc.vel[0] * m[0] - m[1]);
    m[2] = m[2] + sc.s[2] * (sc.vel[1] * m[0] - m[2]);
    m[3] = m[3] + sc.s[3] * (sc.vel[2] * m[0] - m[3]);
    m[4] = m[4] + sc.s[4] * (T(0) - m[4]);
    m[5] = m[5] + sc.s[5] * (T(0) - m[5]);
    d3q6_populations(m, f, sc.inv_lam);
  } else if constexpr (SCHEME == 1) {
    const T m0 = f[0] + f[1];
    T m1 = sc.lam * (f[0] - f[1]);
    m1 = m1 + sc.s[1] * (sc.eq * m0 - m1);
    const T a = m1 * sc.inv_lam;
    f[0] = T(0.5) * (m0 + a);
    f[1] = T(0.5) * (m0 - a);
  } else if constexpr (SCHEME == 2) {
    const T m0 = f[0] + f[1] + f[2];
    T m1 = sc.lam * (f[1] - f[2]);
    T m2 = (sc.lam * sc.lam) * (f[1] + f[2]);
    m1 = m1 + sc.s[1] * (T(0.5) * m0 * m0 - m1);
    m2 = m2 + sc.s[2] * (sc.eq * (sc.lam * sc.lam) * m0 - m2);
    const T a = m2 * (sc.inv_lam * sc.inv_lam), b = m1 * sc.inv_lam;
    f[0] = m0 - a;
    f[1] = T(0.5) * (a + b);
    f[2] = T(0.5) * (a - b);
  } else if constexpr (SCHEME == 4) {
    T u[4], m1[4], m2[4], m3[4], fx[4], fy[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const T *g = f + 4 * i;
      u[i] = ((g[0] + g[1]) + g[2]) + g[3];
      m1[i] = sc.lam * (g[0] - g[2]);
      m2[i] = sc.lam * (g[1] - g[3]);
      m3[i] = (sc.lam * sc.lam) * ((g[0] - g[1]) + (g[2] - g[3]));
    }
    euler_fluxes(u, sc.eq, fx, fy);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const T a = m1[i] + sc.s[4 * i + 1] * (fx[i] - m1[i]);
      const T b = m2[i] + sc.s[4 * i + 2] * (fy[i] - m2[i]);
      const T c = m3[i] + sc.s[4 * i + 3] * (T(0) - m3[i]);
      d2q4_populations(u[i], a, b, c, sc.inv_lam, f + 4 * i);
    }
  } else {
    T m[9], e[9];
    d2q9_moments(f, m, sc.lam);
    d2q9_equilibrium(m[0], m[1], m[2], sc.lam, e);
#pragma unroll
    for (int i = 3; i < 9; ++i) m[i] = m[i] + sc.s[i] * (e[i] - m[i]);
    d2q9_populations(m, f, sc.inv_lam);
  }
}

// Moments m = M f of one cell (the same bases as the collision below).
template <int SCHEME, typename T>
__device__ __forceinline__ void moments(const T *f, T *m, T L) {
  if constexpr (SCHEME == 5) {
    d3q6_moments(f, m, L);
  } else if constexpr (SCHEME == 1) {
    m[0] = f[0] + f[1];
    m[1] = L * (f[0] - f[1]);
  } else if constexpr (SCHEME == 2) {
    m[0] = f[0] + f[1] + f[2];
    m[1] = L * (f[1] - f[2]);
    m[2] = (L * L) * (f[1] + f[2]);
  } else if constexpr (SCHEME == 4) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const T *g = f + 4 * i;
      m[4 * i] = ((g[0] + g[1]) + g[2]) + g[3];
      m[4 * i + 1] = L * (g[0] - g[2]);
      m[4 * i + 2] = L * (g[1] - g[3]);
      m[4 * i + 3] = (L * L) * ((g[0] - g[1]) + (g[2] - g[3]));
    }
  } else {
    d2q9_moments(f, m, L);
  }
}

// f = M^{-1} m_eq(m) from the conserved moments (initial datum of Algorithm 1).
template <int SCHEME, typename T>
__device__ __forceinline__ void equilibrium_populations(const T *mc, T *f, const SchemeC<T> &sc) {
  if constexpr (SCHEME == 5) {
    const T m[6] = {mc[0], sc.vel[0] * mc[0], sc.vel[1] * mc[0], sc.vel[2] * mc[0], T(0), T(0)};
    d3q6_populations(m, f, sc.inv_lam);
  } else if constexpr (SCHEME == 1) {
    const T a = (sc.eq * mc[0]) * sc.inv_lam;
    f[0] = T(0.5) * (mc[0] + a);
    f[1] = T(0.5) * (mc[0] - a);
  } else if constexpr (SCHEME == 2) {
    const T u = mc[0];
    const T m1 = T(0.5) * u * u, m2 = sc.eq * (sc.lam * sc.lam) * u;
    const T a = m2 * (sc.inv_lam * sc.inv_lam), b = m1 * sc.inv_lam;
    f[0] = u - a;
    f[1] = T(0.5) * (a + b);
    f[2] = T(0.5) * (a - b);
  } else if constexpr (SCHEME == 4) {
    T fx[4], fy[4];
    euler_fluxes(mc, sc.eq, fx, fy);
#pragma unroll
    for (int i = 0; i < 4; ++i) d2q4_populations(mc[i], fx[i], fy[i], T(0), sc.inv_lam, f + 4 * i);
  } else {
    T m[9];
    m[0] = mc[0];
    m[1] = mc[1];
    m[2] = mc[2];
    d2q9_equilibrium(mc[0], mc[1], mc[2], sc.lam, m);
    d2q9_populations(m, f, sc.inv_lam);
  }
}

}  // namespace mrlbm
