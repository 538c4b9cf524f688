/*
 * Plain FP64 CPU oracle of the multiresolution-adapted lattice Boltzmann step
 * (Bellotti, Gouarin, Graille, Massot, arXiv 2103.02903).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark; never by the GPU library, with which it shares
 * no code. Build with -ffp-contract=off and without fast-math: the prediction,
 * projection and detail expressions below are evaluated in the order written.
 * Loops whose iterations write disjoint cells from read-only inputs carry an
 * OpenMP pragma (a build with -fopenmp spreads them over the host cores), and
 * the scatters of the adjoint run one population per thread, each in its
 * serial order; no reduction is parallel, so every result is independent of
 * the thread count, bit for bit.
 *
 * Readings of the paper taken here (each is listed with its justification in
 * the design notes of the repository):
 *  - 2D prediction: the cross term enters with the tensor-product sign
 *    +(-1)^{dx+dy} Q_xy (Appendix 2 builds the 2D operator as a Kronecker
 *    product of the 1D one); only this sign is exact on the monomial x*y.
 *    3D likewise: every pair term with +(-1)^{da+db} and the triple term with
 *    +(-1)^{dx+dy+dz} (the Kronecker product of three 1D operators; the
 *    printed minus on the pair terms is not exact on x*y).
 *  - 3D runs periodic boundaries only (the paper's 3D test has no wall).
 *  - The thresholded set is closed under ancestors (parent group of every kept
 *    group) before the enlargement H_eps, so that H_eps acts on a tree.
 *  - Neighbour addition shifts by eta^h in cells of the kept cell's own level.
 *  - At the finest level (n = J - l = 0) the transport is the plain shift
 *    f(k - eta), which the E/A formula equals in exact arithmetic.
 *  - Collision is written m + S (m_eq - m), equal to (I - S) m + S m_eq.
 *  - D2Q9: diagonal logical velocities are (+-1, +-1) as the rows of M imply;
 *    the equilibrium uses |q|^2 and c_s^4 rho where the printed text is garbled.
 *  - Boundaries (section "Boundary conditions"): an axis is periodic, or has a
 *    wall at both ends. At a wall the prediction, the details and the
 *    reconstruction see each level extended by even reflection across the wall
 *    (the paper does not say how its stencils are completed there; reflection
 *    commutes with the symmetric prediction stencil, so the reconstruction of
 *    a level is that of the mirrored periodic problem). The set operations of
 *    the mesh (neighbour addition, grading box) ignore cells beyond a wall. In
 *    the transport, a finest cell of E beyond a wall takes the side's
 *    condition (copy, bounce back, anti bounce back, eq. refBoundaryConditions)
 *    evaluated either on the leaf itself or on the reconstruction, as eq.
 *    AdvectionOnBoundary allows; a cell beyond two walls (a corner) takes the
 *    condition of the x wall.
 */
#include "mr_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define MAXQ 16

/* Host threads of the parallel loops: sets the count when n > 0; returns the
 * count the next parallel loop uses. */
int orc_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
}

/* ---- Level geometry (section "Nested lattices"): N_l = 2^l cells per axis ---- */

static int side(int l) { return 1 << l; }
static int64_t ncells(const orc_params *P, int l) { return (int64_t)1 << (P->dim * l); }
static int wrapi(int i, int n) { i %= n; return i < 0 ? i + n : i; }

/* Walls: axis a (0 = x, 1 = y) has walls when either of its sides is not
 * periodic (3D: periodic only, refused by bad_bc). */
static int wall_axis(const orc_params *P, int a) { return P->bc[2 * a] != 0 || P->bc[2 * a + 1] != 0; }
static int has_walls(const orc_params *P) { return wall_axis(P, 0) || (P->dim == 2 && wall_axis(P, 1)); }
/* Index i (|overflow| < n) along axis a for the MR operators: periodic wrap, or
 * even reflection across a wall (cell -1 is cell 0, cell n is cell n-1). */
static int mr_axis(const orc_params *P, int a, int i, int n) {
  if (!wall_axis(P, a)) return wrapi(i, n);
  return i < 0 ? -1 - i : i >= n ? 2 * n - 1 - i : i;
}
/* Side of the domain beyond which index (x, y) of level l lies (0 x-, 1 x+,
 * 2 y-, 3 y+; x first), or -1 if inside or only beyond periodic sides. */
static int beyond_wall(const orc_params *P, int l, int x, int y) {
  const int n = 1 << l;
  if (wall_axis(P, 0) && (x < 0 || x >= n)) return x < 0 ? 0 : 1;
  if (P->dim == 2 && wall_axis(P, 1) && (y < 0 || y >= n)) return y < 0 ? 2 : 3;
  return -1;
}

int64_t orc_level_offset(const orc_params *P, int l) {
  int64_t off = 0;
  for (int m = P->jmin; m < l; ++m) off += ncells(P, m);
  return off;
}

int64_t orc_total_cells(const orc_params *P) { return orc_level_offset(P, P->jmax + 1); }

static uint8_t *tree_at(const orc_params *P, const uint8_t *tree, int l) {
  return (uint8_t *)tree + orc_level_offset(P, l);
}
static double *val_at(const orc_params *P, const double *v, int l, int h) {
  return (double *)v + (int64_t)P->q * orc_level_offset(P, l) + (int64_t)h * ncells(P, l);
}
static int64_t cell_index(const orc_params *P, int l, int x, int y, int z) {
  const int64_t n = side(l);
  return P->dim == 1 ? x : P->dim == 2 ? (int64_t)x + n * y : (int64_t)x + n * ((int64_t)y + n * z);
}
static int64_t cell_index_wrapped(const orc_params *P, int l, int x, int y, int z) {
  const int n = side(l);
  return cell_index(P, l, wrapi(x, n), P->dim >= 2 ? wrapi(y, n) : 0, P->dim == 3 ? wrapi(z, n) : 0);
}
/* Cell (x, y) of level l (d <= 2) as the MR operators read it (wrap or reflection). */
static int64_t cell_index_mr(const orc_params *P, int l, int x, int y) {
  int n = side(l);
  return P->dim == 1 ? mr_axis(P, 0, x, n) : (int64_t)mr_axis(P, 0, x, n) + (int64_t)n * mr_axis(P, 1, y, n);
}
/* Cell (x, y, z) of level l for the set operations: wrapped on periodic axes,
 * -1 beyond a wall. */
static int64_t cell_index_set(const orc_params *P, int l, int x, int y, int z) {
  return beyond_wall(P, l, x, y) >= 0 ? -1 : cell_index_wrapped(P, l, x, y, z);
}
static void cell_coords(const orc_params *P, int l, int64_t c, int *x, int *y, int *z) {
  const int64_t n = side(l);
  *x = (int)(c % n);
  *y = P->dim >= 2 ? (int)((c / n) % n) : 0;
  *z = P->dim == 3 ? (int)(c / (n * n)) : 0;
}
static int nchildren(const orc_params *P) { return 1 << P->dim; }
/* Child sigma of (x, y, z): sigma bit 0 is the x offset, bit 1 the y offset,
 * bit 2 the z offset. */
static int64_t child_index(const orc_params *P, int l, int x, int y, int z, int sigma) {
  return cell_index(P, l + 1, 2 * x + (sigma & 1), 2 * y + ((sigma >> 1) & 1), 2 * z + ((sigma >> 2) & 1));
}
static int is_leaf(const orc_params *P, const uint8_t *tree, int l, int64_t c) {
  if (!tree_at(P, tree, l)[c]) return 0;
  if (l == P->jmax) return 1;
  int x, y, z;
  cell_coords(P, l, c, &x, &y, &z);
  return !tree_at(P, tree, l + 1)[child_index(P, l, x, y, z, 0)];
}
static int is_internal(const orc_params *P, const uint8_t *tree, int l, int64_t c) {
  return tree_at(P, tree, l)[c] && !is_leaf(P, tree, l, c);
}

/* ---- Scheme data (section "Collision and transport"; D2Q9 in the von Karman
 *      section, Lallemand-Luo) ---- */

void orc_velocities(const orc_params *P, int *eta) {
  static const int d1q2[2][2] = {{1, 0}, {-1, 0}};
  static const int d1q3[3][2] = {{0, 0}, {1, 0}, {-1, 0}};
  static const int d2q9[9][2] = {{0, 0},  {1, 0},  {0, 1},   {-1, 0}, {0, -1},
                                 {1, 1},  {-1, 1}, {-1, -1}, {1, -1}};
  /* D2Q4: lambda (cos(k pi / 2), sin(k pi / 2)), k = 0..3, for every variable */
  static const int d2q4[4][2] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};
  if (P->scheme == 5) {
    /* D3Q6: lambda cos(pi h) along x (h = 0, 1), y (h = 2, 3), z (h = 4, 5) */
    for (int h = 0; h < 6; ++h) {
      eta[3 * h] = eta[3 * h + 1] = eta[3 * h + 2] = 0;
      eta[3 * h + h / 2] = (h & 1) ? -1 : 1;
    }
    return;
  }
  if (P->scheme == 4) {
    for (int h = 0; h < P->q; ++h) { eta[3 * h] = d2q4[h & 3][0]; eta[3 * h + 1] = d2q4[h & 3][1]; eta[3 * h + 2] = 0; }
    return;
  }
  const int(*t)[2] = P->scheme == 1 ? d1q2 : P->scheme == 2 ? d1q3 : d2q9;
  for (int h = 0; h < P->q; ++h) { eta[3 * h] = t[h][0]; eta[3 * h + 1] = t[h][1]; eta[3 * h + 2] = 0; }
}

void orc_moment_matrix(const orc_params *P, double *M) {
  const double L = P->lambda, L2 = L * L, L3 = L2 * L, L4 = L2 * L2;
  memset(M, 0, sizeof(double) * P->q * P->q);
  if (P->scheme == 1) {
    const double m[2][2] = {{1, 1}, {L, -L}};
    memcpy(M, m, sizeof m);
  } else if (P->scheme == 2) {
    const double m[3][3] = {{1, 1, 1}, {0, L, -L}, {0, L2, L2}};
    memcpy(M, m, sizeof m);
  } else if (P->scheme == 5) {
    /* section "Three dimensional advection equation": the D3Q6 matrix */
    const double m[6][6] = {{1, 1, 1, 1, 1, 1},       {L, -L, 0, 0, 0, 0},     {0, 0, L, -L, 0, 0},
                            {0, 0, 0, 0, L, -L},      {L2, L2, -L2, -L2, 0, 0}, {L2, L2, 0, 0, -L2, -L2}};
    memcpy(M, m, sizeof m);
  } else if (P->scheme == 4) {
    /* section "Systems of hyperbolic conservation laws": the same D2Q4 matrix
     * for each of the four variables (block diagonal) */
    const double m[4][4] = {{1, 1, 1, 1}, {L, 0, -L, 0}, {0, L, 0, -L}, {L2, -L2, L2, -L2}};
    for (int i = 0; i < 4; ++i)
      for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) M[(4 * i + r) * 16 + 4 * i + c] = m[r][c];
  } else {
    const double m[9][9] = {
        {1, 1, 1, 1, 1, 1, 1, 1, 1},
        {0, L, 0, -L, 0, L, -L, -L, L},
        {0, 0, L, 0, -L, L, L, -L, -L},
        {-4 * L2, -L2, -L2, -L2, -L2, 2 * L2, 2 * L2, 2 * L2, 2 * L2},
        {0, -2 * L3, 0, 2 * L3, 0, L3, -L3, -L3, L3},
        {0, 0, -2 * L3, 0, 2 * L3, L3, L3, -L3, -L3},
        {4 * L4, -2 * L4, -2 * L4, -2 * L4, -2 * L4, L4, L4, L4, L4},
        {0, L2, -L2, L2, -L2, 0, 0, 0, 0},
        {0, 0, 0, 0, 0, L2, -L2, L2, -L2}};
    memcpy(M, m, sizeof m);
  }
}

/* Gauss-Jordan elimination with partial pivoting. Returns 0 on success. */
int orc_moment_matrix_inverse(const orc_params *P, double *Minv) {
  const int q = P->q;
  double A[MAXQ][2 * MAXQ];
  double M[MAXQ * MAXQ];
  orc_moment_matrix(P, M);
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < 2 * q; ++j) A[i][j] = j < q ? M[i * q + j] : (j - q == i ? 1.0 : 0.0);
  for (int col = 0; col < q; ++col) {
    int piv = col;
    for (int r = col + 1; r < q; ++r)
      if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
    if (A[piv][col] == 0.0) return -1;
    if (piv != col)
      for (int j = 0; j < 2 * q; ++j) { double t = A[col][j]; A[col][j] = A[piv][j]; A[piv][j] = t; }
    const double d = A[col][col];
    for (int j = 0; j < 2 * q; ++j) A[col][j] /= d;
    for (int r = 0; r < q; ++r) {
      if (r == col || A[r][col] == 0.0) continue;
      const double f = A[r][col];
      for (int j = 0; j < 2 * q; ++j) A[r][j] -= f * A[col][j];
    }
  }
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < q; ++j) Minv[i * q + j] = A[i][q + j];
  return 0;
}

/* Equilibrium moments as functions of the conserved ones. */
void orc_equilibrium(const orc_params *P, const double *m, double *meq) {
  const double L = P->lambda;
  if (P->scheme == 1) {
    meq[0] = m[0];
    meq[1] = P->eq_param * m[0];
  } else if (P->scheme == 2) {
    meq[0] = m[0];
    meq[1] = 0.5 * m[0] * m[0];
    meq[2] = P->eq_param * L * L * m[0];
  } else if (P->scheme == 5) {
    /* D3Q6 advection: m_eq = (u, V_x u, V_y u, V_z u, 0, 0) */
    meq[0] = m[0];
    meq[1] = P->vel[0] * m[0];
    meq[2] = P->vel[1] * m[0];
    meq[3] = P->vel[2] * m[0];
    meq[4] = 0.0;
    meq[5] = 0.0;
  } else if (P->scheme == 4) {
    /* Euler system: conserved u = (rho, rho u, rho v, E), pressure from
     * E = p / (gamma - 1) + rho (u^2 + v^2) / 2; variable i relaxes its first
     * moments towards the fluxes Phi_x,i(u), Phi_y,i(u) and its last one to 0 */
    const double rho = m[0], mx = m[4], my = m[8], E = m[12];
    const double u = mx / rho, v = my / rho;
    const double p = (P->eq_param - 1.0) * (E - 0.5 * rho * (u * u + v * v));
    const double fx[4] = {mx, mx * u + p, mx * v, u * (E + p)};
    const double fy[4] = {my, my * u, my * v + p, v * (E + p)};
    for (int i = 0; i < 4; ++i) {
      meq[4 * i] = m[4 * i];
      meq[4 * i + 1] = fx[i];
      meq[4 * i + 2] = fy[i];
      meq[4 * i + 3] = 0.0;
    }
  } else {
    const double rho = m[0], qx = m[1], qy = m[2];
    const double cs2 = L * L / 3.0;
    const double q2 = qx * qx + qy * qy;
    meq[0] = rho;
    meq[1] = qx;
    meq[2] = qy;
    meq[3] = 3.0 * (-2.0 * cs2 * rho + q2 / rho);
    meq[4] = -3.0 * cs2 * qx;
    meq[5] = -3.0 * cs2 * qy;
    meq[6] = 9.0 * (cs2 * cs2 * rho - cs2 * q2 / rho);
    meq[7] = (qx * qx - qy * qy) / rho;
    meq[8] = qx * qy / rho;
  }
}

/* Collision in moment space (eq. CollisionOnFinest / AdaptiveCollision). */
static void collide_with(const orc_params *P, const double *M, const double *Minv, double *f) {
  const int q = P->q;
  double m[MAXQ] = {0}, meq[MAXQ] = {0};
  for (int i = 0; i < q; ++i) {
    double acc = 0.0;
    for (int j = 0; j < q; ++j) acc += M[i * q + j] * f[j];
    m[i] = acc;
  }
  orc_equilibrium(P, m, meq);
  for (int i = 0; i < q; ++i) m[i] = m[i] + P->s[i] * (meq[i] - m[i]);
  for (int i = 0; i < q; ++i) {
    double acc = 0.0;
    for (int j = 0; j < q; ++j) acc += Minv[i * q + j] * m[j];
    f[i] = acc;
  }
}

void orc_collide_cell(const orc_params *P, double *f) {
  double M[MAXQ * MAXQ], Minv[MAXQ * MAXQ];
  orc_moment_matrix(P, M);
  orc_moment_matrix_inverse(P, Minv);
  collide_with(P, M, Minv, f);
}

/* ---- Multiresolution operators (section "Projection and prediction operators") ---- */

/* Table 1, gamma = 1. */
static const double C1 = -0.125;
/* Table 1: the coefficients c_1 .. c_gamma of the prediction of half-width
 * gamma = 1, 2, 3 (exact dyadic rationals). */
static const double CG[4][3] = {{0, 0, 0}, {-0.125, 0, 0}, {-22.0 / 128, 3.0 / 128, 0},
                                {-201.0 / 1024, 11.0 / 256, -5.0 / 1024}};
static int gam(const orc_params *P) { return P->gamma > 0 ? P->gamma : 1; }

/* Prediction of child (cx, cy, cz) at level l from the dense data Fp of level l-1:
 * 1D:  f_parent + (-1)^dx * Q_x,  Q_x = sum_alpha c_alpha (f_{p+alpha} - f_{p-alpha});
 * 2D:  tensor product, ((f + (-1)^dx Qx) + (-1)^dy Qy) + (-1)^(dx+dy) Qxy;
 * 3D:  the same with the axis terms Qx, Qy, Qz, the pair terms Qxy, Qxz, Qyz and
 *      the triple term Qxyz, added in that order. */
static double predict_at(const orc_params *P, const double *Fp, int l, int cx, int cy, int cz) {
  const int n = side(l - 1), g = gam(P);
  const double *c = CG[g];
  const int px = cx >> 1;
  const double sx = (cx & 1) ? -1.0 : 1.0;
  if (P->dim == 1) {
    /* Q = sum over alpha = 1..gamma of c_alpha (F(p + alpha) - F(p - alpha)), alpha ascending */
    double Q = c[0] * (Fp[mr_axis(P, 0, px + 1, n)] - Fp[mr_axis(P, 0, px - 1, n)]);
    for (int a = 2; a <= g; ++a) Q = Q + c[a - 1] * (Fp[mr_axis(P, 0, px + a, n)] - Fp[mr_axis(P, 0, px - a, n)]);
    return Fp[px] + sx * Q;
  }
  const int py = cy >> 1;
  const double sy = (cy & 1) ? -1.0 : 1.0;
  if (P->dim == 3) {
    const int pz = cz >> 1;
    const double sz = (cz & 1) ? -1.0 : 1.0;
#define A3(a, b, t) Fp[(int64_t)wrapi(px + (a), n) + (int64_t)n * ((int64_t)wrapi(py + (b), n) + (int64_t)n * wrapi(pz + (t), n))]
    /* axis terms, alpha ascending */
    double Qx = c[0] * (A3(1, 0, 0) - A3(-1, 0, 0));
    double Qy = c[0] * (A3(0, 1, 0) - A3(0, -1, 0));
    double Qz = c[0] * (A3(0, 0, 1) - A3(0, 0, -1));
    for (int a = 2; a <= g; ++a) {
      Qx = Qx + c[a - 1] * (A3(a, 0, 0) - A3(-a, 0, 0));
      Qy = Qy + c[a - 1] * (A3(0, a, 0) - A3(0, -a, 0));
      Qz = Qz + c[a - 1] * (A3(0, 0, a) - A3(0, 0, -a));
    }
    /* pair terms in the plane of axes (u, v): the 2D cross term of that plane,
     * beta (v) outer, alpha (u) inner from (1, 1) */
#define PAIR(a, b, U) \
  ((c[(a) - 1] * c[(b) - 1]) * (((U((a), (b)) - U(-(a), (b))) - U((a), -(b))) + U(-(a), -(b))))
#define XY(a, b) A3(a, b, 0)
#define XZ(a, b) A3(a, 0, b)
#define YZ(a, b) A3(0, a, b)
    double Qxy = 0.0, Qxz = 0.0, Qyz = 0.0;
    for (int b = 1; b <= g; ++b)
      for (int a = 1; a <= g; ++a) {
        if (a == 1 && b == 1) {
          Qxy = PAIR(1, 1, XY);
          Qxz = PAIR(1, 1, XZ);
          Qyz = PAIR(1, 1, YZ);
        } else {
          Qxy = Qxy + PAIR(a, b, XY);
          Qxz = Qxz + PAIR(a, b, XZ);
          Qyz = Qyz + PAIR(a, b, YZ);
        }
      }
    /* triple term: tau (z) outer, beta (y), alpha (x) inner, from (1, 1, 1);
     * the eight values with the signs of the product of the three offsets */
    double Qxyz = 0.0;
    for (int t = 1; t <= g; ++t)
      for (int b = 1; b <= g; ++b)
        for (int a = 1; a <= g; ++a) {
          const double v = (((((((A3(a, b, t) - A3(-a, b, t)) - A3(a, -b, t)) - A3(a, b, -t)) + A3(-a, -b, t)) +
                              A3(-a, b, -t)) + A3(a, -b, -t)) - A3(-a, -b, -t));
          const double term = ((c[a - 1] * c[b - 1]) * c[t - 1]) * v;
          Qxyz = (a == 1 && b == 1 && t == 1) ? term : Qxyz + term;
        }
    const double f0 = A3(0, 0, 0);
#undef XY
#undef XZ
#undef YZ
#undef PAIR
#undef A3
    return ((((((f0 + sx * Qx) + sy * Qy) + sz * Qz) + (sx * sy) * Qxy) + (sx * sz) * Qxz) +
            (sy * sz) * Qyz) + ((sx * sy) * sz) * Qxyz;
  }
#define AT(a, b) Fp[(int64_t)mr_axis(P, 0, (a), n) + (int64_t)n * mr_axis(P, 1, (b), n)]
  double Qx = c[0] * (AT(px + 1, py) - AT(px - 1, py));
  double Qy = c[0] * (AT(px, py + 1) - AT(px, py - 1));
  for (int a = 2; a <= g; ++a) {
    Qx = Qx + c[a - 1] * (AT(px + a, py) - AT(px - a, py));
    Qy = Qy + c[a - 1] * (AT(px, py + a) - AT(px, py - a));
  }
  /* tensor-product cross term: beta (y) outer, alpha (x) inner, starting with
   * (1, 1); each product c_alpha c_beta is exact */
#define TERM(a, b) \
  ((c[(a) - 1] * c[(b) - 1]) * (((AT(px + (a), py + (b)) - AT(px - (a), py + (b))) - AT(px + (a), py - (b))) + \
                                AT(px - (a), py - (b))))
  double Qxy = TERM(1, 1);
  for (int b = 1; b <= g; ++b)
    for (int a = (b == 1 ? 2 : 1); a <= g; ++a) Qxy = Qxy + TERM(a, b);
#undef TERM
  return ((AT(px, py) + sx * Qx) + sy * Qy) + (sx * sy) * Qxy;
#undef AT
}

double orc_predict(const orc_params *P, const double *Fp, int l, int cx, int cy) {
  return predict_at(P, Fp, l, cx, cy, 0);
}
double orc_predict3(const orc_params *P, const double *Fp, int l, int cx, int cy, int cz) {
  return predict_at(P, Fp, l, cx, cy, cz);
}

/* Projection: average of the 2^d children of (px, py, pz), children read from
 * the dense data Fc of level l+1 and summed in the order of sigma. */
static double project(const orc_params *P, const double *Fc, int l, int px, int py, int pz) {
  if (P->dim == 1) return 0.5 * (Fc[2 * px] + Fc[2 * px + 1]);
  if (P->dim == 3) {
    double acc = Fc[child_index(P, l, px, py, pz, 0)];
    for (int sigma = 1; sigma < 8; ++sigma) acc = acc + Fc[child_index(P, l, px, py, pz, sigma)];
    return 0.125 * acc;
  }
  const int64_t n = side(l + 1);
  const double a00 = Fc[2 * px + n * (2 * py)];
  const double a10 = Fc[2 * px + 1 + n * (2 * py)];
  const double a01 = Fc[2 * px + n * (2 * py + 1)];
  const double a11 = Fc[2 * px + 1 + n * (2 * py + 1)];
  return 0.25 * (((a00 + a10) + a01) + a11);
}

int orc_reconstruct(const orc_params *P, const uint8_t *tree, double *values) {
  /* Upward: internal tree cells hold the projection of their children. */
  for (int l = P->jmax - 1; l >= P->jmin; --l) {
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < ncells(P, l); ++c) {
      if (!is_internal(P, tree, l, c)) continue;
      int x, y, z;
      cell_coords(P, l, c, &x, &y, &z);
      for (int h = 0; h < P->q; ++h)
        val_at(P, values, l, h)[c] = project(P, val_at(P, values, l + 1, h), l, x, y, z);
    }
  }
  /* Downward: cells outside the tree receive the zero-detail prediction. */
  for (int l = P->jmin + 1; l <= P->jmax; ++l) {
    const uint8_t *t = tree_at(P, tree, l);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < ncells(P, l); ++c) {
      if (t[c]) continue;
      int x, y, z;
      cell_coords(P, l, c, &x, &y, &z);
      for (int h = 0; h < P->q; ++h)
        val_at(P, values, l, h)[c] = predict_at(P, val_at(P, values, l - 1, h), l, x, y, z);
    }
  }
  return 0;
}

/* ---- Details and the sibling l-infinity metric (sections "Details and local
 *      regularity" and "Mesh coarsening") ---- */

int orc_details(const orc_params *P, const uint8_t *tree, const double *values, double *D) {
  const int64_t total = orc_total_cells(P);
  for (int64_t i = 0; i < total; ++i) D[i] = -1.0;
  for (int l = P->jmin + 1; l <= P->jmax; ++l) {
    const uint8_t *tp = tree_at(P, tree, l - 1), *tc = tree_at(P, tree, l);
    double *Dp = D + orc_level_offset(P, l - 1);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < ncells(P, l - 1); ++p) {
      int px, py, pz;
      cell_coords(P, l - 1, p, &px, &py, &pz);
      if (!tp[p] || !tc[child_index(P, l - 1, px, py, pz, 0)]) continue;
      double dmax = 0.0;
      for (int h = 0; h < P->q; ++h) {
        const double *Fc = val_at(P, values, l, h), *Fp = val_at(P, values, l - 1, h);
        double s2 = 0.0;
        for (int sigma = 0; sigma < nchildren(P); ++sigma) {
          const int cx = 2 * px + (sigma & 1), cy = 2 * py + ((sigma >> 1) & 1), cz = 2 * pz + ((sigma >> 2) & 1);
          const double d = Fc[cell_index(P, l, cx, cy, cz)] - predict_at(P, Fp, l, cx, cy, cz);
          if (P->metric) s2 = s2 + d * d;
          else if (fabs(d) > dmax) dmax = fabs(d);
        }
        if (P->metric) {
          s2 = ldexp(s2, -P->dim); /* square of 2^{-d/2} (sum of d^2)^{1/2} */
          if (s2 > dmax) dmax = s2;
        }
      }
      Dp[p] = dmax;
    }
  }
  return 0;
}

/* ---- Time-adaptive mesh: G o H_eps o T_eps (section "Construction of the time
 *      adaptive mesh", eq. Thresholding, eq. AdditionNeigh, refinement rule,
 *      grading definition) ---- */

static void mark_group(const orc_params *P, uint8_t *tl, int l, int gx, int gy, int gz) {
  /* all children at level l of the cell (gx, gy, gz) of level l-1 */
  for (int sigma = 0; sigma < nchildren(P); ++sigma) tl[child_index(P, l - 1, gx, gy, gz, sigma)] = 1;
}

/* Thresholds eps_l = 2^{d(l-J)} eps and 2^{mu_bar + d} eps_l, indexed by level. */
static void thresholds(const orc_params *P, double *eps_l, double *ref_l) {
  for (int l = 0; l <= P->jmax; ++l) {
    eps_l[l] = ldexp(P->eps, P->dim * (l - P->jmax));
    ref_l[l] = ldexp(eps_l[l], P->dim) * exp2(P->mu_bar);
  }
  if (P->metric) /* the l2 metric is kept squared: compare with squared thresholds */
    for (int l = 0; l <= P->jmax; ++l) {
      eps_l[l] = eps_l[l] * eps_l[l];
      ref_l[l] = ref_l[l] * ref_l[l];
    }
}

static int adapt_tree_thr(const orc_params *P, const uint8_t *told, const double *D, const double *eps_lv,
                          const double *ref_lv, uint8_t *tnew);

int orc_adapt_tree(const orc_params *P, const uint8_t *told, const double *D, uint8_t *tnew) {
  double eps_l[64], ref_l[64];
  thresholds(P, eps_l, ref_l);
  return adapt_tree_thr(P, told, D, eps_l, ref_l, tnew);
}

static int adapt_tree_thr(const orc_params *P, const uint8_t *told, const double *D, const double *eps_lv,
                          const double *ref_lv, uint8_t *tnew) {
  const int J = P->jmax, jmin = P->jmin, d = P->dim;
  const int64_t total = orc_total_cells(P);
  int eta[3 * MAXQ];
  orc_velocities(P, eta);
  uint8_t *keep = calloc((size_t)total, 1);
  if (!keep) return -1;

  /* T_eps: level jmin always; deeper cells of the old tree whose sibling-group
   * metric reaches eps_l = 2^{d(l-J)} eps. */
  memset(tree_at(P, keep, jmin), 1, (size_t)ncells(P, jmin));
  for (int l = jmin + 1; l <= J; ++l) {
    const double eps_l = eps_lv[l];
    const uint8_t *t = tree_at(P, told, l);
    const double *Dp = D + orc_level_offset(P, l - 1);
    uint8_t *k = tree_at(P, keep, l);
    for (int64_t c = 0; c < ncells(P, l); ++c) {
      if (!t[c]) continue;
      int x, y, z;
      cell_coords(P, l, c, &x, &y, &z);
      if (Dp[cell_index(P, l - 1, x >> 1, y >> 1, z >> 1)] >= eps_l) k[c] = 1;
    }
  }
  /* Ancestor closure: a kept group keeps the group of its parent. */
  for (int l = J; l >= jmin + 2; --l) {
    const uint8_t *k = tree_at(P, keep, l);
    uint8_t *kp = tree_at(P, keep, l - 1);
    for (int64_t c = 0; c < ncells(P, l); ++c) {
      if (!k[c]) continue;
      int x, y, z;
      cell_coords(P, l, c, &x, &y, &z);
      mark_group(P, kp, l - 1, x >> 2, y >> 2, z >> 2);
    }
  }
  /* H_eps: neighbours along every velocity, and children of groups whose metric
   * reaches 2^{mu_bar + d} eps_l. */
  memset(tnew, 0, (size_t)total);
  for (int l = jmin; l <= J; ++l) {
    const uint8_t *k = tree_at(P, keep, l);
    uint8_t *tn = tree_at(P, tnew, l);
    const double refine_thr = ref_lv[l];
    for (int64_t c = 0; c < ncells(P, l); ++c) {
      if (!k[c]) continue;
      int x, y, z;
      cell_coords(P, l, c, &x, &y, &z);
      tn[c] = 1;
      for (int h = 0; h < P->q; ++h) {
        const int64_t nb = cell_index_set(P, l, x - eta[3 * h], y - eta[3 * h + 1], z - eta[3 * h + 2]);
        if (nb >= 0) tn[nb] = 1;
      }
      if (l > jmin && l < J) {
        const double Dg = D[orc_level_offset(P, l - 1) + cell_index(P, l - 1, x >> 1, y >> 1, z >> 1)];
        if (Dg >= refine_thr) mark_group(P, tree_at(P, tnew, l + 1), l + 1, x, y, z);
      }
    }
  }
  /* G: minimal graded complete tree, swept from the finest level down. */
  for (int l = J; l >= jmin + 1; --l) {
    uint8_t *tn = tree_at(P, tnew, l), *tp = tree_at(P, tnew, l - 1);
    for (int64_t c = 0; c < ncells(P, l); ++c) {
      if (!tn[c]) continue;
      int x, y, z;
      cell_coords(P, l, c, &x, &y, &z);
      mark_group(P, tn, l, x >> 1, y >> 1, z >> 1);
    }
    const int g = gam(P), gy = d >= 2 ? g : 0, gz = d == 3 ? g : 0;
    for (int64_t c = 0; c < ncells(P, l); ++c) {
      if (!tn[c]) continue;
      int x, y, z;
      cell_coords(P, l, c, &x, &y, &z);
      const int px = x >> 1, py = y >> 1, pz = z >> 1;
      for (int az = -gz; az <= gz; ++az)
        for (int ay = -gy; ay <= gy; ++ay)
          for (int ax = -g; ax <= g; ++ax) {
            const int64_t nb = cell_index_set(P, l - 1, px + ax, py + ay, pz + az);
            if (nb >= 0) tp[nb] = 1;
          }
    }
  }
  memset(tree_at(P, tnew, jmin), 1, (size_t)ncells(P, jmin));
  free(keep);
  return 0;
}

/* ---- Data transfer to the new mesh ---- */

int orc_transfer(const orc_params *P, const uint8_t *told, const double *vold, const uint8_t *tnew,
                 double *vnew) {
  (void)told; /* the dense reconstruction already holds copy, projection and prediction values */
  for (int l = P->jmin; l <= P->jmax; ++l)
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < ncells(P, l); ++c) {
      if (!is_leaf(P, tnew, l, c)) continue;
      for (int h = 0; h < P->q; ++h) val_at(P, vnew, l, h)[c] = val_at(P, vold, l, h)[c];
    }
  return 0;
}

/* ---- MR transport (eq. AdaptiveAdvectionPhase with the sets E and A built
 *      from the cell splitting B, eq. CellSplitting) ---- */

/* Index of the velocity opposite to h (eta^{h+} = -eta^h). */
static int opposite(const orc_params *P, const int *eta, int h) {
  for (int k = 0; k < P->q; ++k)
    if (eta[3 * k] == -eta[3 * h] && eta[3 * k + 1] == -eta[3 * h + 1] && eta[3 * k + 2] == -eta[3 * h + 2]) return k;
  return h;
}

/* Boundary sides valid: each 0..3; an axis periodic on both sides or walled on
 * both; 1D has no y sides; 3D is periodic; the reconstruction evaluation flag
 * is 0 or 1. */
static int bad_bc(const orc_params *P) {
  for (int k = 0; k < 4; ++k)
    if (P->bc[k] < 0 || P->bc[k] > 3) return 1;
  for (int a = 0; a < 2; ++a)
    if ((P->bc[2 * a] == 0) != (P->bc[2 * a + 1] == 0)) return 1;
  if (P->dim == 1 && (P->bc[2] || P->bc[3])) return 1;
  if (P->dim == 3 && (P->bc[0] || P->bc[1] || P->bc[2] || P->bc[3])) return 1;
  return P->bc_eval != 0 && P->bc_eval != 1;
}

/* Population h entering the domain from the finest cell beyond wall `side`
 * whose image under eta^h is the finest cell (ix, iy) of the leaf (l, c), eq.
 * AdvectionOnBoundary with eq. refBoundaryConditions: the side's condition on
 * population h (copy) or on its opposite hd (bounce back; anti bounce back with
 * the sign changed), evaluated on the leaf (bc_eval 0) or on the
 * reconstruction at (ix, iy) (bc_eval 1). */
static double wall_value(const orc_params *P, const double *vs, int side, int h, int hd, int l, int64_t c, int ix,
                         int iy) {
  const int kind = P->bc[side];
  const int g = kind == 1 ? h : hd;
  const double v = P->bc_eval ? val_at(P, vs, P->jmax, g)[cell_index(P, P->jmax, ix, iy, 0)] : val_at(P, vs, l, g)[c];
  return kind == 3 ? -v : v;
}

int orc_transport(const orc_params *P, const uint8_t *tree, const double *vs, double *out,
                  int definition_form) {
  const int J = P->jmax, d = P->dim;
  int eta[3 * MAXQ];
  orc_velocities(P, eta);
  if (bad_bc(P)) return -1;
  for (int l = P->jmin; l <= J; ++l) {
    const int n = J - l, w = 1 << n, wy = d >= 2 ? w : 1, wz = d == 3 ? w : 1;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t c = 0; c < ncells(P, l); ++c) {
      if (!is_leaf(P, tree, l, c)) continue;
      int x, y, z;
      cell_coords(P, l, c, &x, &y, &z);
      /* B = [bx0, bx0+w) x [by0, by0+wy) x [bz0, bz0+wz) */
      const int bx0 = x * w, by0 = y * wy, bz0 = z * wz;
#define IN_B(a, b, t) ((a) >= bx0 && (a) < bx0 + w && (b) >= by0 && (b) < by0 + wy && (t) >= bz0 && (t) < bz0 + wz)
      for (int h = 0; h < P->q; ++h) {
        const int ex = eta[3 * h], ey = eta[3 * h + 1], ez = eta[3 * h + 2], hd = opposite(P, eta, h);
        const double *FJ = val_at(P, vs, J, h);
        const double fl = val_at(P, vs, l, h)[c];
        double res;
        if (ex == 0 && ey == 0 && ez == 0) {
          res = fl;
        } else if (n == 0) {
          const int sd = beyond_wall(P, J, x - ex, y - ey);
          res = sd >= 0 ? wall_value(P, vs, sd, h, hd, l, c, x, y)
                        : FJ[cell_index_wrapped(P, J, x - ex, y - ey, z - ez)];
        } else if (definition_form) {
          double s = 0.0;
          for (int kz = bz0; kz < bz0 + wz; ++kz)
            for (int ky = by0; ky < by0 + wy; ++ky)
              for (int kx = bx0; kx < bx0 + w; ++kx) {
                const int sd = beyond_wall(P, J, kx - ex, ky - ey);
                s += sd >= 0 ? wall_value(P, vs, sd, h, hd, l, c, kx, ky)
                             : FJ[cell_index_wrapped(P, J, kx - ex, ky - ey, kz - ez)];
              }
          res = ldexp(s, -d * n);
        } else {
          double sE = 0.0, sA = 0.0;
          for (int kz = bz0; kz < bz0 + wz; ++kz)
            for (int ky = by0; ky < by0 + wy; ++ky)
              for (int kx = bx0; kx < bx0 + w; ++kx) {
                /* E = (B - eta) \ B: the cell k - eta, if it left B (beyond a wall: the condition) */
                const int jx = kx - ex, jy = ky - ey, jz = kz - ez;
                if (!IN_B(jx, jy, jz)) {
                  const int sd = beyond_wall(P, J, jx, jy);
                  sE += sd >= 0 ? wall_value(P, vs, sd, h, hd, l, c, kx, ky) : FJ[cell_index_wrapped(P, J, jx, jy, jz)];
                }
              }
          for (int kz = bz0; kz < bz0 + wz; ++kz)
            for (int ky = by0; ky < by0 + wy; ++ky)
              for (int kx = bx0; kx < bx0 + w; ++kx) {
                /* A = B \ (B - eta): the cell k whose image k + eta left B */
                if (!IN_B(kx + ex, ky + ey, kz + ez)) sA += FJ[cell_index(P, J, kx, ky, kz)];
              }
          res = fl + ldexp(sE - sA, -d * n);
        }
        val_at(P, out, l, h)[c] = res;
      }
#undef IN_B
    }
  }
  return 0;
}

int orc_collide(const orc_params *P, const uint8_t *tree, double *values) {
  double M[MAXQ * MAXQ], Minv[MAXQ * MAXQ];
  orc_moment_matrix(P, M);
  if (orc_moment_matrix_inverse(P, Minv)) return -1;
  for (int l = P->jmin; l <= P->jmax; ++l)
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < ncells(P, l); ++c) {
      double f[MAXQ];
      if (!is_leaf(P, tree, l, c)) continue;
      for (int h = 0; h < P->q; ++h) f[h] = val_at(P, values, l, h)[c];
      collide_with(P, M, Minv, f);
      for (int h = 0; h < P->q; ++h) val_at(P, values, l, h)[c] = f[h];
    }
  return 0;
}

/* ---- Algorithm 1 (Overall solver) ---- */

int orc_init(const orc_params *P, const double *m0, uint8_t *tree, double *values) {
  const int J = P->jmax, q = P->q;
  const int nc = P->scheme == 3 ? 3 : P->scheme == 4 ? 4 : 1;
  const int stride = P->scheme == 4 ? 4 : 1; /* moment index of conserved variable k: stride * k */
  const int64_t NJ = ncells(P, J);
  double Minv[MAXQ * MAXQ], m[MAXQ], meq[MAXQ];
  if (orc_moment_matrix_inverse(P, Minv)) return -1;
  memset(tree, 1, (size_t)orc_total_cells(P));
  memset(values, 0, sizeof(double) * (size_t)(q * orc_total_cells(P)));
  for (int64_t c = 0; c < NJ; ++c) {
    for (int i = 0; i < q; ++i) m[i] = 0.0;
    for (int k = 0; k < nc; ++k) m[stride * k] = m0[(int64_t)k * NJ + c];
    orc_equilibrium(P, m, meq);
    for (int i = 0; i < q; ++i) {
      double acc = 0.0;
      for (int j = 0; j < q; ++j) acc += Minv[i * q + j] * meq[j];
      val_at(P, values, J, i)[c] = acc;
    }
  }
  return 0;
}

int orc_step(const orc_params *P, uint8_t *tree, double *values) {
  if (bad_bc(P)) return -1;
  const int64_t total = orc_total_cells(P);
  double *D = malloc(sizeof(double) * (size_t)total);
  double *vnew = calloc((size_t)(P->q * total), sizeof(double));
  uint8_t *tnew = malloc((size_t)total);
  int rc = -1;
  if (!D || !vnew || !tnew) goto done;
  /* mesh adaptation with details of the old solution */
  orc_reconstruct(P, tree, values);
  orc_details(P, tree, values, D);
  orc_adapt_tree(P, tree, D, tnew);
  /* data transfer to the new leaves */
  orc_transfer(P, tree, values, tnew, vnew);
  /* transport on the new leaves from the reconstruction of the transferred data */
  orc_reconstruct(P, tnew, vnew);
  orc_transport(P, tnew, vnew, values, 0);
  /* collision on the new leaves */
  orc_collide(P, tnew, values);
  memcpy(tree, tnew, (size_t)total);
  rc = 0;
done:
  free(D);
  free(vnew);
  free(tnew);
  return rc;
}

int orc_uniform_step(const orc_params *P, double *fJ) {
  const int J = P->jmax, q = P->q;
  const int64_t NJ = ncells(P, J);
  int eta[3 * MAXQ];
  double M[MAXQ * MAXQ], Minv[MAXQ * MAXQ], f[MAXQ];
  orc_velocities(P, eta);
  orc_moment_matrix(P, M);
  if (orc_moment_matrix_inverse(P, Minv)) return -1;
  if (bad_bc(P)) return -1;
  double *g = malloc(sizeof(double) * (size_t)(q * NJ));
  if (!g) return -1;
  for (int h = 0; h < q; ++h)
    for (int64_t c = 0; c < NJ; ++c) {
      int x, y, z;
      cell_coords(P, J, c, &x, &y, &z);
      const int sd = beyond_wall(P, J, x - eta[3 * h], y - eta[3 * h + 1]);
      if (sd < 0) {
        g[h * NJ + c] = fJ[h * NJ + cell_index_wrapped(P, J, x - eta[3 * h], y - eta[3 * h + 1], z - eta[3 * h + 2])];
      } else {  /* the boundary cell's own value of h (copy) or of its opposite */
        const int kind = P->bc[sd], src = kind == 1 ? h : opposite(P, eta, h);
        g[h * NJ + c] = kind == 3 ? -fJ[src * NJ + c] : fJ[src * NJ + c];
      }
    }
  for (int64_t c = 0; c < NJ; ++c) {
    for (int h = 0; h < q; ++h) f[h] = g[h * NJ + c];
    collide_with(P, M, Minv, f);
    for (int h = 0; h < q; ++h) fJ[h * NJ + c] = f[h];
  }
  free(g);
  return 0;
}

/* ---- Diagnostics ---- */

int orc_leaf_counts(const orc_params *P, const uint8_t *tree, int64_t *counts) {
  for (int l = 0; l <= P->jmax; ++l) counts[l] = 0;
  for (int l = P->jmin; l <= P->jmax; ++l)
    for (int64_t c = 0; c < ncells(P, l); ++c) counts[l] += is_leaf(P, tree, l, c);
  return 0;
}

double orc_mass(const orc_params *P, const uint8_t *tree, const double *values) {
  double mass = 0.0;
  for (int l = P->jmin; l <= P->jmax; ++l) {
    const double vol = ldexp(1.0, P->dim * (P->jmax - l)); /* in finest-cell volumes */
    for (int64_t c = 0; c < ncells(P, l); ++c) {
      if (!is_leaf(P, tree, l, c)) continue;
      for (int h = 0; h < P->q; ++h) mass += vol * val_at(P, values, l, h)[c];
    }
  }
  return mass;
}

/* Bit 1: level jmin incomplete; bit 2: a sibling group incomplete; bit 4: a
 * cell without its parent; bit 8: a prediction stencil outside the tree. */
int orc_check_tree(const orc_params *P, const uint8_t *tree) {
  int bad = 0;
  const int d = P->dim;
  const uint8_t *t0 = tree_at(P, tree, P->jmin);
  for (int64_t c = 0; c < ncells(P, P->jmin); ++c)
    if (!t0[c]) bad |= 1;
  for (int l = P->jmin + 1; l <= P->jmax; ++l) {
    const uint8_t *t = tree_at(P, tree, l), *tp = tree_at(P, tree, l - 1);
    for (int64_t p = 0; p < ncells(P, l - 1); ++p) {
      int px, py, pz, cnt = 0;
      cell_coords(P, l - 1, p, &px, &py, &pz);
      for (int sigma = 0; sigma < nchildren(P); ++sigma) cnt += t[child_index(P, l - 1, px, py, pz, sigma)];
      if (cnt != 0 && cnt != nchildren(P)) bad |= 2;
      if (cnt && !tp[p]) bad |= 4;
      const int g = gam(P), gy = d >= 2 ? g : 0, gz = d == 3 ? g : 0;
      if (cnt)
        for (int az = -gz; az <= gz; ++az)
          for (int ay = -gy; ay <= gy; ++ay)
            for (int ax = -g; ax <= g; ++ax) {
              const int64_t nb = cell_index_set(P, l - 1, px + ax, py + ay, pz + az);
              if (nb >= 0 && !tp[nb]) bad |= 8;
            }
    }
  }
  return bad;
}

/* ---- The mesh decision in single precision (for a single-precision solver):
 *      the same projection, prediction and detail expressions evaluated in float,
 *      thresholds rounded to float. ---- */

static float *valf_at(const orc_params *P, const float *v, int l, int h) {
  return (float *)v + (int64_t)P->q * orc_level_offset(P, l) + (int64_t)h * ncells(P, l);
}

static float predict_f32(const orc_params *P, const float *Fp, int l, int cx, int cy, int cz) {
  const int n = side(l - 1), g = gam(P);
  float c[3];
  for (int a = 0; a < 3; ++a) c[a] = (float)CG[g][a]; /* exact in float */
  const int px = cx >> 1;
  const float sx = (cx & 1) ? -1.0f : 1.0f;
  if (P->dim == 1) {
    float Q = c[0] * (Fp[mr_axis(P, 0, px + 1, n)] - Fp[mr_axis(P, 0, px - 1, n)]);
    for (int a = 2; a <= g; ++a) Q = Q + c[a - 1] * (Fp[mr_axis(P, 0, px + a, n)] - Fp[mr_axis(P, 0, px - a, n)]);
    return Fp[px] + sx * Q;
  }
  const int py = cy >> 1;
  const float sy = (cy & 1) ? -1.0f : 1.0f;
  if (P->dim == 3) { /* predict_at's 3D expression, in float */
    const int pz = cz >> 1;
    const float sz = (cz & 1) ? -1.0f : 1.0f;
#define A3(a, b, t) Fp[(int64_t)wrapi(px + (a), n) + (int64_t)n * ((int64_t)wrapi(py + (b), n) + (int64_t)n * wrapi(pz + (t), n))]
    float Qx = c[0] * (A3(1, 0, 0) - A3(-1, 0, 0));
    float Qy = c[0] * (A3(0, 1, 0) - A3(0, -1, 0));
    float Qz = c[0] * (A3(0, 0, 1) - A3(0, 0, -1));
    for (int a = 2; a <= g; ++a) {
      Qx = Qx + c[a - 1] * (A3(a, 0, 0) - A3(-a, 0, 0));
      Qy = Qy + c[a - 1] * (A3(0, a, 0) - A3(0, -a, 0));
      Qz = Qz + c[a - 1] * (A3(0, 0, a) - A3(0, 0, -a));
    }
#define PAIR(a, b, U) \
  ((c[(a) - 1] * c[(b) - 1]) * (((U((a), (b)) - U(-(a), (b))) - U((a), -(b))) + U(-(a), -(b))))
#define XY(a, b) A3(a, b, 0)
#define XZ(a, b) A3(a, 0, b)
#define YZ(a, b) A3(0, a, b)
    float Qxy = 0.0f, Qxz = 0.0f, Qyz = 0.0f;
    for (int b = 1; b <= g; ++b)
      for (int a = 1; a <= g; ++a) {
        if (a == 1 && b == 1) {
          Qxy = PAIR(1, 1, XY);
          Qxz = PAIR(1, 1, XZ);
          Qyz = PAIR(1, 1, YZ);
        } else {
          Qxy = Qxy + PAIR(a, b, XY);
          Qxz = Qxz + PAIR(a, b, XZ);
          Qyz = Qyz + PAIR(a, b, YZ);
        }
      }
    float Qxyz = 0.0f;
    for (int t = 1; t <= g; ++t)
      for (int b = 1; b <= g; ++b)
        for (int a = 1; a <= g; ++a) {
          const float v = (((((((A3(a, b, t) - A3(-a, b, t)) - A3(a, -b, t)) - A3(a, b, -t)) + A3(-a, -b, t)) +
                             A3(-a, b, -t)) + A3(a, -b, -t)) - A3(-a, -b, -t));
          const float term = ((c[a - 1] * c[b - 1]) * c[t - 1]) * v;
          Qxyz = (a == 1 && b == 1 && t == 1) ? term : Qxyz + term;
        }
    const float f0 = A3(0, 0, 0);
#undef XY
#undef XZ
#undef YZ
#undef PAIR
#undef A3
    return ((((((f0 + sx * Qx) + sy * Qy) + sz * Qz) + (sx * sy) * Qxy) + (sx * sz) * Qxz) + (sy * sz) * Qyz) +
           ((sx * sy) * sz) * Qxyz;
  }
#define AT(a, b) Fp[(int64_t)mr_axis(P, 0, (a), n) + (int64_t)n * mr_axis(P, 1, (b), n)]
  float Qx = c[0] * (AT(px + 1, py) - AT(px - 1, py));
  float Qy = c[0] * (AT(px, py + 1) - AT(px, py - 1));
  for (int a = 2; a <= g; ++a) {
    Qx = Qx + c[a - 1] * (AT(px + a, py) - AT(px - a, py));
    Qy = Qy + c[a - 1] * (AT(px, py + a) - AT(px, py - a));
  }
#define TERM(a, b) \
  ((c[(a) - 1] * c[(b) - 1]) * (((AT(px + (a), py + (b)) - AT(px - (a), py + (b))) - AT(px + (a), py - (b))) + \
                                AT(px - (a), py - (b))))
  float Qxy = TERM(1, 1);
  for (int b = 1; b <= g; ++b)
    for (int a = (b == 1 ? 2 : 1); a <= g; ++a) Qxy = Qxy + TERM(a, b);
#undef TERM
  return ((AT(px, py) + sx * Qx) + sy * Qy) + (sx * sy) * Qxy;
#undef AT
}

static float project_f32(const orc_params *P, const float *Fc, int l, int px, int py, int pz) {
  if (P->dim == 1) return 0.5f * (Fc[2 * px] + Fc[2 * px + 1]);
  if (P->dim == 3) {
    float acc = Fc[child_index(P, l, px, py, pz, 0)];
    for (int sigma = 1; sigma < 8; ++sigma) acc = acc + Fc[child_index(P, l, px, py, pz, sigma)];
    return 0.125f * acc;
  }
  const int64_t n = side(l + 1);
  const float a00 = Fc[2 * px + n * (2 * py)], a10 = Fc[2 * px + 1 + n * (2 * py)];
  const float a01 = Fc[2 * px + n * (2 * py + 1)], a11 = Fc[2 * px + 1 + n * (2 * py + 1)];
  return 0.25f * (((a00 + a10) + a01) + a11);
}

int orc_new_tree_f32(const orc_params *P, const uint8_t *tree, const float *leaf_values, uint8_t *tnew,
                     double *D_out) {
  const int64_t total = orc_total_cells(P);
  float *v = malloc(sizeof(float) * (size_t)(P->q * total));
  double *D = D_out ? D_out : malloc(sizeof(double) * (size_t)total);
  if (!v || !D) { free(v); if (!D_out) free(D); return -1; }
  memcpy(v, leaf_values, sizeof(float) * (size_t)(P->q * total));
  for (int l = P->jmax - 1; l >= P->jmin; --l)
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < ncells(P, l); ++c) {
      if (!is_internal(P, tree, l, c)) continue;
      int x, y, z;
      cell_coords(P, l, c, &x, &y, &z);
      for (int h = 0; h < P->q; ++h) valf_at(P, v, l, h)[c] = project_f32(P, valf_at(P, v, l + 1, h), l, x, y, z);
    }
  for (int l = P->jmin + 1; l <= P->jmax; ++l)
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < ncells(P, l); ++c) {
      if (tree_at(P, tree, l)[c]) continue;
      int x, y, z;
      cell_coords(P, l, c, &x, &y, &z);
      for (int h = 0; h < P->q; ++h) valf_at(P, v, l, h)[c] = predict_f32(P, valf_at(P, v, l - 1, h), l, x, y, z);
    }
  for (int64_t i = 0; i < total; ++i) D[i] = -1.0;
  for (int l = P->jmin + 1; l <= P->jmax; ++l) {
    const uint8_t *tp = tree_at(P, tree, l - 1), *tc = tree_at(P, tree, l);
    double *Dp = D + orc_level_offset(P, l - 1);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < ncells(P, l - 1); ++p) {
      int px, py, pz;
      cell_coords(P, l - 1, p, &px, &py, &pz);
      if (!tp[p] || !tc[child_index(P, l - 1, px, py, pz, 0)]) continue;
      float dmax = 0.0f;
      for (int h = 0; h < P->q; ++h) {
        float s2 = 0.0f;
        for (int sigma = 0; sigma < nchildren(P); ++sigma) {
          const int cx = 2 * px + (sigma & 1), cy = 2 * py + ((sigma >> 1) & 1), cz = 2 * pz + ((sigma >> 2) & 1);
          const float dd = valf_at(P, v, l, h)[cell_index(P, l, cx, cy, cz)] -
                           predict_f32(P, valf_at(P, v, l - 1, h), l, cx, cy, cz);
          if (P->metric) s2 = s2 + dd * dd;
          else if (fabsf(dd) > dmax) dmax = fabsf(dd);
        }
        if (P->metric) {
          s2 = ldexpf(s2, -P->dim);
          if (s2 > dmax) dmax = s2;
        }
      }
      Dp[p] = (double)dmax;
    }
  }
  double eps_l[64], ref_l[64];
  thresholds(P, eps_l, ref_l);
  for (int l = 0; l <= P->jmax; ++l) {
    eps_l[l] = (double)(float)eps_l[l];
    ref_l[l] = (double)(float)ref_l[l];
  }
  const int rc = adapt_tree_thr(P, tree, D, eps_l, ref_l, tnew);
  free(v);
  if (!D_out) free(D);
  return rc;
}

/* One step of Algorithm 1 on a given new mesh (the adaptation is replaced by
 * `tnew`, which must be a graded complete tree whose cells all have their
 * parent in `tree`): transfer, transport, collide. */
int orc_step_frozen(const orc_params *P, uint8_t *tree, const uint8_t *tnew, double *values) {
  if (bad_bc(P)) return -1;
  const int64_t total = orc_total_cells(P);
  double *vnew = calloc((size_t)(P->q * total), sizeof(double));
  if (!vnew) return -1;
  orc_reconstruct(P, tree, values);
  orc_transfer(P, tree, values, tnew, vnew);
  orc_reconstruct(P, tnew, vnew);
  orc_transport(P, tnew, vnew, values, 0);
  orc_collide(P, tnew, values);
  memcpy(tree, tnew, (size_t)total);
  free(vnew);
  return 0;
}

/* ---- Adjoint on frozen meshes: transposes of the linear maps of one step and
 *      of the linearised collision. Each scatter-adds into its output in a fixed
 *      loop order. ---- */

/* Stencil of the prediction of child (cx, cy) at level l: the parent-level cells
 * (indices into level l-1) and weights such that the prediction equals
 * sum_k w[k] F[idx[k]]. Returns the number of terms (3 in 1D, 9 in 2D). */
int orc_predict_stencil(const orc_params *P, int l, int cx, int cy, int64_t *idx, double *w) {
  if (has_walls(P) || P->scheme >= 4 || gam(P) > 1) return -1;
  const int n = side(l - 1);
  const int px = cx >> 1;
  const double sx = (cx & 1) ? -1.0 : 1.0;
  if (P->dim == 1) {
    idx[0] = px; w[0] = 1.0;
    idx[1] = wrapi(px + 1, n); w[1] = sx * C1;
    idx[2] = wrapi(px - 1, n); w[2] = -sx * C1;
    return 3;
  }
  const int py = cy >> 1;
  const double sy = (cy & 1) ? -1.0 : 1.0, c2 = sx * sy * C1 * C1;
  int k = 0;
#define PUT(a, b, ww) do { idx[k] = cell_index_wrapped(P, l - 1, (a), (b), 0); w[k] = (ww); ++k; } while (0)
  PUT(px, py, 1.0);
  PUT(px + 1, py, sx * C1);
  PUT(px - 1, py, -sx * C1);
  PUT(px, py + 1, sy * C1);
  PUT(px, py - 1, -sy * C1);
  PUT(px + 1, py + 1, c2);
  PUT(px - 1, py + 1, -c2);
  PUT(px + 1, py - 1, -c2);
  PUT(px - 1, py - 1, c2);
#undef PUT
  return k;
}

/* Transpose of orc_reconstruct: `g` holds a dense adjoint (any cell); on return
 * the leaf entries hold the adjoint of the leaf values and all others are 0. */
int orc_reconstruct_T(const orc_params *P, const uint8_t *tree, double *g) {
  if (has_walls(P) || P->scheme >= 4 || gam(P) > 1) return -1;
  const double inv = 1.0 / nchildren(P);
  /* Each population is its own linear map: the populations run in parallel,
   * each with the loop order below. */
#pragma omp parallel for schedule(static, 1)
  for (int h = 0; h < P->q; ++h) {
    int64_t idx[9];
    double w[9];
    for (int l = P->jmax; l >= P->jmin + 1; --l) { /* predictions, finest first */
      const uint8_t *t = tree_at(P, tree, l);
      double *gl = val_at(P, g, l, h), *gp = val_at(P, g, l - 1, h);
      for (int64_t c = 0; c < ncells(P, l); ++c) {
        if (t[c]) continue;
        int x, y, z;
        cell_coords(P, l, c, &x, &y, &z);
        const int nk = orc_predict_stencil(P, l, x, y, idx, w);
        for (int k = 0; k < nk; ++k) gp[idx[k]] += w[k] * gl[c];
        gl[c] = 0.0;
      }
    }
    for (int l = P->jmin; l <= P->jmax - 1; ++l) { /* projections, coarsest first */
      double *gl = val_at(P, g, l, h), *gc = val_at(P, g, l + 1, h);
      for (int64_t c = 0; c < ncells(P, l); ++c) {
        if (!is_internal(P, tree, l, c)) continue;
        int x, y, z;
        cell_coords(P, l, c, &x, &y, &z);
        for (int sigma = 0; sigma < nchildren(P); ++sigma) gc[child_index(P, l, x, y, z, sigma)] += inv * gl[c];
        gl[c] = 0.0;
      }
    }
  }
  return 0;
}

/* Transpose of orc_transport (E/A form): adds into the dense `gs` the adjoint of
 * the reconstruction F* from the leaf adjoints `ob` of the transported values. */
int orc_transport_T(const orc_params *P, const uint8_t *tree, const double *ob, double *gs) {
  if (has_walls(P) || P->scheme >= 4 || gam(P) > 1) return -1;
  const int J = P->jmax, d = P->dim;
  int eta[3 * MAXQ];
  orc_velocities(P, eta);
  /* populations in parallel, each with the loop order below */
#pragma omp parallel for schedule(static, 1)
  for (int h = 0; h < P->q; ++h) {
    const int ex = eta[3 * h], ey = eta[3 * h + 1];
    double *GJ = val_at(P, gs, J, h);
    for (int l = P->jmin; l <= J; ++l) {
      const int n = J - l, w = 1 << n, wy = d == 2 ? w : 1;
      for (int64_t c = 0; c < ncells(P, l); ++c) {
        if (!is_leaf(P, tree, l, c)) continue;
        int x, y, z;
        cell_coords(P, l, c, &x, &y, &z);
        const int bx0 = x * w, by0 = y * wy;
        const double a = val_at(P, ob, l, h)[c];
        if (ex == 0 && ey == 0) {
          val_at(P, gs, l, h)[c] += a;
        } else if (n == 0) {
          GJ[cell_index_wrapped(P, J, x - ex, y - ey, 0)] += a;
        } else {
          val_at(P, gs, l, h)[c] += a;
          const double sa = ldexp(a, -d * n);
          for (int ky = by0; ky < by0 + wy; ++ky)
            for (int kx = bx0; kx < bx0 + w; ++kx) {
              const int jx = kx - ex, jy = ky - ey;
              if (!(jx >= bx0 && jx < bx0 + w && jy >= by0 && jy < by0 + wy))
                GJ[cell_index_wrapped(P, J, jx, jy, 0)] += sa;
              const int ix = kx + ex, iy = ky + ey;
              if (!(ix >= bx0 && ix < bx0 + w && iy >= by0 && iy < by0 + wy)) GJ[cell_index(P, J, kx, ky, 0)] -= sa;
            }
        }
      }
    }
  }
  return 0;
}

/* Transpose of orc_transfer: the new leaf value is the old dense reconstruction
 * at the same cell, so its adjoint adds there. */
int orc_transfer_T(const orc_params *P, const uint8_t *tnew, const double *gnew, double *gold) {
  for (int l = P->jmin; l <= P->jmax; ++l)
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < ncells(P, l); ++c) {
      if (!is_leaf(P, tnew, l, c)) continue;
      for (int h = 0; h < P->q; ++h) val_at(P, gold, l, h)[c] += val_at(P, gnew, l, h)[c];
    }
  return 0;
}

/* Jacobian d m_eq / d m (q x q, row-major); only the conserved columns are non-zero. */
void orc_equilibrium_jacobian(const orc_params *P, const double *m, double *Je) {
  const int q = P->q;
  const double L = P->lambda;
  memset(Je, 0, sizeof(double) * q * q);
  if (P->scheme >= 4) return; /* the adjoint covers schemes 1..3 (its entry points refuse the others) */
  if (P->scheme == 1) {
    Je[0] = 1.0;
    Je[1 * q + 0] = P->eq_param;
  } else if (P->scheme == 2) {
    Je[0] = 1.0;
    Je[1 * q + 0] = m[0];
    Je[2 * q + 0] = P->eq_param * L * L;
  } else {
    const double rho = m[0], qx = m[1], qy = m[2], cs2 = L * L / 3.0;
    const double q2 = qx * qx + qy * qy, r2 = rho * rho;
    Je[0 * q + 0] = 1.0;
    Je[1 * q + 1] = 1.0;
    Je[2 * q + 2] = 1.0;
    Je[3 * q + 0] = 3.0 * (-2.0 * cs2 - q2 / r2);
    Je[3 * q + 1] = 6.0 * qx / rho;
    Je[3 * q + 2] = 6.0 * qy / rho;
    Je[4 * q + 1] = -3.0 * cs2;
    Je[5 * q + 2] = -3.0 * cs2;
    Je[6 * q + 0] = 9.0 * (cs2 * cs2 + cs2 * q2 / r2);
    Je[6 * q + 1] = -18.0 * cs2 * qx / rho;
    Je[6 * q + 2] = -18.0 * cs2 * qy / rho;
    Je[7 * q + 0] = -(qx * qx - qy * qy) / r2;
    Je[7 * q + 1] = 2.0 * qx / rho;
    Je[7 * q + 2] = -2.0 * qy / rho;
    Je[8 * q + 0] = -qx * qy / r2;
    Je[8 * q + 1] = qy / rho;
    Je[8 * q + 2] = qx / rho;
  }
}

/* Adjoint of the collision at one cell: f is the pre-collision state, a the
 * adjoint of the post-collision state; returns the adjoint of f in fb and adds
 * the derivative with respect to each relaxation rate into sb. */
static void collide_T_cell(const orc_params *P, const double *M, const double *Minv, const double *f, const double *a,
                           double *fb, double *sb) {
  const int q = P->q;
  double m[MAXQ] = {0}, meq[MAXQ] = {0}, b[MAXQ], cvec[MAXQ], Je[MAXQ * MAXQ];
  for (int i = 0; i < q; ++i) {
    double acc = 0.0;
    for (int j = 0; j < q; ++j) acc += M[i * q + j] * f[j];
    m[i] = acc;
  }
  orc_equilibrium(P, m, meq);
  orc_equilibrium_jacobian(P, m, Je);
  for (int k = 0; k < q; ++k) { /* b = M^{-T} a */
    double acc = 0.0;
    for (int j = 0; j < q; ++j) acc += Minv[j * q + k] * a[j];
    b[k] = acc;
  }
  for (int i = 0; i < q; ++i) {
    double acc = (1.0 - P->s[i]) * b[i];
    for (int k = 0; k < q; ++k) acc += Je[k * q + i] * P->s[k] * b[k];
    cvec[i] = acc;
  }
  for (int j = 0; j < q; ++j) { /* fb = M^T c */
    double acc = 0.0;
    for (int i = 0; i < q; ++i) acc += M[i * q + j] * cvec[i];
    fb[j] = acc;
  }
  for (int k = 0; k < q; ++k) sb[k] += b[k] * (meq[k] - m[k]);
}

int orc_collide_T(const orc_params *P, const uint8_t *tree, const double *h, const double *abar, double *hbar,
                  double *sbar) {
  double M[MAXQ * MAXQ], Minv[MAXQ * MAXQ], f[MAXQ], a[MAXQ], fb[MAXQ];
  orc_moment_matrix(P, M);
  if (orc_moment_matrix_inverse(P, Minv)) return -1;
  for (int l = P->jmin; l <= P->jmax; ++l)
    for (int64_t c = 0; c < ncells(P, l); ++c) {
      if (!is_leaf(P, tree, l, c)) continue;
      for (int k = 0; k < P->q; ++k) {
        f[k] = val_at(P, h, l, k)[c];
        a[k] = val_at(P, abar, l, k)[c];
      }
      collide_T_cell(P, M, Minv, f, a, fb, sbar);
      for (int k = 0; k < P->q; ++k) val_at(P, hbar, l, k)[c] = fb[k];
    }
  return 0;
}

/* Adjoint of the initial datum f = M^{-1} m_eq(m0) on the finest level: from the
 * adjoint abar of the finest-level values, the adjoint of m0 ([nc][N_J^d]). */
int orc_init_T(const orc_params *P, const double *m0, const double *abar, double *mbar) {
  if (P->scheme >= 4) return -1;
  const int q = P->q, J = P->jmax, nc = P->scheme == 3 ? 3 : 1;
  const int64_t NJ = ncells(P, J);
  double Minv[MAXQ * MAXQ], m[MAXQ], Je[MAXQ * MAXQ], b[MAXQ];
  if (orc_moment_matrix_inverse(P, Minv)) return -1;
  for (int64_t c = 0; c < NJ; ++c) {
    for (int i = 0; i < q; ++i) m[i] = i < nc ? m0[(int64_t)i * NJ + c] : 0.0;
    orc_equilibrium_jacobian(P, m, Je);
    for (int k = 0; k < q; ++k) {
      double acc = 0.0;
      for (int j = 0; j < q; ++j) acc += Minv[j * q + k] * val_at(P, abar, J, j)[c];
      b[k] = acc;
    }
    for (int j = 0; j < nc; ++j) {
      double acc = 0.0;
      for (int k = 0; k < q; ++k) acc += Je[k * q + j] * b[k];
      mbar[(int64_t)j * NJ + c] = acc;
    }
  }
  return 0;
}

/* Pre-collision values h of one frozen-mesh step (transfer, reconstruction,
 * transport), written at the leaves of tnew. */
static int step_precollision(const orc_params *P, const uint8_t *told, const uint8_t *tnew, const double *vold,
                             double *h) {
  const int64_t total = orc_total_cells(P);
  double *G = malloc(sizeof(double) * (size_t)(P->q * total));
  double *g = calloc((size_t)(P->q * total), sizeof(double));
  if (!G || !g) { free(G); free(g); return -1; }
  memcpy(G, vold, sizeof(double) * (size_t)(P->q * total));
  orc_reconstruct(P, told, G);
  orc_transfer(P, told, G, tnew, g);
  orc_reconstruct(P, tnew, g);
  orc_transport(P, tnew, g, h, 0);
  free(G);
  free(g);
  return 0;
}

/* One adjoint step: given the leaf values vold of `told` before the step and the
 * adjoint anew of the leaf values of `tnew` after it, the adjoint aold of vold;
 * adds d/ds into sbar. */
int orc_adjoint_step(const orc_params *P, const uint8_t *told, const uint8_t *tnew, const double *vold,
                     const double *anew, double *aold, double *sbar) {
  if (has_walls(P) || P->scheme >= 4 || gam(P) > 1) return -1;
  const int64_t total = orc_total_cells(P), n = P->q * total;
  double *h = calloc((size_t)n, sizeof(double)), *hb = calloc((size_t)n, sizeof(double));
  double *gs = calloc((size_t)n, sizeof(double));
  int rc = -1;
  if (!h || !hb || !gs) goto done;
  if (step_precollision(P, told, tnew, vold, h)) goto done;
  orc_collide_T(P, tnew, h, anew, hb, sbar);
  orc_transport_T(P, tnew, hb, gs);
  orc_reconstruct_T(P, tnew, gs);  /* gs: adjoint of the transferred leaf values */
  memset(aold, 0, sizeof(double) * (size_t)n);
  orc_transfer_T(P, tnew, gs, aold);
  orc_reconstruct_T(P, told, aold);
  rc = 0;
done:
  free(h);
  free(hb);
  free(gs);
  return rc;
}
