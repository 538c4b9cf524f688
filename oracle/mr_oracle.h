/*
 * Plain FP64 CPU oracle of the multiresolution-adapted lattice Boltzmann step
 * (Bellotti, Gouarin, Graille, Massot, arXiv 2103.02903).
 *
 * TEST INFRASTRUCTURE ONLY. This code is the slow, obviously correct reference
 * that the GPU library is checked against. Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it. It shares no code,
 * header, table or helper with the GPU library, and the GPU library never
 * calls it.
 *
 * Storage is dense per level: every level l = jmin..J keeps a value for every
 * one of its N_l^d cells (N_l = 2^l), so every reconstruction is a plain array
 * lookup. This costs O(q * sum_l 2^{dl}) per step, which is the point: nothing
 * is blocked, fused or reordered beyond what the paper states.
 *
 * Flat array layouts shared with the Python wrapper:
 *   tree   uint8  [level jmin..J][cell]        1 = cell is in the complete tree
 *   values double [level jmin..J][h][cell]     cell index = x (1D), x + N_l*y (2D),
 *                                              x + N_l*(y + N_l*z) (3D)
 *   (vectorial D2Q4: population h = 4 i + k is velocity k of the scheme of
 *   conserved variable i; moment 4 i + j is moment j of that scheme)
 *   detail double [level jmin..J][cell]        D(parent) stored at the parent's slot
 */
#ifndef MR_ORACLE_H
#define MR_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int dim;        /* 1, 2 or 3 */
  int q;          /* 2 (D1Q2), 3 (D1Q3), 9 (D2Q9), 16 (four D2Q4), 6 (D3Q6) */
  int scheme;     /* 1 = D1Q2 advection, 2 = D1Q3 Burgers, 3 = D2Q9 Lallemand-Luo MRT,
                     4 = vectorial D2Q4 for the Euler system (four D2Q4 schemes,
                     one per conserved variable rho, rho u, rho v, E),
                     5 = D3Q6 advection (section "Three dimensional advection
                     equation"; periodic, no adjoint) */
  int jmin, jmax; /* coarsest and finest level */
  int pad_;
  double lambda;   /* lattice velocity, Delta x / Delta t */
  double eq_param; /* D1Q2: advection velocity V; D1Q3: alpha; D2Q9: unused; Euler: gamma_gas */
  double eps;      /* threshold epsilon >= 0 */
  double mu_bar;   /* regularity guess in [0, 2*gamma+1] */
  double s[16];    /* relaxation rate of each moment (0 for conserved moments) */
  /* Boundary of each side (section "Boundary conditions"), order x-, x+, y-, y+:
   * 0 periodic, 1 copy, 2 bounce back, 3 anti bounce back (eq. refBoundaryConditions).
   * An axis is periodic when both of its sides are 0, else both must be walls;
   * 1D uses x only. */
  int bc[4];
  /* Evaluation of the incoming values at a wall (eq. AdvectionOnBoundary):
   * 0 directly on the leaf (the paper's choice), 1 by the reconstruction. */
  int bc_eval;
  /* Prediction stencil half-width gamma = 1, 2 or 3 (Table 1; the grading box
   * grows with it), and the sibling metric of the details: 0 the max norm of
   * section "Mesh coarsening", 1 the l2 form of its footnote,
   * 2^{-d/2} (sum over the siblings of d^2)^{1/2}. */
  int gamma;
  int metric;
  int pad3_;
  /* D3Q6: the advection velocity (V_x, V_y, V_z) of the equilibrium
   * m_eq = (u, V_x u, V_y u, V_z u, 0, 0); unused by the other schemes. */
  double vel[3];
} orc_params;

/* Number of cells summed over levels jmin..J, and the offset of level l. */
int64_t orc_total_cells(const orc_params *P);
int64_t orc_level_offset(const orc_params *P, int l);

/* Initial datum at equilibrium on the full finest mesh (Algorithm 1):
 * m0 holds the conserved moments at the finest cells, layout [nc][N_J^d]
 * (nc = 1 for D1Q2/D1Q3, 3 for D2Q9: rho, q_x, q_y; 4 for the Euler system:
 * rho, rho u, rho v, E). */
int orc_init(const orc_params *P, const double *m0, uint8_t *tree, double *values);

/* Reconstruction on every cell of every level: projection upward on internal
 * tree cells, then zero-detail prediction downward on cells outside the tree.
 * `values` must hold the leaf values; on return it is dense on every level. */
int orc_reconstruct(const orc_params *P, const uint8_t *tree, double *values);

/* Prediction of one child cell (level l, index cx[,cy[,cz]]) from the dense
 * data of level l-1 of one population. */
double orc_predict(const orc_params *P, const double *parent_level, int l, int cx, int cy);
double orc_predict3(const orc_params *P, const double *parent_level, int l, int cx, int cy, int cz);

/* Details: for every parent p at level l-1 whose children are in the tree,
 * D[l-1][p] = max_h max_children |f - prediction| (metric 0), or
 * max_h 2^{-d} sum_children (f - prediction)^2, the square of the l2 form
 * (metric 1; compared with squared thresholds). Other slots are set to -1.
 * `values` must be dense (output of orc_reconstruct). */
int orc_details(const orc_params *P, const uint8_t *tree, const double *values, double *D);

/* New tree G(H_eps(T_eps(tree))) from the old tree and its details. */
int orc_adapt_tree(const orc_params *P, const uint8_t *told, const double *D, uint8_t *tnew);

/* One full time step of Algorithm 1, in place: adapt, transfer, transport,
 * collide. `values` holds leaf values (post-collision) before and after. */
int orc_step(const orc_params *P, uint8_t *tree, double *values);

/* Pieces of the step, exposed for the tests. */
int orc_transfer(const orc_params *P, const uint8_t *told, const double *values_old_dense,
                 const uint8_t *tnew, double *values_new);
int orc_transport(const orc_params *P, const uint8_t *tree, const double *values_dense,
                  double *values_out, int definition_form);
int orc_collide(const orc_params *P, const uint8_t *tree, double *values);
void orc_collide_cell(const orc_params *P, double *f);

/* Mesh decision in single precision: reconstruction and details of the float
 * leaf values evaluated in float (same expressions and order), thresholds
 * rounded to float; optionally returns the float details (as double). */
int orc_new_tree_f32(const orc_params *P, const uint8_t *tree, const float *leaf_values, uint8_t *tnew,
                     double *D_out);

/* One step on a given new mesh (transfer, transport, collide). */
int orc_step_frozen(const orc_params *P, uint8_t *tree, const uint8_t *tnew, double *values);

/* Adjoint on frozen meshes (transposes of the step's linear maps and of the
 * linearised collision; each adds into its output in a fixed order). Periodic
 * boundaries, gamma = 1, d <= 2 and the schemes 1..3 only: otherwise they
 * return -1. */
int orc_predict_stencil(const orc_params *P, int l, int cx, int cy, int64_t *idx, double *w);
int orc_reconstruct_T(const orc_params *P, const uint8_t *tree, double *g);
int orc_transport_T(const orc_params *P, const uint8_t *tree, const double *ob, double *gs);
int orc_transfer_T(const orc_params *P, const uint8_t *tnew, const double *gnew, double *gold);
void orc_equilibrium_jacobian(const orc_params *P, const double *m, double *Je);
int orc_collide_T(const orc_params *P, const uint8_t *tree, const double *h, const double *abar, double *hbar,
                  double *sbar);
int orc_init_T(const orc_params *P, const double *m0, const double *abar, double *mbar);
int orc_adjoint_step(const orc_params *P, const uint8_t *told, const uint8_t *tnew, const double *vold,
                     const double *anew, double *aold, double *sbar);

/* Uniform reference scheme on level J only: values layout [h][N_J^d]; at a wall
 * the incoming population of a boundary cell is set from that cell by the
 * side's condition (eq. refBoundaryConditions). */
int orc_uniform_step(const orc_params *P, double *fJ);

/* Moment matrix M and its inverse (q*q, row-major), and equilibrium moments. */
void orc_moment_matrix(const orc_params *P, double *M);
int orc_moment_matrix_inverse(const orc_params *P, double *Minv);
void orc_equilibrium(const orc_params *P, const double *m, double *meq);
/* Logical velocities eta^h, layout [q][3] (components beyond the dimension 0). */
void orc_velocities(const orc_params *P, int *eta);

/* Host threads of the oracle's parallel per-cell loops (results do not depend
 * on it): sets the count when n > 0, returns the count in use. */
int orc_threads(int n);

/* Diagnostics. */
int orc_leaf_counts(const orc_params *P, const uint8_t *tree, int64_t *counts /* [J+1] */);
double orc_mass(const orc_params *P, const uint8_t *tree, const double *values);
int orc_check_tree(const orc_params *P, const uint8_t *tree); /* 0 = graded complete tree */

#ifdef __cplusplus
}
#endif
#endif
