/*
 * FP64 CPU oracle for the MPM Lite implicit step — TEST INFRASTRUCTURE ONLY.
 *
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  The product path (the HIP library) never links,
 * includes or calls anything here; the two share no code.
 *
 * Everything is plain, slow and written straight from the paper:
 *   - particle -> cell-centre unload (Sec. 3.1, 3.2; Alg. 2),
 *   - centre -> node gather and node -> centre sampling (Sec. 3.3),
 *   - the rotation-free stretch reference and its reconstruction from the
 *     resampled Kirchhoff stress (Sec. 4.2, 4.3, App. C),
 *   - the incremental potential on the voxel hex mesh (Sec. 4.2, Alg. 3),
 *     minimised by a projected Newton method with Jacobi-PCG,
 *   - load back to particles (Sec. 3.1, Alg. 4).
 *
 * Grid convention (dense): N^3 cells, (N+1)^3 nodes, origin 0, spacing dx.
 *   node (i,j,k)  -> index (i*(N+1)+j)*(N+1)+k,  position (i,j,k)*dx
 *   cell (i,j,k)  -> index (i*N+j)*N+k,          centre ((i,j,k)+1/2)*dx
 * Matrices are row-major 3x3 (9 doubles); G_ab = dv_a/dx_b.
 * All pointers are host pointers owned by the caller.
 * Functions return 0 on success, a negative code on error.
 */
#ifndef MPM_ORACLE_H
#define MPM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* OR_WATER: J-based inviscid fluid (Sec. 3, Water), psi = kappa/2 (J - 1)^2;
 * its bulk modulus kappa travels in or_material.lambda (mu unused), and its
 * particles carry F = J^{1/3} I. */
enum { OR_NEOHOOKEAN = 0, OR_FIXED_COROTATED = 1, OR_HENCKY = 2, OR_WATER = 3 };
enum { OR_PLASTIC_NONE = 0, OR_PLASTIC_VON_MISES = 1, OR_PLASTIC_DRUCKER_PRAGER = 2 };
/* OR_BC_SLIP_PLANE: a frictionless wall.  Its box does not move; on the
 * active nodes inside it the velocity component along the wall normal is
 * fixed at 0 and the two tangential components stay free.  The normal axis
 * is the one nonzero entry of `velocity` (the other two must be 0). */
enum { OR_BC_STICKY_BOX = 0, OR_BC_MOVING_BOX = 1, OR_BC_SLIP_PLANE = 2 };

enum {
  OR_OK = 0,
  OR_ERR_ARG = -1,
  OR_ERR_DOMAIN = -2,        /* stress outside the invertible range of the model */
  OR_ERR_NOT_CONVERGED = -3,
  OR_ERR_LINESEARCH = -4,
  OR_ERR_OUTSIDE = -5        /* a particle's stencil leaves the grid */
};

typedef struct {
  int32_t model;     /* OR_NEOHOOKEAN, OR_FIXED_COROTATED, OR_HENCKY, OR_WATER */
  int32_t plastic;   /* OR_PLASTIC_* */
  double mu, lambda;
  double yield_stress;   /* von Mises: Kirchhoff yield stress */
  double friction_deg;   /* Drucker-Prager friction angle (degrees) */
} or_material;

typedef struct {
  int32_t n;   /* cells per axis */
  double dx;
} or_grid;

typedef struct {
  int32_t kind;              /* OR_BC_* */
  double lo[3], hi[3];       /* box at time 0 (inclusive) */
  double velocity[3];        /* prescribed velocity (MOVING_BOX; STICKY_BOX uses 0);
                                SLIP_PLANE: the wall normal, one nonzero entry */
} or_bc;

typedef struct {
  double newton_rtol, pcg_rtol, armijo_c;
  int32_t max_newton, max_pcg, max_ls;
  /* 1: fixed-point plasticity inside Newton (Sec. 7, Fixed-Point Plasticity):
   * at every Newton iterate the plastic centres' trial F is return-mapped and
   * the iteration's energy uses the resulting base (or_plastic_base) */
  int32_t fixed_point_plasticity;
  /* > 0: instead of Newton-PCG, this many sweeps of vertex block descent
   * (Sec. 5, VBD): 8 node colours by index parity; per colour the gradient
   * and projected tangent are evaluated at the current velocity and every
   * free node of the colour takes v_i -= H_ii^{-1} g_i with the 3x3 node
   * block H_ii = m_i I + sum_c (its block of Abar_c) */
  int32_t vbd_sweeps;
  /* 1: the CG is preconditioned with the inverted 3x3 node blocks of H
   * (or_block_jacobi) instead of its diagonal */
  int32_t block_jacobi;
} or_solver_opts;

typedef struct {
  int32_t newton_iters, pcg_iters_total, ls_halvings;
  double g0_norm, g_norm, energy;
} or_solver_stats;

/* ---- constitutive models (per call: one material point) ---- */
double or_psi(const or_material* mat, const double F[9]);
int or_piola(const or_material* mat, const double F[9], double P[9]);
int or_tau(const or_material* mat, const double F[9], double tau[9]);
int or_dpdf(const or_material* mat, const double F[9], double A[81]);
int or_stretch(const or_material* mat, const double tau[9], double S[9]);
int or_svd3(const double F[9], double U[9], double sig[3], double V[9]);
int or_sym_eigen(int32_t n, const double* A, double* w, double* Q);
int or_project_psd(int32_t n, double* A);
int or_cardano_largest(double p, double q, double* m);
int or_plastic_project(const or_material* mat, double F[9], double* eps_acc);

/* ---- grid stages ---- */
int or_unload(const or_grid* g, int64_t np, const double* x, const double* v,
              const double* G, const double* F, const double* m, const double* V,
              const int32_t* mat, int32_t nmat, const or_material* mats,
              double* mc, double* vc, double* Gc, double* Vck, double* tauck,
              double* mi, double* vi);
/* fixed[node]: bit a set when velocity component a of the node is prescribed
 * (vfix holds its value); a component is a degree of freedom when the node
 * has mass and its bit is clear.  Every routine below that takes `fixed`
 * reads it this way. */
int or_node_bcs(const or_grid* g, const double* mi, int32_t nbc, const or_bc* bcs,
                double time, uint8_t* fixed, double* vfix);
int or_reconstruct(const or_grid* g, int32_t nmat, const or_material* mats,
                   const double* Vck, const double* tauck, double* Sck);
int or_energy_grad(const or_grid* g, int32_t nmat, const or_material* mats, double dt,
                   const double* mi, const double* vhat, const uint8_t* fixed,
                   const double* Vck, const double* Sck, const double* v,
                   double* energy, double* grad);
int or_tangent(const or_grid* g, int32_t nmat, const or_material* mats, double dt,
               const double* Vck, const double* Sck, const double* v, int32_t project,
               double* Abar);
int or_hv(const or_grid* g, const double* mc, const double* mi, const uint8_t* fixed,
          const double* Abar, const double* u, double* Hu);
/* Fixed-point plasticity base (Sec. 7, Fixed-Point Plasticity): for every
 * centre and material with plasticity, F = (I + dt G_c(v)) S0 is return-mapped
 * (the particles' projection) to F_E and Seff = (I + dt G_c(v))^{-1} F_E; where
 * nothing yields, and for materials without plasticity, Seff = S0.  S0, Seff:
 * [nmat][ncell][9]. */
int or_plastic_base(const or_grid* g, int32_t nmat, const or_material* mats, double dt,
                    const double* Vck, const double* S0, const double* v, double* Seff);
int or_explicit_force(const or_grid* g, int32_t nmat, const double* Vck,
                      const double* tauck, double* f);
int or_jacobi_diag(const or_grid* g, const double* mc, const double* mi, const uint8_t* fixed,
                   const double* Abar, double* D);
int or_block_jacobi(const or_grid* g, const double* mc, const double* mi, const uint8_t* fixed,
                    const double* Abar, double* Binv);
int or_solve(const or_grid* g, int32_t nmat, const or_material* mats, double dt,
             const double* mc, const double* mi, const double* vhat, const uint8_t* fixed,
             const double* Vck, const double* Sck, const or_solver_opts* opts,
             double* v, or_solver_stats* stats);
int or_node_to_centre(const or_grid* g, const double* mc, const double* vnode,
                      double* vc, double* Gc);
int or_load(const or_grid* g, double dt, const double* mc, const double* vnode,
            int64_t np, const int32_t* mat, const or_material* mats,
            double* x, double* v, double* G, double* F, double* eps_acc);
/* Load with the FLIP/PIC transfer (Sec. 3, Degradation to FLIP/PIC):
 * v_p <- flip (v_p + dv_p) + (1 - flip) v_PIC with dv the increment
 * vnode - vnode_old sampled like v; x advects with v_PIC. */
int or_load_flip(const or_grid* g, double dt, const double* mc, const double* vnode,
                 const double* vnode_old, double flip, int64_t np, const int32_t* mat,
                 const or_material* mats, double* x, double* v, double* G, double* F,
                 double* eps_acc);
int or_step(const or_grid* g, int32_t nmat, const or_material* mats, double dt,
            const double gravity[3], int32_t nbc, const or_bc* bcs, double time,
            const or_solver_opts* opts, int64_t np, double* x, double* v, double* G,
            double* F, const double* m, const double* V, const int32_t* mat,
            double* eps_acc, or_solver_stats* stats, double* vnode_out);
/* Explicit branch of Integrate (Sec. 4 opening, Eq. explicitforce): unload,
 * Dirichlet sets, v = vhat + dt f / m on free nodes with f the explicit
 * internal force, then load.  vnode_out (may be NULL) gets the node velocity. */
int or_step_explicit(const or_grid* g, int32_t nmat, const or_material* mats, double dt,
                     const double gravity[3], int32_t nbc, const or_bc* bcs, double time,
                     int64_t np, double* x, double* v, double* G, double* F, const double* m,
                     const double* V, const int32_t* mat, double* eps_acc, double* vnode_out);

#ifdef __cplusplus
}
#endif
#endif
