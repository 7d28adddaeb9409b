/*
 * mpmlite.h — C-ABI of the MI355X (gfx950) implementation of the MPM Lite
 * implicit step: linear-kernel particle <-> quadrature resampling and the
 * particle-free incremental-potential Newton solve on the voxel hex mesh.
 *
 * The problem statement follows Alg. 1 of the paper: particle state
 * (x, v, F, G, m, V, material) in, the same state at n+1 out; the mesh is
 * implied by (dx, origin, dims) and rebuilt every step (the grid is
 * transient, Sec. 6).  Sub-steps are exported for testing and measurement.
 *
 * Conventions
 *   - Units SI.  Nodes at origin + i*dx, i in [0, dims]; cells (quadrature
 *     points) at origin + (c + 1/2)*dx, c in [0, dims-1].  dims must be
 *     multiples of 4 (the library tiles cells in 4x4x4 blocks).
 *   - Matrices row-major 3x3; G_ab = dv_a/dx_b.
 *   - Particle arrays are DEVICE pointers, SoA per field, particle-major:
 *     x, v [n][3]; F, G [n][3][3]; m, V0, plastic [n]; mat [n] (int32).
 *     Double precision, or single precision staged to double (the dtype
 *     field of mpl_particles).  The caller owns them; the library never
 *     frees or reallocates them.
 *   - "Dense" grid vectors used by the sub-step entry points are DEVICE
 *     arrays over ALL nodes (dims+1)^3 (or cells dims^3), index
 *     (i*(Ny) + j)*(Nz) + k with i the x index, component-interleaved
 *     ([node][3] for vectors).  Values at inactive nodes are ignored on
 *     input and written as 0 on output.
 *   - All device work is ordered on the stream given to mpl_create.  Calls
 *     synchronise that stream only to read solver control scalars (norms,
 *     energies, iteration flags) back to the host.
 *   - The context owns its grid scratch (grown on demand, reused across
 *     steps, freed by mpl_destroy), from hipMalloc or from the caller's
 *     allocator callbacks (mpl_create_with_allocator).
 *
 * Errors: every call returns an mpl_status; 0 is success.  No exception
 * crosses the ABI.  mpl_last_error() returns a per-context message.
 */
#ifndef MPMLITE_H
#define MPMLITE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPL_MAX_MATERIALS 4

typedef int32_t mpl_status;
enum {
  MPL_OK = 0,
  MPL_ERR_INVALID_ARG = -1,
  MPL_ERR_HIP = -2,
  MPL_ERR_OOM = -3,
  MPL_ERR_NOT_CONVERGED = -4,  /* Newton hit max_newton (state is the last iterate) */
  MPL_ERR_LINESEARCH = -5,     /* no step length passed the line search */
  MPL_ERR_NONFINITE = -6,      /* NaN/Inf in a solver quantity */
  MPL_ERR_DOMAIN = -7,         /* stress outside a model's invertible range, or a
                                  particle stencil leaving the grid */
  MPL_ERR_STATE = -8           /* sub-step called before the step it depends on */
};

/* Constitutive models (Sec. 4.3) and plasticity (applied to particle F). */
/* MPL_WATER: J-based inviscid fluid (Sec. 3, Water), psi = kappa/2 (J - 1)^2
 * with the bulk modulus kappa given as E (nu is not used) and no plasticity;
 * its particles leave each step with F = J^{1/3} I, J updated as
 * (1 + dt tr G_p) J. */
enum { MPL_NEOHOOKEAN = 0, MPL_FIXED_COROTATED = 1, MPL_HENCKY = 2, MPL_WATER = 3 };
enum { MPL_PLASTIC_NONE = 0, MPL_PLASTIC_VON_MISES = 1, MPL_PLASTIC_DRUCKER_PRAGER = 2 };
/* Dirichlet node sets.  The paper treats the mesh as FEM nodes, so a
 * boundary condition is a constraint on node velocities (Sec. 1 and the
 * Integrate step of Alg. 1, v^{n+1} prescribed on constrained nodes):
 *   MPL_BC_STICKY_BOX  every active node in the box has v = 0;
 *   MPL_BC_MOVING_BOX  the box moves with `velocity` (shifted by velocity *
 *                      time) and every active node in it has v = velocity;
 *   MPL_BC_SLIP_PLANE  a frictionless wall: the box does not move, and on
 *                      every active node in it the velocity component along
 *                      the wall normal is 0 while the two tangential
 *                      components stay free.  The normal axis is the one
 *                      nonzero entry of `velocity` (its sign and size do not
 *                      matter); anything else is MPL_ERR_INVALID_ARG.
 * A component, once fixed by any box, stays fixed; its value comes from the
 * last box that fixes it (sticky and moving boxes fix all three). */
enum { MPL_BC_STICKY_BOX = 0, MPL_BC_MOVING_BOX = 1, MPL_BC_SLIP_PLANE = 2 };
/* Precision of the stored tangent and of the Hessian-vector product. */
enum { MPL_F32 = 0, MPL_F64 = 1 };
/* Preconditioner of the Newton linear systems (the preconditioned
 * matrix-free CG of Sec. 5): the inverse diagonal of H (Jacobi); the
 * inverses of its 3x3 node blocks H_ii = m_i I + sum_c (node block of
 * B_c^T Abar_c B_c), which couple a node's three velocity components
 * (block-Jacobi; single-reduction CG only, MPL_CG_CLASSIC=1 rejects it); the
 * learned network (see below); or one geometric multigrid V-cycle (see
 * "multigrid" below), the multigrid-preconditioned CG that the paper names
 * beside plain PCG as an off-the-shelf solver of the same potential (Sec. 7,
 * the vertex block descent comparison). */
enum { MPL_PRECOND_JACOBI = 0, MPL_PRECOND_BLOCK_JACOBI = 1, MPL_PRECOND_LEARNED = 2,
       MPL_PRECOND_MULTIGRID = 3 };

typedef struct {
  double dx;
  double origin[3];
  int32_t dims[3]; /* cells per axis, multiples of 4 */
} mpl_grid;

typedef struct {
  int32_t model;        /* MPL_NEOHOOKEAN | MPL_FIXED_COROTATED | MPL_HENCKY | MPL_WATER */
  int32_t plastic;      /* MPL_PLASTIC_* */
  double E, nu, rho;    /* Young's modulus, Poisson ratio, density (rho unused by the step) */
  double yield_stress;  /* von Mises Kirchhoff yield stress */
  double friction_deg;  /* Drucker-Prager friction angle */
} mpl_material;

typedef struct {
  int32_t hv_precision;   /* MPL_F32 (production) or MPL_F64 (parity) */
  int32_t precond;        /* MPL_PRECOND_JACOBI, _BLOCK_JACOBI or _LEARNED */
  double newton_rtol;     /* stop when |g_free| <= newton_rtol * |g_free(vhat)| */
  double pcg_rtol;        /* stop CG when |r| <= pcg_rtol * |b| */
  int32_t max_newton, max_pcg, max_ls;
  double armijo_c;        /* sufficient-decrease constant */
  int32_t pcg_check_every;/* host polls the device convergence flag every k iterations (inside
                             mpl_step/mpl_solve the first poll of Newton iteration j comes after
                             3/4 of the previous step's count for j; iterations past convergence
                             are no-ops on the device). MPL_GRAPHS=1 in the environment at
                             context creation replays the k iterations from a HIP graph */
  int32_t time_kernels;   /* HIP events around Hessian-vector products: 0 none; 1 every launch
                             (CG chunks then run without graphs); 2 one iteration per CG
                             chunk, its position rotating from chunk to chunk (with graphs:
                             the chunk's last iteration, run eagerly) */
  int32_t warm_start;     /* 1: start the CG of Newton iteration j from the direction that
                             iteration j of the previous solve of this context found (the
                             tolerance stays relative to |b|); 2: from the linear extrapolation
                             2 x_{n-1} - x_{n-2} of the last two solves' directions (1 until two
                             exist); 3: the quadratic one 3 x_{n-1} - 3 x_{n-2} + x_{n-3}; 4: the
                             combination W c of the last (up to) three that minimises the
                             energy norm of the error, (W^T H W) c = W^T b with the current
                             tangent (three extra products and one host synchronisation per
                             solve); 0: start from zero */
  int32_t transfer;       /* MPL_TRANSFER_APIC: the paper's transfers with the affine terms of
                             G_p and G_c (default); MPL_TRANSFER_FLIP_PIC: their FLIP/PIC
                             degradation (Sec. 3, Degradation to FLIP/PIC): G_p does not enter
                             the grid (centre and node velocities are plain weighted averages),
                             and the load interpolates the new node velocity (PIC, which also
                             advects) and the node increment v - v^n (FLIP, added to v_p^n) */
  double flip_ratio;      /* MPL_TRANSFER_FLIP_PIC: v_p <- flip_ratio v_FLIP + (1 - flip_ratio)
                             v_PIC, in [0, 1] */
  int32_t plasticity;     /* MPL_PLASTICITY_AFTER_SOLVE: the plastic projection acts on the
                             particles' F in the load only (default); MPL_PLASTICITY_FIXED_POINT:
                             in addition, at every Newton iterate v the plastic centres' trial
                             F = (I + dt G_c(v)) S_c is return-mapped to F_E and that Newton
                             iteration's energy, gradient and tangent use the base
                             (I + dt G_c(v))^{-1} F_E (Sec. 7, Fixed-Point Plasticity); CG then
                             solves for the elastic response only.  Converges linearly, so it
                             needs more Newton iterations */
  int32_t plastic_anderson;/* with MPL_PLASTICITY_FIXED_POINT: 0 plain fixed point (default); m in
                             1..4: Anderson acceleration of the iterates v_k with the last m + 1
                             Newton updates f_k = v_{k+1} - v_k (after the line search): v_{k+1} =
                             v_k + f_k - sum_j gamma_j (dv_j + df_j), gamma the least-squares fit of
                             f_k by the differences df_j; the accelerated iterate is taken when its
                             gradient (with its own plastic base) is finite and smaller than at v_k,
                             else the plain update, and the history restarts */
  double newton_forcing;  /* 0: every Newton system is solved to pcg_rtol (default).  > 0: inexact
                             Newton with the forcing terms of Eisenstat and Walker (1996, choice 2):
                             the CG of Newton iteration k stops at max(pcg_rtol, eta_k) |b| with
                             eta_0 = newton_forcing, eta_k = min(newton_forcing,
                             0.9 (|g_k| / |g_{k-1}|)^2), raised to 0.9 eta_{k-1}^2 when that exceeds
                             0.1, and never below 0.5 newton_rtol |g_0| / |g_k| (no solve tighter than
                             the Newton tolerance needs).  Newton still stops on newton_rtol */
  int32_t vbd_sweeps;     /* > 0: instead of Newton-PCG, this many sweeps of vertex block descent
                             (Sec. 5, VBD) on the same potential: 8 node colours by index parity;
                             per colour the gradient and the projected FP64 cell tangents are
                             evaluated at the current velocity and every free node of the colour
                             takes v_i -= H_ii^{-1} g_i with its 3x3 block H_ii = m_i I + sum over
                             its cells of their blocks.  Not combined with
                             MPL_PLASTICITY_FIXED_POINT.  The stats report the sweeps as
                             newton_iters and no CG iterations */
  int32_t mg_levels;      /* MPL_PRECOND_MULTIGRID: levels of the V-cycle counting the step's
                             grid, 2..MPL_MG_MAX_LEVELS (0: 4); fewer when a level's cell count
                             per axis is odd or its half would drop below 4 */
  int32_t mg_smooth;      /* damped-Jacobi sweeps before and after each coarse correction
                             (0: 2) */
  int32_t mg_coarse_sweeps;/* damped-Jacobi sweeps on the coarsest level (0: 4) */
  double mg_omega;        /* omega_l lambda_l of every level's sweeps, in (0, 2) (0: 1.6) */
} mpl_solver_opts;

enum { MPL_PLASTICITY_AFTER_SOLVE = 0, MPL_PLASTICITY_FIXED_POINT = 1 };

enum { MPL_TRANSFER_APIC = 0, MPL_TRANSFER_FLIP_PIC = 1 };

/* Particle state (device arrays, SoA, particle-major, see Conventions).
 * dtype is the precision of x, v, F, G, m, V0 and plastic: MPL_F64, or
 * MPL_F32, whose arrays are copied to FP64 staging buffers of the context on
 * entry and the results (x, v, F, G, plastic) rounded back on success; the
 * step computes in FP64 either way.  in and out of one call must have the
 * same dtype. */
typedef struct {
  int64_t n;
  int32_t dtype;                              /* MPL_F64 or MPL_F32 */
  void *x, *v, *F, *G, *m, *V0, *plastic;     /* device; plastic may be NULL */
  int32_t* mat;                               /* device */
} mpl_particles;

typedef struct {
  int32_t kind;           /* MPL_BC_STICKY_BOX | MPL_BC_MOVING_BOX | MPL_BC_SLIP_PLANE */
  double lo[3], hi[3];    /* box at time 0, inclusive (tolerance 1e-6 dx) */
  double velocity[3];     /* MOVING_BOX: prescribed velocity; the box moves with it;
                             SLIP_PLANE: the wall normal (one nonzero entry) */
} mpl_bc;

typedef struct {
  int32_t newton_iters, pcg_iters, ls_halvings, fallbacks;
  int32_t active_cells, active_nodes, free_dofs, cell_blocks, node_blocks;
  double g0_norm, g_norm, energy;
  double hv_ms_total;     /* summed HIP-event time of the timed Hv launches (time_kernels 1 or 2) */
  int32_t hv_calls;       /* number of timed Hv launches */
  double ms_unload, ms_reconstruct, ms_newton, ms_load;  /* host wall clock per stage */
  int32_t domain_events;  /* stretch reconstructions clamped (model range) */
  int32_t tangent_entries;/* stored tangent values read per cell by one Hv: 45 (dense
                             symmetric 9x9) or 25 (single-material FP32 factored form) */
  double hv_model_bytes;  /* bytes one Hv must move by the library's count: 25 values per
                             factored cell, 45 per dense tangent-carrying cell, + 2 x 3
                             values (u read, Hu written) per active node, in the tangent's
                             precision */
  int32_t pcg_per_newton[8]; /* CG iterations of Newton iterations 0..7 */
  int32_t graph_replays;  /* CG chunks launched from captured HIP graphs (0: all eager) */
  int32_t upd_calls;      /* timed launches of the single-reduction CG update kernel */
  double upd_ms_total;    /* their summed HIP-event time (time_kernels 1 or 2) */
  double upd_model_bytes; /* algorithmic bytes of one update launch: 28 e + 55 per free node
                             (e = 4 or 8 bytes for the tangent's precision): p, s, Dinv, m,
                             two product pieces and r read, p, s, u, r written, dx every
                             second and x every eighth iteration */
  int32_t tangent_cells;  /* cells that carry a tangent (some V_{c,k} > 0) */
  int32_t factored_cells; /* of those, cells stored in the factored FP32 layout (25 values read
                             per product): all with one material, with several materials the
                             cells of blocks where no cell holds two materials */
} mpl_stats;

typedef struct mpl_ctx mpl_ctx;

/* Optional device-memory callbacks for a context's grid scratch, so that
 * the caller's allocator (for example PyTorch's caching allocator) owns
 * every buffer the library uses.  alloc returns a device pointer of at
 * least `bytes` bytes (aligned to 256 bytes) for use on hip_stream, or NULL
 * on failure (the call then fails with MPL_ERR_OOM); free releases a
 * pointer alloc returned, with the size it was asked for.  The library
 * synchronises its stream before it frees a buffer.  user is passed back
 * unchanged.  Both callbacks must be set. */
typedef struct {
  void* (*alloc)(void* user, size_t bytes, void* hip_stream);
  void (*free)(void* user, void* ptr, size_t bytes, void* hip_stream);
  void* user;
} mpl_allocator;

/* Library version string. */
const char* mpl_version(void);

/* Create a context.  grid, mats (n_mats <= MPL_MAX_MATERIALS) and opts are
 * copied (the materials also to a device table of the context's own).
 * hip_stream is a hipStream_t (NULL = default stream).  On failure *out is
 * NULL and the status says why.  Contexts share no device state, so several
 * may run at once on one GPU from different host threads and streams; one
 * context must be used by one host thread at a time. */
mpl_status mpl_create(const mpl_grid* grid, const mpl_material* mats, int32_t n_mats,
                      const mpl_solver_opts* opts, void* hip_stream, mpl_ctx** out);
/* mpl_create with the context's device memory taken from the caller's
 * callbacks (allocator may be NULL: hipMalloc/hipFree, as mpl_create). */
mpl_status mpl_create_with_allocator(const mpl_grid* grid, const mpl_material* mats, int32_t n_mats,
                                     const mpl_solver_opts* opts, void* hip_stream,
                                     const mpl_allocator* allocator, mpl_ctx** out);
void mpl_destroy(mpl_ctx* ctx);
const char* mpl_last_error(const mpl_ctx* ctx);
/* Replace the solver options (e.g. tolerances) of an existing context.  A
 * change of warm_start empties the CG start histories of the earlier solves. */
mpl_status mpl_set_opts(mpl_ctx* ctx, const mpl_solver_opts* opts);

/* Alg. 1: one implicit time step.  Unload (Alg. 2), Dirichlet sets and
 * vhat = v^n + dt*gravity on free nodes, stretch reconstruction and the
 * Newton-PCG minimisation of the incremental potential (Alg. 3), Load with
 * advection, F update and plastic projection (Alg. 4).  in may alias out;
 * when they differ and the call fails, out is untouched.  time is the
 * simulation time at the start of the step (moves MOVING_BOX sets).
 * stats (host pointer, may be NULL) receives counters and timings. */
mpl_status mpl_step(mpl_ctx* ctx, const mpl_particles* in, mpl_particles* out, double dt,
                    const double gravity[3], const mpl_bc* bcs, int32_t n_bcs, double time,
                    mpl_stats* stats);

/* Integrate, explicit branch (the explicit case of the Integrate algorithm;
 * Sec. 4 opening, Eq. explicitforce): one explicit time step.  Unload
 * (Alg. 2), Dirichlet sets and vhat as in mpl_step; then the internal nodal
 * force from the unloaded per-centre volumes and Kirchhoff stresses,
 *   f_i = -sum_c sum_k V_{c,k} tau_{c,k} grad w_ic,
 * and v_i^{n+1} = vhat_i + dt f_i / m_i on free nodes, the prescribed
 * velocity on Dirichlet nodes and zero on massless nodes (no stretch
 * reconstruction, no solve); then Load (Alg. 4).  Arguments, aliasing and
 * failure behaviour as for mpl_step.  stats (host, may be NULL) gets the
 * grid counts and the stage times, ms_newton holding the force and node
 * update; its solver counters are zero. */
mpl_status mpl_step_explicit(mpl_ctx* ctx, const mpl_particles* in, mpl_particles* out, double dt,
                             const double gravity[3], const mpl_bc* bcs, int32_t n_bcs, double time,
                             mpl_stats* stats);

/* ---- sub-steps (the same kernels mpl_step runs) ---- */

/* Alg. 2 (Sec. 3.1-3.3): bin particles by dual cell, Kirchhoff stress per
 * particle, atomics-free particle->centre scatter of m, mv, mG, V_k, V_k tau_k
 * (per-block LDS tiles, halo centres staged and combined in a fixed order),
 * normalisation, centre->node gather of m_i and v_i^n, Dirichlet sets and
 * vhat.  Also resets the Newton iterate to vhat. */
mpl_status mpl_unload(mpl_ctx* ctx, const mpl_particles* in, double dt, const double gravity[3],
                      const mpl_bc* bcs, int32_t n_bcs, double time);
/* Alg. 3 first loop (Sec. 4.3, App. C): S_{c,k} from tau_{c,k} (FP64). */
mpl_status mpl_reconstruct_stretch(mpl_ctx* ctx);
/* Incremental potential Phi and its gradient (Sec. 4.2) at the dense node
 * velocity v (device, [(dims+1)^3][3], FP64) or, if v is NULL, at the
 * library's current iterate.  energy: host pointer (may be NULL); grad:
 * device dense array (may be NULL), zero on fixed/massless nodes. */
mpl_status mpl_energy_grad(mpl_ctx* ctx, const double* v, double* energy, double* grad);
/* Per-cell projected tangent Abar_c (9x9 symmetric, 45 stored entries) and
 * the Jacobi diagonal at v (dense device FP64, or NULL = current iterate),
 * stored in `precision` (MPL_F32 or MPL_F64). */
mpl_status mpl_build_tangent(mpl_ctx* ctx, const double* v, int32_t precision);
/* Matrix-free Hessian-vector product Hu = M u + sum_c B_c^T Abar_c B_c u on
 * free DOFs, with the tangent of the last mpl_build_tangent.  u, Hu: dense
 * device arrays [(dims+1)^3][3] of float (MPL_F32) or double (MPL_F64). */
mpl_status mpl_hv(mpl_ctx* ctx, const void* u, void* Hu, int32_t precision);
/* Allocation-free variant of mpl_hv, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments and result as mpl_hv
 * (the same kernels).  Its block-layout copies of u and Hu and the
 * product's per-cell pieces are carved from one fixed device array of
 * MPL_HV_NOALLOC_MAX_BYTES per GPU, held until the process ends, instead of
 * the context's buffers: 2 x 3 x (active node blocks x 64) + 6 x (active
 * cell blocks x 64) values of the precision (each part rounded up to 256
 * bytes) must fit, else MPL_ERR_INVALID_ARG (the 128^3 one-million-cell
 * workload fits in MPL_F32, not in MPL_F64).  Every call on one GPU shares
 * that array and leaves its contents there: calls that overlap on one GPU
 * (other streams, threads or contexts) race.  Enqueues kernels only on the
 * context's stream (no allocation, no memset, no event, no
 * synchronisation); the context's device must be current.  The tangent
 * must have been built (mpl_build_tangent or a solve) beforehand, which is
 * where the context allocates. */
#define MPL_HV_NOALLOC_MAX_BYTES (64ll << 20)
mpl_status mpl_hv_noalloc(mpl_ctx* ctx, const void* u, void* Hu, int32_t precision);
/* Jacobi-PCG on H x = b (b, x dense device FP64), tolerance and iteration
 * cap from the options; iters (host, may be NULL) gets the iteration count
 * and rel_resid (host, may be NULL) the recurrence residual |r|/|b|. */
mpl_status mpl_pcg(mpl_ctx* ctx, const double* b, double* x, int32_t* iters, double* rel_resid);
/* Newton minimisation of Phi from vhat; the solution stays in the context
 * and is copied to v_out (dense device FP64) if non-NULL. */
mpl_status mpl_solve(mpl_ctx* ctx, double* v_out, mpl_stats* stats);
/* Explicit branch of Integrate after mpl_unload (the force and node update
 * of mpl_step_explicit).  The new velocity becomes the context's velocity,
 * so mpl_load with v = NULL moves the particles with it.  v_out, f_out:
 * dense device FP64 arrays [(dims+1)^3][3] or NULL; f_out gets f_i on every
 * node with mass (Dirichlet nodes included) and zero elsewhere. */
mpl_status mpl_integrate_explicit(mpl_ctx* ctx, double* v_out, double* f_out);
/* Alg. 4: node->centre sampling of v (dense device FP64, or NULL = the
 * solved or explicitly integrated velocity), centre->particle interpolation, x += dt v_p,
 * F <- (I + dt G_p) F, plastic projection.  Uses the binning of the last
 * unload; in must be the particles passed to it. */
mpl_status mpl_load(mpl_ctx* ctx, const double* v, const mpl_particles* in, mpl_particles* out,
                    double dt);

/* Dense export of grid fields (device output, FP64). */
enum {
  MPL_FIELD_MASS_C = 0,   /* cells, 1 */
  MPL_FIELD_VEL_C = 1,    /* cells, 3 (v_c of the unload) */
  MPL_FIELD_GRAD_C = 2,   /* cells, 9 (G_c of the unload) */
  MPL_FIELD_VOL_CK = 3,   /* cells, n_mats (material-major: [k][cell]) */
  MPL_FIELD_TAU_CK = 4,   /* cells, n_mats*9 ([k][cell][9]) */
  MPL_FIELD_S_CK = 5,     /* cells, n_mats*9 ([k][cell][9]) */
  MPL_FIELD_ABAR = 6,     /* cells, 81 (full symmetric 9x9) */
  MPL_FIELD_MASS_I = 7,   /* nodes, 1 */
  MPL_FIELD_VEL_I = 8,    /* nodes, 3 (v_i^n of the unload) */
  MPL_FIELD_VHAT = 9,     /* nodes, 3 */
  MPL_FIELD_FIXED = 10,   /* nodes, 1: the prescribed velocity components of the
                             node, bit a for component a (7.0 = all three) */
  MPL_FIELD_V = 11,       /* nodes, 3 (current Newton iterate / solution) */
  MPL_FIELD_DIAG = 12,    /* nodes, 3 (inverse Jacobi diagonal; 0 on fixed/massless nodes) */
  MPL_FIELD_BLOCK_DIAG = 13 /* nodes, 9 (inverted 3x3 node block of H, row-major; 0 on
                             * fixed/massless nodes; needs a tangent built with
                             * precond = MPL_PRECOND_BLOCK_JACOBI) */
};
mpl_status mpl_export_field(mpl_ctx* ctx, int32_t field, double* dense_out);

/* ---- multigrid ----
 *
 * Geometric V-cycle on the voxel mesh (the textbook algorithm; the paper
 * names multigrid-preconditioned CG without defining it, Sec. 7).  Level 0
 * is the step's grid; level l + 1 halves every axis, its cell (I, J, K) being
 * the union of the level-l cells (2I + a, 2J + b, 2K + c), a, b, c in {0, 1},
 * and its nodes the even level-l nodes.  Coarse operator: the same
 * one-point Q1 product (Sec. 3.3) with the coarse spacing, the coarse cell's
 * tangent being the sum of its children's (dense 45 values), plus the
 * lumped coarse mass m_C = P^T m.  P is trilinear interpolation of node
 * values (weight 1 on a co-located node, 1/2 per axis across an odd offset),
 * the restriction is P^T, both zero on fixed or massless DOFs; component a of
 * a coarse node is fixed when the co-located level-l node has mass and that
 * component fixed.  Smoothing: mg_smooth damped-Jacobi sweeps
 * x <- x + omega_l D^-1 (b - A x) before (the first from x = 0) and after each
 * coarse correction, mg_coarse_sweeps on the coarsest level; omega_l =
 * mg_omega / lambda_l with lambda_l the Rayleigh quotient after 20 power
 * iterations on D^-1/2 A D^-1/2 from x_0 = +-1 on the free DOFs, the sign of
 * DOF q = 3 (dense node index of the level) + a being the top bit of
 * SplitMix64(q) (state (q + 1) * 0x9E3779B97F4A7C15 through the published
 * finaliser).  The cycle is symmetric; PCG (Hestenes-Stiefel, r and x in
 * FP64, the cycle in the tangent's precision) uses it as its preconditioner.
 * The hierarchy is built on first use after each tangent build. */
#define MPL_MG_MAX_LEVELS 6
/* One V-cycle z = B r on dense node vectors (FP64, device; [nodes][3]) with
 * the current tangent (mpl_build_tangent first); uses the solver options'
 * mg_* fields.  *n_levels (host, may be NULL) receives the level count and
 * omega (host, MPL_MG_MAX_LEVELS entries, may be NULL) each level's damping.
 * Returns after the context's stream has finished the cycle.  Errors:
 * MPL_ERR_STATE without a tangent; MPL_ERR_NONFINITE when a level's power
 * iteration gives a negative or non-finite eigenvalue estimate. */
mpl_status mpl_mg_apply(mpl_ctx* ctx, const double* r, double* z, int32_t* n_levels, double* omega);
/* Dense export of a multigrid level's data (level >= 1; the hierarchy of the
 * current tangent is built first): field 0 node mass (nodes, 1), 1 fixed
 * components (nodes, 1; bit a for component a, as MPL_FIELD_FIXED), 2 the
 * coarse tangent (cells, 81: full symmetric 9x9), 3 the inverse Jacobi
 * diagonal (nodes, 3).  The level's grid has dims / 2^level cells per axis;
 * dense_out (device, FP64) holds (dims/2^l + 1)^3 node rows or (dims/2^l)^3
 * cell rows.  Returns after the copy; MPL_ERR_INVALID_ARG for a level outside
 * 1 .. n_levels - 1 or an unknown field. */
mpl_status mpl_mg_export(mpl_ctx* ctx, int32_t level, int32_t field, double* dense_out);

/* ---- learned preconditioner ----
 *
 * The paper solves the Newton systems with plain PCG (Alg. 3); this library
 * adds an optional learned preconditioner for them.  A 4-level 3-D U-Net
 * (channels 16/32/64/128; two 3x3x3 convolutions with ReLU per level and
 * side, 2x2x2 stride-2 convolutions down, 2x2x2 stride-2 transposed
 * convolutions up, skip concatenation, a final 1x1x1 convolution) runs on a
 * dense box over all grid nodes (each axis padded up to a multiple of 8),
 * with BF16 weights and activations and FP32 accumulation.  Input channels
 * of node i (free nodes; zero elsewhere): D_i^{-1/2} r_i / s (3), the log of
 * the node's mean diagonal over the free-node mean (1), 1 (1), 11 zero
 * channels.  Output channels 0-2 = o_i; the preconditioned residual is
 *   z_i = D_i^{-1} r_i + s D_i^{-1/2} o_i,   s^2 = sum_free D^{-1} r^2 / (free DOFs),
 * with D the Jacobi diagonal.  Zero weights therefore give Jacobi.  Solves
 * with precond = MPL_PRECOND_LEARNED use flexible CG (Polak-Ribiere beta) and
 * switch to Jacobi for the rest of the solve when z.r <= 0, on NaN/Inf, or
 * when |r| drops by less than 10% over 10 iterations (mpl_stats.fallbacks).
 *
 * Parameters are a flat FP32 vector: for each layer in execution order
 * (enc0a enc0b down0 enc1a enc1b down1 enc2a enc2b down2 bota botb up2 dec2a
 * dec2b up1 dec1a dec1b up0 dec0a dec0b out) W[tap][in][out] then bias[out],
 * taps enumerated with the last spatial axis fastest.  Host pointers below
 * are marked; all tensors are device pointers otherwise. */

/* Number of FP32 parameters (*n, host). */
mpl_status mpl_precond_param_count(mpl_ctx* ctx, int64_t* n);
/* Copy n FP32 parameters from HOST memory; resets the optimiser state. */
mpl_status mpl_precond_set_weights(mpl_ctx* ctx, const float* params_host, int64_t n);
/* Copy the current FP32 parameters to HOST memory. */
mpl_status mpl_precond_get_weights(mpl_ctx* ctx, float* params_host, int64_t n);
/* Network forward on a dense box: x [X][Y][Z][16] FP32, dims = {X, Y, Z}
 * (host, multiples of 8); y [X][Y][Z][16] FP32 (BF16-rounded values). */
mpl_status mpl_nn_forward(mpl_ctx* ctx, const float* x, const int32_t dims[3], float* y);
/* Parameter gradient (FP32, flat, device) of <dy, network(x)>. */
mpl_status mpl_nn_backward(mpl_ctx* ctx, const float* x, const int32_t dims[3], const float* dy,
                           float* grad);
/* One layer of the network on caller tensors, with the kernels of
 * mpl_nn_forward / mpl_nn_backward: layer index in execution order (see the
 * parameter layout above), dims = the network box (multiples of 8; the
 * layer's input and output live at the box >> level of its input and
 * output).  x [in voxels][Ci] (for the decoders' first layers, the
 * concatenation [up, skip]) and dy [out voxels][Co] are device FP32, rounded
 * to BF16 as the network stores them.  y [out voxels][Co] receives the
 * layer output (after ReLU), dx [in voxels][Ci] the gradient w.r.t. x of
 * <dy, y> (not for layer 0, whose input is the network input) and dparams
 * the layer's slice of the parameter gradient (W then bias, FP32); each may
 * be NULL. */
mpl_status mpl_nn_layer_grad(mpl_ctx* ctx, int32_t layer, const float* x, const int32_t dims[3],
                             const float* dy, float* y, float* dx, float* dparams);
/* One Adam step (lr, betas 0.9/0.999, eps 1e-8) on the masked relative L2
 * loss |m (y - t)|^2 / |m t|^2 over output channels 0-2: x [X][Y][Z][16],
 * t [X][Y][Z][3], mask [X][Y][Z] (FP32, device).  *loss (host, may be NULL)
 * receives the loss before the step; grads_out (device FP32,
 * mpl_precond_param_count values, may be NULL) the parameter gradient of
 * that loss, the one the step applies. */
mpl_status mpl_precond_train_step(mpl_ctx* ctx, const float* x, const float* t, const float* mask,
                                  const int32_t dims[3], float lr, float* loss, float* grads_out);
/* z = learned preconditioner applied to r at the Jacobi diagonal of the last
 * mpl_build_tangent (r, z dense device FP64 node vectors). */
mpl_status mpl_precond_apply(mpl_ctx* ctx, const double* r, double* z);
/* Allocate room for `capacity` training pairs on the current grid's box
 * (weights must be set first; 48 bytes per box voxel and pair) and empty
 * the store. */
mpl_status mpl_precond_reserve(mpl_ctx* ctx, int32_t capacity);
/* Collection mode for later mpl_solve / mpl_step calls (every = 0 turns it
 * off): while the store has room, every Newton system is solved to rtol
 * with Jacobi PCG, that solution is the Newton direction, and the same
 * iteration is repeated to store (features of r_k, target
 * D^{1/2}(x* - x_k - D^{-1} r_k)/s, free mask) every `every` iterations. */
mpl_status mpl_precond_collect(mpl_ctx* ctx, int32_t every, double rtol);
/* Online training for later mpl_pcg / mpl_solve / mpl_step calls (every = 0
 * turns it off; weights must be set): inside each linear solve, at the first
 * convergence poll and then every `every` iterations, `steps` Adam steps
 * (learning rate lr) on the energy-norm loss of the solver's current
 * residual r under the current Newton matrix H:
 *   L(z) = (z^T H z / 2 - z^T r) / (r^T D^{-1} r),  z = preconditioner(r),
 * minimised by z = H^{-1} r.  The solve itself is unchanged (its vectors and
 * scalars are not touched); the network changes between its iterations. */
mpl_status mpl_precond_online(mpl_ctx* ctx, int32_t every, int32_t steps, float lr);
/* Online training counters (host pointers, may be NULL): total steps taken,
 * the mean loss of the network before each training burst since the last
 * call, and the mean loss of the Jacobi preconditioner z = D^{-1} r on the
 * same residuals (both then reset).  Lower is better; the network beats
 * Jacobi on those residuals when its loss is below the Jacobi one. */
mpl_status mpl_precond_online_stats(mpl_ctx* ctx, int64_t* steps_done, double* mean_loss,
                                    double* mean_jacobi_loss);
/* Energy-norm loss of the learned preconditioner on a residual, with the
 * kernels of the online training (mpl_precond_online): r is a dense device
 * FP64 node vector; with the Jacobi diagonal D of the last
 * mpl_build_tangent and its Newton matrix H,
 *   z = D^{-1} r + s D^{-1/2} o,  s^2 = sum_free D^{-1} r^2 / (free DOFs),
 *   L(z) = (z^T H z / 2 - z^T r) / (r^T D^{-1} r),
 *   dL/do = s D^{-1/2} (H z - r) / (r^T D^{-1} r)   (free DOFs, 0 elsewhere).
 * o is the network output o_box [X][Y][Z][16] (device FP32 in the layout of
 * mpl_nn_forward, channels 0-2 used, values rounded to BF16 as the network
 * stores them) or, when o_box is NULL, the network's forward on the features
 * of r.  loss and loss_jacobi (host, may be NULL) receive L(z) and the loss
 * of the Jacobi preconditioner z = D^{-1} r; grad_o (dense device FP64 node
 * vector, may be NULL) receives dL/do.  The network's weights are not
 * changed.  Needs weights and a tangent (MPL_ERR_STATE otherwise). */
mpl_status mpl_precond_energy_loss(mpl_ctx* ctx, const double* r, const float* o_box, double* loss,
                                   double* loss_jacobi, double* grad_o);
/* One Adam step of the network's FP32 parameters with a caller-given
 * parameter gradient grad (device FP32, mpl_precond_param_count values),
 * learning rate lr, betas 0.9/0.999, eps 1e-8 and bias correction
 * (Kingma and Ba, 2015); the step number continues from the previous Adam
 * steps since mpl_precond_set_weights, which resets the moments. */
mpl_status mpl_precond_adam_step(mpl_ctx* ctx, const float* grad, float lr);
/* Append one training pair built from the caller's vectors (dense device
 * FP64 node vectors): the residual r = b - H x of a CG iterate x and the
 * solution xstar of H x = b, under the Jacobi diagonal D of the last
 * mpl_build_tangent; the pair stores the network features of r and the
 * target sqrt(D) (xstar - x - D^{-1} r) / s (the output for which the map of
 * mpl_precond_energy_loss gives z = xstar - x).  Needs room in the store
 * (mpl_precond_reserve; MPL_ERR_OOM when full). */
mpl_status mpl_precond_record_pair(mpl_ctx* ctx, const double* r, const double* x, const double* xstar);
/* Copy stored training pair i (0 <= i < mpl_precond_sample_count) to device
 * FP32 arrays on the network box of the current grid (each axis dims + 1
 * rounded up to a multiple of 8): feat [X][Y][Z][16] (the BF16 features as
 * FP32), target [X][Y][Z][3], mask [X][Y][Z] (1 on free nodes).  Any of
 * the three may be NULL. */
mpl_status mpl_precond_get_sample(mpl_ctx* ctx, int32_t i, float* feat, float* target, float* mask);
/* Number of stored training pairs (*n, host). */
mpl_status mpl_precond_sample_count(mpl_ctx* ctx, int32_t* n);
/* n_steps Adam steps on the stored pairs, visited in a pseudo-random order
 * fixed by seed; losses (host, may be NULL) gets each step's loss. */
mpl_status mpl_precond_train(mpl_ctx* ctx, int32_t n_steps, float lr, uint32_t seed, float* losses);

#ifdef __cplusplus
}
#endif
#endif
