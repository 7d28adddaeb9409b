// Internal state of the MI355X implicit-step library.
//
// HBM layout (everything per step is rebuilt from the particles):
//   * cells are tiled in 4x4x4 blocks; only blocks touched by a particle
//     stencil are allocated ("active cell blocks", compact ids in
//     lexicographic block order).  Cell field f of cell l (l = (lx*4+ly)*4+lz)
//     in compact block b lives at f[b*64 + l]; multi-component fields are
//     component-major ([comp][n_cells]) so one wavefront reads 64 consecutive
//     values per component;
//   * nodes are tiled the same way; a node block is active when it holds a
//     corner of an active cell block (cell block cb has its corners in node
//     blocks cb + {0,1}^3);
//   * dense block maps (one int per block of the whole grid) translate block
//     coordinates to compact ids (-1 = inactive).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mpmlite.h"
#include "mpl_math.h"

#define MPL_BS 4
#define MPL_BC 64  // cells (or nodes) per block

// Packed index of the symmetric 9x9 tangent (upper triangle, row-major).
__host__ __device__ constexpr int sym9(int r, int c) {
  return (r <= c) ? (r * 9 - r * (r - 1) / 2 + (c - r)) : (c * 9 - c * (c - 1) / 2 + (r - c));
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};
struct NNState;
struct MGState;

// Dirichlet boxes of the current step as the centre->node kernel reads them
// (a per-context device copy, so that contexts on other streams never share it).
struct BCDev {
  int n;
  int kind[16];
  int axis[16];  // MPL_BC_SLIP_PLANE: the normal axis
  double lo[16][3], hi[16][3], vel[16][3];
};

struct GraphCache {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* key[24] = {};
  int keyn[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int time_mode = 0;  // opts.time_kernels at capture
};

// Device-resident solver scalars (one instance per context).
struct SolverScalars {
  double rz, rz_new, rr, pq, alpha, beta, bnorm2, tol2;
  double red[8];      // generic reduction outputs
  // flexible CG with the learned preconditioner
  double s2;          // sum over free DOFs of Dinv r^2 (network input scale)
  double rr_mark;     // r.r at the last stagnation checkpoint
  double alpha_last;  // single-reduction CG: step length of the last completed iteration
  int32_t fallback;   // 1: switched to Jacobi
  int32_t fb_new;     // 1: switched in this iteration (restart the direction)
  int32_t nn_off;     // 1: skip the network (converged or fallen back)
  int32_t fallbacks;  // number of switches (0 or 1 per solve)
  int32_t done;       // 0 running, 1 converged, 2 breakdown
  int32_t iters;
  int32_t err;        // binning / domain error flags
  int32_t domain_count;
  int32_t n_cblk, n_nblk;
  int32_t n_active_cells, n_active_nodes, n_free_dofs;
  int32_t n_tan_cells;  // cells that carry a tangent (some V_{c,k} != 0)
  int32_t n_fact_cells; // cells stored in the factored layout (several materials: per-block choice)
};

// FP64 view of the boundary's particle arrays (the kernels' layout).
struct Parts64 {
  int64_t n;
  double *x, *v, *F, *G, *m, *V0, *plastic;
  int32_t* mat;
};

struct mpl_ctx {
  int device = 0;  // HIP device current at mpl_create
  mpl_allocator allocator{};  // caller's device-memory callbacks (alloc NULL: hipMalloc)
  // grid
  int dims[3];
  int cbd[3];   // cell-block grid dims (dims/4)
  int nbd[3];   // node-block grid dims (dims/4 + 1)
  double dx, inv_dx, origin[3];
  // materials and options
  int nmat = 1;
  mpl_material mats_in[MPL_MAX_MATERIALS];
  mpl::MatParams mats[MPL_MAX_MATERIALS];
  mpl_solver_opts opts;
  hipStream_t stream = nullptr;
  // private non-blocking stream used only to capture CG chunks into graphs
  // (the caller's stream may be the null stream, which cannot be captured);
  // the graphs are launched on `stream`
  hipStream_t cap_stream = nullptr;
  hipEvent_t cap_order[2] = {nullptr, nullptr};  // orders graph launches with `stream`
  std::string last_error;

  // state flags
  bool unloaded = false, reconstructed = false, tangent_built = false, solved = false;
  int tangent_precision = MPL_F32;
  bool tan_factored = false;     // the stored FP32 tangent is in factored form
  bool tan_mixed = false;        // several materials in FP32: factored or dense per cell block (cfmt)
  bool factored_enabled = true;  // MPL_DENSE_TANGENT=1 in the environment turns it off
  double dt = 0.0;
  int64_t np = 0;
  int n_cblk = 0, n_nblk = 0;

  // binning
  DevBuf cflag, cmap, nflag, nmap, scan_tmp, ccoord, ncoord, c_nbr_node, n_nbr_cell,
      pcell, pkey, bin_count, bin_start, bin_fill, sorted;
  // cell fields (FP64 unless noted)
  DevBuf mc, qc, Gc, Vk, Tk, Sk, Qc, ecell, Abar32, Abar64, Y32, Y64, vcl, Gcl, dvcl;
  // tangent storage: only cells with some V_{c,k} != 0, block-major
  // (Abar[45*coff[cb] + e*count(cb) + rank]), with a 64-bit active mask per
  // cell block (see tan_slot in mpl_grid.h)
  DevBuf cmask, ccnt, coff;
  DevBuf p2c_halo;  // particle -> centre scatter: per-block halo staging
  DevBuf pstage;    // FP64 staging of single-precision particle arrays
  DevBuf cfmt, fcnt; // per cell block: tangent layout (1 factored) and its factored-cell count
  // Anderson acceleration of fixed-point plasticity: the last iterates v and
  // Newton updates f (block layout, FP64), oldest first
  static constexpr int kAA = 5;
  DevBuf aa_v[kAA], aa_f[kAA], aa_tmp, aa_part;
  int aa_n = 0;
  // node fields
  // Dt, mt: inverse Jacobi diagonal and mass in the tangent's precision
  // (read by the CG vector kernels)
  DevBuf Dt, mt;
  // Bj, Bjt: inverted 3x3 node blocks of H (xx, yy, zz, xy, yz, xz), FP64
  // and in the tangent's precision, when block-Jacobi is selected
  DevBuf Bj, Bjt;
  DevBuf Aoff;  // off-diagonal node-block sums of the factored tangent (block-Jacobi only)
  bool bj_built = false;  // Bj/Bjt match the current tangent
  DevBuf mi, vn, vhat, flags, v, g, vt, dir, r, x, p32, p64, q32, q64, z, D, partials,
      dense_tmp32, dense_tmp64;
  // scalars
  DevBuf scal;
  SolverScalars* dscal() const { return (SolverScalars*)scal.p; }
  SolverScalars hscal;

  // captured PCG iteration chunks (replayed while the key matches); one
  // cache per iteration kind (Jacobi, learned, single-reduction Jacobi)
  bool graphs_enabled = false;  // MPL_GRAPHS=1: CG chunks replay from HIP graphs
  GraphCache pcg_cache[3];
  // training-pair collection during Newton solves (0 = off)
  int collect_every = 0;
  double collect_rtol = 1e-10;
  DevBuf xstar;
  DevBuf bcbuf;     // device copy of bc_host
  DevBuf cntbuf;    // per-block active/free counts of the unload
  DevBuf matbuf;    // device copy of mats (MPL_MAX_MATERIALS entries)
  DevBuf Seff;      // fixed-point plasticity: return-mapped base, 9 entries per centre and material
  bool s_general = false;  // energy and tangent read Seff instead of the symmetric stretch
  BCDev bc_host{};  // host staging of the step's Dirichlet boxes (outlives the async copy)
  int fallbacks_total = 0;
  // online training of the learned preconditioner during Newton solves
  // (energy-norm loss on the solver's own residuals; 0 = off)
  int online_every = 0, online_steps = 0;
  float online_lr = 0.f;
  int64_t online_done = 0;     // training steps taken
  double online_loss_sum = 0;  // sum of first-step losses since the last read
  double online_ref_sum = 0;   // the same losses for the Jacobi preconditioner
  int64_t online_loss_n = 0;
  DevBuf ozt, ohz, ogr, opieces;
  // single-reduction CG: u = Dinv r and s = running H p (tangent precision)
  DevBuf cg_u, cg_s, cg_dx;
  DevBuf cg_red;  // its two-level reduction: per-workgroup sums and a ticket counter
  // warm start: the CG solutions of Newton iteration j of the last solves
  // (dense node arrays, so that they survive the change of active blocks),
  // in a ring of kHist per Newton index: whist[j][(whead[j] - k) mod len] is
  // the k-th newest, wcount[j] of them valid
  static constexpr int kWarm = 4;
  static constexpr int kHist = 3;
  DevBuf whist[kWarm][kHist], wtmp, warm_x0;
  int whead[kWarm] = {0, 0, 0, 0}, wcount[kWarm] = {0, 0, 0, 0};
  int whist_len = 0;  // ring length the current warm_start mode uses
  DevBuf gal_w, gal_u, gal_y, gal_part;  // warm_start 4: Galerkin start work space
  bool cg_single = true;  // MPL_CG_CLASSIC=1 in the environment selects the two-reduction loop

  // learned preconditioner (allocated on first use)
  NNState* nn = nullptr;
  // multigrid preconditioner (allocated on first use; mpl_mg.hip)
  MGState* mg = nullptr;
  int tangent_serial = 0;  // incremented by every tangent build

  // timing
  hipEvent_t ev[2] = {nullptr, nullptr};
  std::vector<hipEvent_t> hv_events;
  int hv_event_used = 0;
  bool hv_sample = false;  // time_kernels 2: this launch is the chunk's timed product
  uint32_t sample_rot = 0; // time_kernels 2: rotates the timed iteration over chunks
  int graph_replays = 0;   // chunks launched from graphs since the solve began
  int pcg_expect = 0;      // Jacobi CG: iterations run before the first convergence poll
  int last_pcg[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // previous step's CG count per Newton index
  double hv_ms_total = 0.0;
  int hv_calls = 0;
  // the same for the single-reduction CG update kernel
  std::vector<hipEvent_t> up_events;
  int up_event_used = 0;
  double up_ms_total = 0.0;
  int up_calls = 0;
  int domain_events = 0;

  size_t ncell_alloc() const { return (size_t)n_cblk * MPL_BC; }
  size_t nnode_alloc() const { return (size_t)n_nblk * MPL_BC; }
};

// Arrays of one level of the block grid as the product, diagonal and vector
// kernels read them (the step's grid, or a multigrid level).
struct LevelArrays {
  int n_cblk = 0, n_nblk = 0;
  int64_t ncell = 0, nnode = 0;  // allocated slots (blocks x 64)
  const int* c_nbr_node = nullptr;
  const int* n_nbr_cell = nullptr;
  const uint64_t* cmask = nullptr;  // tangent-carrying cells per cell block
  const int32_t* coff = nullptr;    // their offsets in the compact tangent
  const void* Abar = nullptr;       // tangent in the solve's precision
  bool fact = false, mixed = false; // factored (one material) or per-block layout (cfmt)
  const uint8_t* cfmt = nullptr;
  const double* mi = nullptr;       // node mass (FP64)
  const uint8_t* flags = nullptr;   // node flags
  double inv_dx = 0.0;
};

// ---------------------------------------------------------------- helpers
mpl_status mpl_fail(mpl_ctx* c, mpl_status st, const std::string& msg);
mpl_status mpl_hip_check(mpl_ctx* c, hipError_t e, const char* what);
mpl_status mpl_ensure(mpl_ctx* c, DevBuf& b, size_t bytes);
mpl_status mpl_sync_scalars(mpl_ctx* c);  // copy device scalars to hscal (synchronises)

#define MPL_TRY(expr)                       \
  do {                                      \
    mpl_status _st = (expr);                \
    if (_st != MPL_OK) return _st;          \
  } while (0)
#define MPL_HIP(c, expr) MPL_TRY(mpl_hip_check((c), (expr), #expr))
#define MPL_LAUNCH(c, kern, grid, block, ...)                                     \
  do {                                                                            \
    if ((grid) > 0) {                                                             \
      hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, (c)->stream, __VA_ARGS__); \
      MPL_HIP(c, hipGetLastError());                                              \
    }                                                                             \
  } while (0)

template <class T>
inline T* P(const DevBuf& b) { return (T*)b.p; }

// Exclusive scan of n int32 values (device), total written to *total_dev.
mpl_status mpl_scan_i32(mpl_ctx* c, const int32_t* in, int32_t* out, int64_t n, int32_t* total_dev);

// Internal stages shared by the entry points.
mpl_status mpl_stage_unload(mpl_ctx* c, const Parts64* in, double dt, const double* gravity,
                            const mpl_bc* bcs, int n_bcs, double time);
mpl_status mpl_stage_reconstruct(mpl_ctx* c);
mpl_status mpl_stage_energy(mpl_ctx* c, const double* v_block, bool want_grad, double* energy,
                            double* gnorm2);
mpl_status mpl_stage_tangent(mpl_ctx* c, const double* v_block, int precision);
mpl_status mpl_stage_hv(mpl_ctx* c, const void* u_block, void* Hu_block, int precision, bool dot);
mpl_status mpl_stage_pcg(mpl_ctx* c, const double* b_block, double* x_block, int* iters,
                         double* rel, const double* x0_block = nullptr);
mpl_status mpl_stage_solve(mpl_ctx* c, mpl_stats* st);
mpl_status mpl_stage_precond_apply(mpl_ctx* c, const double* r_block, double* z_block);
mpl_status mpl_stage_load(mpl_ctx* c, const double* v_block, const Parts64* in,
                          const Parts64* out, double dt);
// dense <-> block conversions for node vectors (3 comps) and scalars
mpl_status mpl_dense_to_block_nodes(mpl_ctx* c, const void* dense, void* block, int comps,
                                    int is_f32);
mpl_status mpl_block_to_dense_nodes(mpl_ctx* c, const void* block, void* dense, int comps,
                                    int is_f32);

// Product pieces (own and halo, 6 x cells values) of K p on a level, with
// the level's stored tangent; kernels return at once when s reports a
// finished solve (s may be null).  With partial, one partial sum of p^T K p
// per group of four cell blocks goes there.
template <class T>
mpl_status mpl_level_hv_pieces(mpl_ctx* c, const LevelArrays& L, const T* p, T* pieces,
                               const SolverScalars* s, double* partial = nullptr);
// Inverse Jacobi diagonal of a level's matrix (FP64 and in T) and its node
// masses in T.
template <class T>
mpl_status mpl_level_diag(mpl_ctx* c, const LevelArrays& L, double* D, T* Dt, T* mt);
// The step grid's arrays as a level (tangent in the precision T).
template <class T>
LevelArrays mpl_level0(const mpl_ctx* c);
// Block maps of a block grid from a dense per-cell-block flag array: compact
// cell and node block ids, their coordinates, and the counts at
// totals_dev[0] (cell blocks) and totals_dev[1] (node blocks).  scan needs
// cell blocks + node blocks + 2 ints.
mpl_status mpl_block_maps(mpl_ctx* c, const int dims[3], const int cbd[3], const int nbd[3],
                          int32_t* cflag, int32_t* cmap, int4* ccoord, int32_t* nflag,
                          int32_t* nmap, int4* ncoord, int32_t* scan, int32_t* totals_dev);
// Neighbour tables (8 node blocks per cell block, 8 cell blocks per node block).
mpl_status mpl_block_neighbours(mpl_ctx* c, const int dims[3], const int cbd[3], const int nbd[3],
                                const int4* ccoord, const int4* ncoord, const int32_t* cmap,
                                const int32_t* nmap, int32_t* c_nbr_node, int32_t* n_nbr_cell,
                                int n_cblk, int n_nblk);
// Multigrid-preconditioned CG on the current tangent (mpl_mg.hip); x0 may be null.
mpl_status mpl_stage_pcg_mg(mpl_ctx* c, const double* b, double* x, int* iters, double* rel,
                            const double* x0);
void mpl_mg_destroy(mpl_ctx* c);

// Allocation-free entry point (mpl_noalloc.hip): fetch the device address of
// the fixed scratch array for the context's device once per device.
void mpl_noalloc_attach(mpl_ctx* c);
// Hessian-vector product on block-layout u into block-layout Hu, with the
// product's per-cell pieces in a caller-given buffer (6 x cells x values);
// launches kernels only.
mpl_status mpl_stage_hv_into(mpl_ctx* c, const void* u, void* Hu, void* pieces, int precision);
// zero the non-free nodes of a block-layout node vector (3 components)
mpl_status mpl_mask_free_nodes(mpl_ctx* c, void* u, int is_f32);
// device memory of the context (the caller's allocator or hipMalloc/hipFree)
mpl_status mpl_dev_alloc(mpl_ctx* c, void** p, size_t bytes);
void mpl_dev_free(mpl_ctx* c, void* p, size_t bytes);
// FP64 views of boundary particle arrays: MPL_F64 arrays in place, MPL_F32
// arrays staged to the context's FP64 buffer (x, v, F, G, m, V0, plastic).
mpl_status mpl_particles_in(mpl_ctx* c, const mpl_particles* p, Parts64* out);
// After a successful load into the staging buffer: round x, v, F, G and
// plastic back into the caller's single-precision arrays.
mpl_status mpl_particles_out(mpl_ctx* c, const Parts64* staged, const mpl_particles* p);
