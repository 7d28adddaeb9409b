// Load (Alg. 4; Sec. 3.1, 3.3), the full step (Alg. 1) and field export.
#include <chrono>
#include <cmath>

#include "mpl_grid.h"

using namespace mpl;

namespace {


struct ParticlesIn {
  const double *x, *v, *F, *G, *m, *V, *plastic;
  const int32_t* mat;
  int64_t n;
};
struct ParticlesOut {
  double *x, *v, *F, *G, *plastic;
};

// v_c = sum_i w_ic v_i (w_ic = 1/8), G_c = sum_i v_i (x) grad w_ic on cells
// with m_c != 0 (hourglass modes of v_i vanish here, Sec. 6).
// With vold (the FLIP/PIC transfer) the node increment v - vold is sampled
// the same way into dvcl.
__global__ __launch_bounds__(64) void k_n2c(const double* __restrict__ v, int64_t nnode,
                                            const int* __restrict__ c_nbr_node,
                                            const double* __restrict__ mc, int64_t ncell,
                                            double inv4dx, double* __restrict__ vcl,
                                            double* __restrict__ Gcl,
                                            const double* __restrict__ vold,
                                            double* __restrict__ dvcl) {
  const int cb = blockIdx.x, l = threadIdx.x;
  const int64_t ci = (int64_t)cb * MPL_BC + l;
  double vc[3] = {0, 0, 0}, G[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, dvc[3] = {0, 0, 0};
  if (mc[ci] != 0.0) {
    for (int d = 0; d < 8; ++d) {
      const int ni = corner_node(c_nbr_node, cb, l, d);
      double gw[3];
      corner_grad(d, inv4dx, gw);
      for (int a = 0; a < 3; ++a) {
        const double va = v[a * nnode + ni];
        vc[a] += va / 8.0;
        if (vold) dvc[a] += (va - vold[a * nnode + ni]) / 8.0;
        for (int b = 0; b < 3; ++b) G[a * 3 + b] += va * gw[b];
      }
    }
  }
  for (int a = 0; a < 3; ++a) vcl[a * ncell + ci] = vc[a];
  for (int e = 0; e < 9; ++e) Gcl[e * ncell + ci] = G[e];
  if (vold)
    for (int a = 0; a < 3; ++a) dvcl[a * ncell + ci] = dvc[a];
}

// v_p = sum_c w_cp v_c, G_p = sum_c w_cp G_c (weights at x^n, as in the
// unload), x += dt v_p, F <- (I + dt G_p) F, then the plastic projection.
// FLIP/PIC transfer (dvcl non-null): v_p <- flip (v_p^n + dv_p) + (1 - flip) v_PIC
// with dv_p interpolated from the centre increments; x advects with v_PIC.
__global__ __launch_bounds__(256) void k_c2p(ParticlesIn in, ParticlesOut out, GridDev g,
                                             const int32_t* __restrict__ cmap,
                      const double* __restrict__ vcl, const double* __restrict__ Gcl, int64_t ncell,
                      double dt, const double* __restrict__ dvcl, double flip,
                      int32_t* __restrict__ err,
    const MatParams* __restrict__ mats) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= in.n) return;
  double xp[3], f[3];
  int b[3];
  for (int a = 0; a < 3; ++a) {
    xp[a] = in.x[3 * p + a];
    const double xi = (xp[a] - g.origin[a]) / g.dx - 0.5;
    const double fb = floor(xi);
    b[a] = (int)fb;
    f[a] = xi - fb;
  }
  double vp[3] = {0, 0, 0}, Gp[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  // the 8 block lookups first, then the centre values four corners at a
  // time, all loads of a batch in flight together; the sums run in corner
  // order (a corner with zero weight or no block adds nothing)
  double w[8];
  int64_t ci[8];
#pragma unroll
  for (int d = 0; d < 8; ++d) {
    const int dx = (d >> 2) & 1, dy = (d >> 1) & 1, dz = d & 1;
    w[d] = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) * (dz ? f[2] : 1.0 - f[2]);
    const int cx = b[0] + dx, cy = b[1] + dy, cz = b[2] + dz;
    // a corner outside the grid (possible with zero weight) has no block
    const bool inside = cx >= 0 && cy >= 0 && cz >= 0 && cx < g.dims[0] && cy < g.dims[1] && cz < g.dims[2];
    const int blk = inside ? cmap[((cx >> 2) * g.cbd[1] + (cy >> 2)) * g.cbd[2] + (cz >> 2)] : -1;
    ci[d] = blk < 0 ? -1 : (int64_t)blk * MPL_BC + local_index(cx & 3, cy & 3, cz & 3);
  }
#pragma unroll
  for (int d = 0; d < 8; ++d)
    if (w[d] != 0.0 && ci[d] < 0) atomicOr(err, 16);
#pragma unroll
  for (int h = 0; h < 8; h += 4) {
    double vv[4][3], GG[4][9];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t c = ci[h + k] < 0 ? 0 : ci[h + k];
#pragma unroll
      for (int a = 0; a < 3; ++a) vv[k][a] = vcl[a * ncell + c];
#pragma unroll
      for (int e = 0; e < 9; ++e) GG[k][e] = Gcl[e * ncell + c];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int d = h + k;
      if (w[d] == 0.0 || ci[d] < 0) continue;
#pragma unroll
      for (int a = 0; a < 3; ++a) vp[a] += w[d] * vv[k][a];
#pragma unroll
      for (int e = 0; e < 9; ++e) Gp[e] += w[d] * GG[k][e];
    }
  }
  double vnew[3] = {vp[0], vp[1], vp[2]};
  if (dvcl) {
    double dvp[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int d = 0; d < 8; ++d) {
      if (w[d] == 0.0 || ci[d] < 0) continue;
#pragma unroll
      for (int a = 0; a < 3; ++a) dvp[a] += w[d] * dvcl[a * ncell + ci[d]];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) vnew[a] = flip * (in.v[3 * p + a] + dvp[a]) + (1.0 - flip) * vp[a];
  }
  double F[9], A[9], Fn[9];
  for (int e = 0; e < 9; ++e) {
    F[e] = in.F[9 * p + e];
    A[e] = dt * Gp[e];
  }
  A[0] += 1.0; A[4] += 1.0; A[8] += 1.0;
  const int k = in.mat[p];
  double dg = 0.0;
  if (mats[k].model == WATER) {
    // J-based water: J <- (1 + dt tr G_p) J, carried as F = J^{1/3} I
    const double Jn = (1.0 + dt * (Gp[0] + Gp[4] + Gp[8])) * det(F);
    if (!(Jn > 0.0)) atomicOr(err, 32);
    const double c = cbrt(Jn);
#pragma unroll
    for (int e = 0; e < 9; ++e) Fn[e] = (e % 4 == 0) ? c : 0.0;
  } else {
    mul(A, F, Fn);
    dg = plastic_project(mats[k], Fn);
  }
  const double pl = in.plastic ? in.plastic[p] : 0.0;
  for (int a = 0; a < 3; ++a) {
    out.v[3 * p + a] = vnew[a];
    out.x[3 * p + a] = xp[a] + dt * vp[a];
  }
  for (int e = 0; e < 9; ++e) {
    out.G[9 * p + e] = Gp[e];
    out.F[9 * p + e] = Fn[e];
  }
  if (out.plastic) out.plastic[p] = pl + dg;
}

template <class T>
__global__ void k_export_cells(const T* __restrict__ src, int comps, int64_t comp_stride,
                               const int4* __restrict__ ccoord, int n_cblk, int nx, int ny, int nz,
                               double* __restrict__ dense, int dense_comps, int comp_offset,
                               int64_t dense_stride) {
  const int b = blockIdx.x, l = threadIdx.x;
  if (b >= n_cblk) return;
  const int4 bc = ccoord[b];
  const int i = bc.x * 4 + local_x(l), j = bc.y * 4 + local_y(l), k = bc.z * 4 + local_z(l);
  const int64_t di = ((int64_t)i * ny + j) * nz + k;
  for (int a = 0; a < comps; ++a)
    dense[dense_stride + di * dense_comps + comp_offset + a] =
        (double)src[a * comp_stride + (int64_t)b * MPL_BC + l];
}

__global__ void k_export_abar32(const float* __restrict__ Ab, const uint64_t* __restrict__ cmask,
                                const int32_t* __restrict__ coff,
                                const int4* __restrict__ ccoord, int n_cblk, int nx, int ny, int nz,
                                double* __restrict__ dense) {
  const int b = blockIdx.x, l = threadIdx.x;
  if (b >= n_cblk) return;
  const int4 bc = ccoord[b];
  const int i = bc.x * 4 + local_x(l), j = bc.y * 4 + local_y(l), k = bc.z * 4 + local_z(l);
  const int64_t di = ((int64_t)i * ny + j) * nz + k;
  const TanSlot ts = tan_slot(cmask, coff, b, l, MPL_TAN_DENSE);
  if (!ts.active) return;
  for (int r = 0; r < 9; ++r)
    for (int c = 0; c < 9; ++c)
      dense[di * 81 + r * 9 + c] = (double)Ab[ts.base + (int64_t)sym9(r, c) * ts.n + ts.rank];
}
__global__ void k_export_abar64(const double* __restrict__ Ab, const uint64_t* __restrict__ cmask,
                                const int32_t* __restrict__ coff,
                                const int4* __restrict__ ccoord, int n_cblk, int nx, int ny, int nz,
                                double* __restrict__ dense) {
  const int b = blockIdx.x, l = threadIdx.x;
  if (b >= n_cblk) return;
  const int4 bc = ccoord[b];
  const int i = bc.x * 4 + local_x(l), j = bc.y * 4 + local_y(l), k = bc.z * 4 + local_z(l);
  const int64_t di = ((int64_t)i * ny + j) * nz + k;
  const TanSlot ts = tan_slot(cmask, coff, b, l, MPL_TAN_DENSE);
  if (!ts.active) return;
  for (int r = 0; r < 9; ++r)
    for (int c = 0; c < 9; ++c) dense[di * 81 + r * 9 + c] = Ab[ts.base + (int64_t)sym9(r, c) * ts.n + ts.rank];
}

// Factored FP32 tangent -> dense 9x9: column c is the factored product
// applied to the unit velocity gradient e_c (FP64 arithmetic on the stored
// FP32 factors).
// With several materials (cfmt given) the blocks use 45 slots per cell and
// a dense block (cfmt 0) is exported as stored.
__global__ void k_export_abar_fact(const float* __restrict__ Ab, const uint64_t* __restrict__ cmask,
                                   const int32_t* __restrict__ coff, const int4* __restrict__ ccoord,
                                   int n_cblk, int nx, int ny, int nz, double* __restrict__ dense,
                                   const uint8_t* __restrict__ cfmt) {
  const int b = blockIdx.x, l = threadIdx.x;
  if (b >= n_cblk) return;
  const int4 bc = ccoord[b];
  const int i0 = bc.x * 4 + local_x(l), j0 = bc.y * 4 + local_y(l), k0 = bc.z * 4 + local_z(l);
  const int64_t di = ((int64_t)i0 * ny + j0) * nz + k0;
  const TanSlot ts = tan_slot(cmask, coff, b, l, cfmt ? MPL_TAN_DENSE : MPL_TAN_FACT);
  if (!ts.active) return;
  if (cfmt && cfmt[b] == 0) {
    for (int r = 0; r < 9; ++r)
      for (int c2 = 0; c2 < 9; ++c2)
        dense[di * 81 + r * 9 + c2] = (double)Ab[ts.base + (int64_t)sym9(r, c2) * ts.n + ts.rank];
    return;
  }
  double f[MPL_TAN_FACT_READ];
  for (int e = 0; e < MPL_TAN_FACT_READ; ++e) f[e] = (double)Ab[ts.base + (int64_t)e * ts.n + ts.rank];
  double U[9];
  quat_to_rot<double>(f[0], f[1], f[2], f[3], U);
  const double* M = f + 4;
  const double* A3 = f + 13;
  const double* pc = f + 19;
  for (int col = 0; col < 9; ++col) {
    double g[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    g[col] = 1.0;
    double t1[9], gh[9], yh[9], t2[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) t1[i * 3 + j] = U[i] * g[j] + U[3 + i] * g[3 + j] + U[6 + i] * g[6 + j];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        gh[i * 3 + j] = t1[i * 3] * M[j] + t1[i * 3 + 1] * M[3 + j] + t1[i * 3 + 2] * M[6 + j];
    yh[0] = A3[0] * gh[0] + A3[1] * gh[4] + A3[2] * gh[8];
    yh[4] = A3[1] * gh[0] + A3[3] * gh[4] + A3[4] * gh[8];
    yh[8] = A3[2] * gh[0] + A3[4] * gh[4] + A3[5] * gh[8];
    yh[1] = pc[0] * gh[1] + pc[1] * gh[3];
    yh[3] = pc[1] * gh[1] + pc[0] * gh[3];
    yh[5] = pc[2] * gh[5] + pc[3] * gh[7];
    yh[7] = pc[3] * gh[5] + pc[2] * gh[7];
    yh[2] = pc[4] * gh[2] + pc[5] * gh[6];
    yh[6] = pc[5] * gh[2] + pc[4] * gh[6];
    for (int a = 0; a < 3; ++a)
      for (int j = 0; j < 3; ++j)
        t2[a * 3 + j] = U[a * 3] * yh[j] + U[a * 3 + 1] * yh[3 + j] + U[a * 3 + 2] * yh[6 + j];
    for (int a = 0; a < 3; ++a)
      for (int bb = 0; bb < 3; ++bb)
        dense[di * 81 + (a * 3 + bb) * 9 + col] =
            t2[a * 3] * M[bb * 3] + t2[a * 3 + 1] * M[bb * 3 + 1] + t2[a * 3 + 2] * M[bb * 3 + 2];
  }
}

// symmetric 6 -> full 9 for tau / S exports
__global__ void k_export_sym(const double* __restrict__ src, int64_t ncell, int K,
                             const int4* __restrict__ ccoord, int n_cblk, int nx, int ny, int nz,
                             double* __restrict__ dense) {
  const int b = blockIdx.x, l = threadIdx.x;
  if (b >= n_cblk) return;
  const int4 bc = ccoord[b];
  const int i = bc.x * 4 + local_x(l), j = bc.y * 4 + local_y(l), k = bc.z * 4 + local_z(l);
  const int64_t di = ((int64_t)i * ny + j) * nz + k;
  const int64_t ci = (int64_t)b * MPL_BC + l;
  const int64_t ncd = (int64_t)nx * ny * nz;
  for (int m = 0; m < K; ++m) {
    double s6[6], A[9];
    for (int q = 0; q < 6; ++q) s6[q] = src[(m * 6 + q) * ncell + ci];
    sym_to_full(s6, A);
    for (int e = 0; e < 9; ++e) dense[(m * ncd + di) * 9 + e] = A[e];
  }
}

__global__ void k_flags_to_double(const uint8_t* __restrict__ fl, double* __restrict__ out,
                                  int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // the prescribed components of an active node, one bit each
  int bits = 0;
  if (fl[i] & MPL_NODE_ACTIVE)
    for (int a = 0; a < 3; ++a) bits |= mpl_free(fl[i], a) ? 0 : (1 << a);
  out[i] = (double)bits;
}

// the six stored entries (xx, yy, zz, xy, yz, xz) of symmetric node blocks,
// component-major, to all nine (row-major), component-major
__global__ void k_sym6_to_9(const double* __restrict__ b6, double* __restrict__ b9, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int map[9] = {0, 3, 5, 3, 1, 4, 5, 4, 2};
  for (int e = 0; e < 9; ++e) b9[e * n + i] = b6[map[e] * n + i];
}

double wall_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

}  // namespace

mpl_status mpl_stage_load(mpl_ctx* c, const double* v, const Parts64* in, const Parts64* out,
                          double dt) {
  if (!c->unloaded) return mpl_fail(c, MPL_ERR_STATE, "load before unload");
  if (!in || !out || in->n != c->np || out->n != in->n)
    return mpl_fail(c, MPL_ERR_INVALID_ARG, "load needs the unloaded particle set");
  if (in->n > 0 && (!out->x || !out->v || !out->F || !out->G))
    return mpl_fail(c, MPL_ERR_INVALID_ARG, "output particle arrays missing");
  const int64_t ncell = (int64_t)c->ncell_alloc(), nnode = (int64_t)c->nnode_alloc();
  MPL_TRY(mpl_ensure(c, c->vcl, 8 * 3 * ncell));
  MPL_TRY(mpl_ensure(c, c->Gcl, 8 * 9 * ncell));
  const bool flip = c->opts.transfer == MPL_TRANSFER_FLIP_PIC;
  if (flip) MPL_TRY(mpl_ensure(c, c->dvcl, 8 * 3 * ncell));
  MPL_LAUNCH(c, k_n2c, c->n_cblk, 64, v, nnode, P<int>(c->c_nbr_node), P<double>(c->mc), ncell,
             0.25 * c->inv_dx, P<double>(c->vcl), P<double>(c->Gcl),
             flip ? P<double>(c->vn) : (const double*)nullptr, flip ? P<double>(c->dvcl) : nullptr);
  ParticlesIn pi{in->x, in->v, in->F, in->G, in->m, in->V0, in->plastic, in->mat, in->n};
  ParticlesOut po{out->x, out->v, out->F, out->G, out->plastic};
  MPL_LAUNCH(c, k_c2p, (int)((in->n + 255) / 256), 256, pi, po, grid_dev(c), P<int32_t>(c->cmap),
             P<double>(c->vcl), P<double>(c->Gcl), ncell, dt,
             flip ? P<double>(c->dvcl) : (const double*)nullptr, c->opts.flip_ratio, &c->dscal()->err, P<MatParams>(c->matbuf));
  MPL_TRY(mpl_sync_scalars(c));
  if (c->hscal.err & 16) return mpl_fail(c, MPL_ERR_HIP, "internal: load reached an inactive block");
  if (c->hscal.err & 32)
    return mpl_fail(c, MPL_ERR_DOMAIN, "a water particle's volume ratio (1 + dt tr G) J is not positive");
  return MPL_OK;
}

extern "C" {

mpl_status mpl_load(mpl_ctx* c, const double* v, const mpl_particles* in, mpl_particles* out,
                    double dt) {
  if (!c) return MPL_ERR_INVALID_ARG;
  if (!c->unloaded) return mpl_fail(c, MPL_ERR_STATE, "load before unload");
  const double* vb = P<double>(c->v);
  if (v) {
    MPL_TRY(mpl_ensure(c, c->vt, 8 * 3 * (int64_t)c->nnode_alloc()));
    MPL_TRY(mpl_dense_to_block_nodes(c, v, c->vt.p, 3, 0));
    vb = P<double>(c->vt);
  } else if (!c->solved) {
    return mpl_fail(c, MPL_ERR_STATE, "load without a velocity needs a solved step");
  }
  if (!in || !out) return MPL_ERR_INVALID_ARG;
  if (out->dtype != in->dtype) return mpl_fail(c, MPL_ERR_INVALID_ARG, "in and out particle dtypes differ");
  Parts64 pin, pout;
  MPL_TRY(mpl_particles_in(c, in, &pin));
  if (in->dtype == MPL_F32) pout = pin;  // load into the staging buffer, then round back
  else MPL_TRY(mpl_particles_in(c, out, &pout));
  MPL_TRY(mpl_stage_load(c, vb, &pin, &pout, dt));
  if (in->dtype == MPL_F32) MPL_TRY(mpl_particles_out(c, &pout, out));
  return MPL_OK;
}

mpl_status mpl_step(mpl_ctx* c, const mpl_particles* in, mpl_particles* out, double dt,
                    const double gravity[3], const mpl_bc* bcs, int32_t n_bcs, double time,
                    mpl_stats* stats) {
  if (!c || !in || !out) return MPL_ERR_INVALID_ARG;
  if (out->dtype != in->dtype) return mpl_fail(c, MPL_ERR_INVALID_ARG, "in and out particle dtypes differ");
  mpl_stats st{};
  double t0 = wall_ms();
  Parts64 pin, pout;
  MPL_TRY(mpl_particles_in(c, in, &pin));
  if (in->dtype == MPL_F32) pout = pin;
  else MPL_TRY(mpl_particles_in(c, out, &pout));
  MPL_TRY(mpl_stage_unload(c, &pin, dt, gravity, bcs, n_bcs, time));
  double t1 = wall_ms();
  MPL_TRY(mpl_stage_reconstruct(c));
  MPL_TRY(mpl_sync_scalars(c));
  double t2 = wall_ms();
  mpl_status s = mpl_stage_solve(c, &st);
  double t3 = wall_ms();
  if (s != MPL_OK) {
    if (stats) *stats = st;
    return s;
  }
  MPL_TRY(mpl_stage_load(c, P<double>(c->v), &pin, &pout, dt));
  if (in->dtype == MPL_F32) MPL_TRY(mpl_particles_out(c, &pout, out));
  double t4 = wall_ms();
  st.active_cells = c->hscal.n_active_cells;
  st.active_nodes = c->hscal.n_active_nodes;
  st.free_dofs = c->hscal.n_free_dofs;
  st.cell_blocks = c->n_cblk;
  st.node_blocks = c->n_nblk;
  st.domain_events = c->hscal.domain_count;
  {
    const int elem = c->tangent_precision == MPL_F32 ? 4 : 8;
    const int32_t nfact = c->tan_factored ? c->hscal.n_tan_cells : (c->tan_mixed ? c->hscal.n_fact_cells : 0);
    st.tangent_entries = c->tan_factored ? MPL_TAN_FACT_READ : MPL_TAN_DENSE;
    st.tangent_cells = c->hscal.n_tan_cells;
    st.factored_cells = nfact;
    st.hv_model_bytes = (double)elem * (MPL_TAN_FACT_READ * (double)nfact +
                                        MPL_TAN_DENSE * (double)(c->hscal.n_tan_cells - nfact)) +
                        6.0 * elem * c->hscal.n_active_nodes;
  }
  st.ms_unload = t1 - t0;
  st.ms_reconstruct = t2 - t1;
  st.ms_newton = t3 - t2;
  st.ms_load = t4 - t3;
  if (stats) *stats = st;
  return MPL_OK;
}

mpl_status mpl_export_field(mpl_ctx* c, int32_t field, double* dense) {
  if (!c || !dense) return MPL_ERR_INVALID_ARG;
  if (!c->unloaded) return mpl_fail(c, MPL_ERR_STATE, "export before unload");
  const int nx = c->dims[0], ny = c->dims[1], nz = c->dims[2];
  const int64_t ncd = (int64_t)nx * ny * nz;
  const int64_t ncell = (int64_t)c->ncell_alloc(), nnode = (int64_t)c->nnode_alloc();
  const int K = c->nmat;
  const int4* cc = P<int4>(c->ccoord);
  auto zero = [&](int64_t count) {
    return mpl_hip_check(c, hipMemsetAsync(dense, 0, sizeof(double) * count, c->stream), "memset");
  };
  switch (field) {
    case MPL_FIELD_MASS_C:
      MPL_TRY(zero(ncd));
      MPL_LAUNCH(c, k_export_cells<double>, c->n_cblk, 64, P<double>(c->mc), 1, ncell, cc, c->n_cblk,
                 nx, ny, nz, dense, 1, 0, (int64_t)0);
      break;
    case MPL_FIELD_VEL_C:
      MPL_TRY(zero(3 * ncd));
      MPL_LAUNCH(c, k_export_cells<double>, c->n_cblk, 64, P<double>(c->qc), 3, ncell, cc, c->n_cblk,
                 nx, ny, nz, dense, 3, 0, (int64_t)0);
      break;
    case MPL_FIELD_GRAD_C:
      MPL_TRY(zero(9 * ncd));
      MPL_LAUNCH(c, k_export_cells<double>, c->n_cblk, 64, P<double>(c->Gc), 9, ncell, cc, c->n_cblk,
                 nx, ny, nz, dense, 9, 0, (int64_t)0);
      break;
    case MPL_FIELD_VOL_CK:
      MPL_TRY(zero(K * ncd));
      for (int k = 0; k < K; ++k)
        MPL_LAUNCH(c, k_export_cells<double>, c->n_cblk, 64, P<double>(c->Vk) + k * ncell, 1, ncell,
                   cc, c->n_cblk, nx, ny, nz, dense, 1, 0, (int64_t)k * ncd);
      break;
    case MPL_FIELD_TAU_CK:
      MPL_TRY(zero(9 * K * ncd));
      MPL_LAUNCH(c, k_export_sym, c->n_cblk, 64, P<double>(c->Tk), ncell, K, cc, c->n_cblk, nx, ny,
                 nz, dense);
      break;
    case MPL_FIELD_S_CK:
      if (!c->reconstructed) return mpl_fail(c, MPL_ERR_STATE, "S before reconstruction");
      MPL_TRY(zero(9 * K * ncd));
      MPL_LAUNCH(c, k_export_sym, c->n_cblk, 64, P<double>(c->Sk), ncell, K, cc, c->n_cblk, nx, ny,
                 nz, dense);
      break;
    case MPL_FIELD_ABAR:
      if (!c->tangent_built) return mpl_fail(c, MPL_ERR_STATE, "tangent not built");
      MPL_TRY(zero(81 * ncd));
      if (c->tangent_precision == MPL_F32 && (c->tan_factored || c->tan_mixed))
        MPL_LAUNCH(c, k_export_abar_fact, c->n_cblk, 64, P<float>(c->Abar32), P<uint64_t>(c->cmask),
                   P<int32_t>(c->coff), cc, c->n_cblk, nx, ny, nz, dense,
                   c->tan_mixed ? (const uint8_t*)P<uint8_t>(c->cfmt) : (const uint8_t*)nullptr);
      else if (c->tangent_precision == MPL_F32)
        MPL_LAUNCH(c, k_export_abar32, c->n_cblk, 64, P<float>(c->Abar32), P<uint64_t>(c->cmask),
                   P<int32_t>(c->coff), cc, c->n_cblk, nx, ny, nz, dense);
      else
        MPL_LAUNCH(c, k_export_abar64, c->n_cblk, 64, P<double>(c->Abar64), P<uint64_t>(c->cmask),
                   P<int32_t>(c->coff), cc, c->n_cblk, nx, ny, nz, dense);
      break;
    case MPL_FIELD_MASS_I:
      MPL_TRY(mpl_block_to_dense_nodes(c, c->mi.p, dense, 1, 0));
      break;
    case MPL_FIELD_VEL_I:
      MPL_TRY(mpl_block_to_dense_nodes(c, c->vn.p, dense, 3, 0));
      break;
    case MPL_FIELD_VHAT:
      MPL_TRY(mpl_block_to_dense_nodes(c, c->vhat.p, dense, 3, 0));
      break;
    case MPL_FIELD_V:
      MPL_TRY(mpl_block_to_dense_nodes(c, c->v.p, dense, 3, 0));
      break;
    case MPL_FIELD_FIXED: {
      MPL_TRY(mpl_ensure(c, c->dense_tmp64, 8 * nnode));
      MPL_LAUNCH(c, k_flags_to_double, (int)((nnode + 255) / 256), 256, P<uint8_t>(c->flags),
                 P<double>(c->dense_tmp64), nnode);
      MPL_TRY(mpl_block_to_dense_nodes(c, c->dense_tmp64.p, dense, 1, 0));
      break;
    }
    case MPL_FIELD_DIAG:
      if (!c->tangent_built) return mpl_fail(c, MPL_ERR_STATE, "tangent not built");
      MPL_TRY(mpl_block_to_dense_nodes(c, c->D.p, dense, 3, 0));
      break;
    case MPL_FIELD_BLOCK_DIAG:
      if (!c->tangent_built || !c->bj_built)
        return mpl_fail(c, MPL_ERR_STATE, "block-Jacobi blocks not built (tangent with precond = block-Jacobi)");
      MPL_TRY(mpl_ensure(c, c->dense_tmp64, 8 * 9 * nnode));
      MPL_LAUNCH(c, k_sym6_to_9, (int)((nnode + 255) / 256), 256, P<double>(c->Bj), P<double>(c->dense_tmp64),
                 nnode);
      MPL_TRY(mpl_block_to_dense_nodes(c, c->dense_tmp64.p, dense, 9, 0));
      break;
    default:
      return mpl_fail(c, MPL_ERR_INVALID_ARG, "unknown field");
  }
  MPL_HIP(c, hipStreamSynchronize(c->stream));
  return MPL_OK;
}

}  // extern "C"
