// Integrate, explicit branch (the explicit case of the Integrate algorithm;
// Sec. 4 opening, Eq. explicitforce):
//   f_i = -sum_c sum_k V_{c,k} tau_{c,k} grad w_ic,
//   v_i^{n+1} = vhat_i + dt f_i / m_i    (vhat_i = v_i^n + dt gravity)
// on free nodes, the prescribed velocity on Dirichlet nodes and zero on
// massless nodes.  The per-centre volumes and Kirchhoff stresses are the
// unload's; there is no stretch reconstruction and no solve.
//
// One wavefront per 4x4x4 node block, one lane per node: the lane gathers
// its 8 surrounding centres in a fixed corner order (no atomics, the same
// result on every run).  A centre's V and tau are read by its 8 corner
// nodes, which sit in at most 8 node blocks; the XCD-major block mapping
// keeps those blocks on one XCD so the re-reads are served by its L2.  The
// kernel runs once per step and moves 7K doubles per centre and 57 bytes
// per node.
#include <chrono>

#include "mpl_grid.h"

using namespace mpl;

namespace {

__global__ __launch_bounds__(64) void k_explicit_nodes(const double* __restrict__ Vk,
                                                       const double* __restrict__ Tk, int64_t ncell,
                                                       int K, const int* __restrict__ n_nbr_cell,
                                                       int n_nblk, const double* __restrict__ mi,
                                                       const uint8_t* __restrict__ flags,
                                                       const double* __restrict__ vhat, int64_t nnode,
                                                       double dt, double inv4dx,
                                                       double* __restrict__ v, double* __restrict__ f) {
  const int nb = xcd_block(blockIdx.x, n_nblk), l = threadIdx.x;
  if (nb >= n_nblk) return;
  const int64_t ni = (int64_t)nb * MPL_BC + l;
  const uint8_t fl = flags[ni];
  double fr[3] = {0.0, 0.0, 0.0};
  if (fl & MPL_NODE_ACTIVE) {
    int cis[8];
    bool ok[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) {
      const int cv = node_cell(n_nbr_cell, nb, l, d);
      ok[d] = cv >= 0;
      cis[d] = ok[d] ? cv : 0;
    }
    for (int k = 0; k < K; ++k) {
      // corners in a fixed order, two batches of four whose loads are all
      // issued before any is used; an absent centre reads centre 0 and an
      // empty one its own zeros, both with V = 0, which subtracts exact zeros
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        double V[4], T[4][6];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t ci = cis[4 * h + j];
          V[j] = Vk[k * ncell + ci];
          // symmetric tau stored as (xx, yy, zz, xy, yz, xz)
#pragma unroll
          for (int e = 0; e < 6; ++e) T[j][e] = Tk[((int64_t)k * 6 + e) * ncell + ci];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int d = 4 * h + j;
          const double Vc = ok[d] ? V[j] : 0.0;
          double gw[3];
          corner_grad(d, inv4dx, gw);
          fr[0] -= Vc * (T[j][0] * gw[0] + T[j][3] * gw[1] + T[j][5] * gw[2]);
          fr[1] -= Vc * (T[j][3] * gw[0] + T[j][1] * gw[1] + T[j][4] * gw[2]);
          fr[2] -= Vc * (T[j][5] * gw[0] + T[j][4] * gw[1] + T[j][2] * gw[2]);
        }
      }
    }
  }
  const double m = mi[ni];
  for (int a = 0; a < 3; ++a) {
    const int64_t i = a * nnode + ni;
    const double vh = vhat[i];
    v[i] = mpl_free(fl, a) ? vh + dt * fr[a] / m : vh;
    if (f) f[i] = fr[a];
  }
}

double wall_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

mpl_status stage_explicit(mpl_ctx* c, bool want_force) {
  if (!c->unloaded) return mpl_fail(c, MPL_ERR_STATE, "explicit integration before unload");
  const int64_t ncell = (int64_t)c->ncell_alloc(), nnode = (int64_t)c->nnode_alloc();
  if (want_force) MPL_TRY(mpl_ensure(c, c->g, 8 * 3 * nnode));
  MPL_LAUNCH(c, k_explicit_nodes, xcd_grid(c->n_nblk), 64, P<double>(c->Vk), P<double>(c->Tk), ncell,
             c->nmat, P<int>(c->n_nbr_cell), c->n_nblk, P<double>(c->mi), P<uint8_t>(c->flags), P<double>(c->vhat), nnode,
             c->dt, 0.25 * c->inv_dx, P<double>(c->v), want_force ? P<double>(c->g) : nullptr);
  // the explicit velocity takes the place of a Newton solution: mpl_load
  // with v = NULL moves the particles with it
  c->solved = true;
  return MPL_OK;
}

}  // namespace

extern "C" {

mpl_status mpl_integrate_explicit(mpl_ctx* c, double* v_out, double* f_out) {
  if (!c) return MPL_ERR_INVALID_ARG;
  MPL_TRY(stage_explicit(c, f_out != nullptr));
  if (v_out) MPL_TRY(mpl_block_to_dense_nodes(c, c->v.p, v_out, 3, 0));
  if (f_out) MPL_TRY(mpl_block_to_dense_nodes(c, c->g.p, f_out, 3, 0));
  return MPL_OK;
}

mpl_status mpl_step_explicit(mpl_ctx* c, const mpl_particles* in, mpl_particles* out, double dt,
                             const double gravity[3], const mpl_bc* bcs, int32_t n_bcs, double time,
                             mpl_stats* stats) {
  if (!c || !in || !out) return MPL_ERR_INVALID_ARG;
  if (out->dtype != in->dtype) return mpl_fail(c, MPL_ERR_INVALID_ARG, "in and out particle dtypes differ");
  mpl_stats st{};
  const double t0 = wall_ms();
  Parts64 pin, pout;
  MPL_TRY(mpl_particles_in(c, in, &pin));
  if (in->dtype == MPL_F32) pout = pin;
  else MPL_TRY(mpl_particles_in(c, out, &pout));
  MPL_TRY(mpl_stage_unload(c, &pin, dt, gravity, bcs, n_bcs, time));
  const double t1 = wall_ms();
  MPL_TRY(stage_explicit(c, false));
  const double t2 = wall_ms();
  MPL_TRY(mpl_stage_load(c, P<double>(c->v), &pin, &pout, dt));
  if (in->dtype == MPL_F32) MPL_TRY(mpl_particles_out(c, &pout, out));
  const double t3 = wall_ms();
  st.active_cells = c->hscal.n_active_cells;
  st.active_nodes = c->hscal.n_active_nodes;
  st.free_dofs = c->hscal.n_free_dofs;
  st.cell_blocks = c->n_cblk;
  st.node_blocks = c->n_nblk;
  st.ms_unload = t1 - t0;
  st.ms_newton = t2 - t1;
  st.ms_load = t3 - t2;
  if (stats) *stats = st;
  return MPL_OK;
}

}  // extern "C"
