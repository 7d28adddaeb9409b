// Integrate, implicit branch (Alg. 3; Sec. 4.2-4.3): stretch reconstruction,
// incremental potential, projected tangent, matrix-free Hessian-vector
// product, Jacobi-PCG and the Newton / line-search driver.
//
// Precision policy: stretch reconstruction, energy, gradient, SVD/polar and
// every dot product / norm are FP64; the stored per-cell tangent and the
// Hessian-vector product run in FP32 (MPL_F32) or FP64 (MPL_F64, parity).
// CG keeps x and r in FP64, the search direction p and Hp in the Hv precision.
//
// Hessian-vector product (the hot loop): one fused pass per 4x4x4 cell block
// (see k_hv_fused) with coalesced component-major loads of the 45 stored
// tangent entries; the CG update kernel assembles the node result.
#include <cmath>
#include <chrono>
#include <functional>

#include "mpl_grid.h"
#include "mpl_nn.h"

using namespace mpl;

namespace {



// G_c(v) = sum over the 8 corners of v_i (x) grad w_ic (Sec. 3.3).
template <class T>
__device__ __forceinline__ void cell_grad(const T* __restrict__ v, int64_t nnode,
                                          const int* __restrict__ c_nbr_node, int cb, int l,
                                          double inv4dx, double* Gm) {
#pragma unroll
  for (int e = 0; e < 9; ++e) Gm[e] = 0.0;
#pragma unroll
  for (int d = 0; d < 8; ++d) {
    const int ni = corner_node(c_nbr_node, cb, l, d);
    double gw[3];
    corner_grad(d, inv4dx, gw);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double va = (double)v[a * nnode + ni];
      Gm[a * 3 + 0] += va * gw[0];
      Gm[a * 3 + 1] += va * gw[1];
      Gm[a * 3 + 2] += va * gw[2];
    }
  }
}

__global__ __launch_bounds__(128) void k_reconstruct(const double* __restrict__ Vk, const double* __restrict__ Tk,
                                                     double* __restrict__ Sk, int64_t ncell, int K,
                              int32_t* __restrict__ domain_count,
    const MatParams* __restrict__ mats) {
  int64_t ci = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ci >= ncell) return;
  for (int k = 0; k < K; ++k) {
    double S6[6] = {1.0, 1.0, 1.0, 0.0, 0.0, 0.0};
    if (Vk[k * ncell + ci] != 0.0) {
      double t6[6], T[9], w[3], Q[9], s[3];
      for (int j = 0; j < 6; ++j) t6[j] = Tk[(k * 6 + j) * ncell + ci];
      sym_to_full(t6, T);
      eig_sym3(T, w, Q);
      if (stretch_from_principal(mats[k], w, s)) atomicAdd(domain_count, 1);
      double S[9];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          S[i * 3 + j] = Q[i * 3] * s[0] * Q[j * 3] + Q[i * 3 + 1] * s[1] * Q[j * 3 + 1] +
                         Q[i * 3 + 2] * s[2] * Q[j * 3 + 2];
      full_to_sym(S, S6);
    }
    for (int j = 0; j < 6; ++j) Sk[(k * 6 + j) * ncell + ci] = S6[j];
  }
}

// Energy per cell sum_k V psi_k((I + dt G) S_k) and, with want_grad, the
// stress content Q_c = sum_k V P_k(F_k) S_k^T.
template <bool WANT_GRAD>
__global__ __launch_bounds__(64) void k_energy_cells(const double* __restrict__ v, int64_t nnode,
                                                     const int* __restrict__ c_nbr_node,
                                                     const double* __restrict__ Vk,
                                                     const double* __restrict__ Sk,
                                                     const double* __restrict__ Sg, int64_t ncell,
                                                     int K, double dt, double inv4dx,
                                                     double* __restrict__ Qc,
                                                     double* __restrict__ partial,
    const MatParams* __restrict__ mats) {
  const int cb = blockIdx.x, l = threadIdx.x;
  const int64_t ci = (int64_t)cb * MPL_BC + l;
  double e = 0.0, Q[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  bool any = false;
  for (int k = 0; k < K; ++k) any = any || (Vk[k * ncell + ci] != 0.0);
  if (any) {
    double Gm[9];
    cell_grad(v, nnode, c_nbr_node, cb, l, inv4dx, Gm);
    double A[9];
    for (int i = 0; i < 9; ++i) A[i] = dt * Gm[i];
    A[0] += 1.0; A[4] += 1.0; A[8] += 1.0;
    for (int k = 0; k < K; ++k) {
      const double V = Vk[k * ncell + ci];
      if (V == 0.0) continue;
      double S6[6], S[9], F[9];
      if (Sg) {  // general base (fixed-point plasticity), 9 entries
        for (int e = 0; e < 9; ++e) S[e] = Sg[(k * 9 + e) * ncell + ci];
      } else {
        for (int j = 0; j < 6; ++j) S6[j] = Sk[(k * 6 + j) * ncell + ci];
        sym_to_full(S6, S);
      }
      mul(A, S, F);
      const double ps = psi(mats[k], F);
      e += V * ps;
      if (WANT_GRAD && isfinite(ps)) {
        double Pm[9], PS[9];
        piola(mats[k], F, Pm);
        mul_nt(Pm, S, PS);  // P S^T (S need not be symmetric)
        for (int i = 0; i < 9; ++i) Q[i] += V * PS[i];
      }
    }
  }
  if (WANT_GRAD)
    for (int i = 0; i < 9; ++i) Qc[i * ncell + ci] = Q[i];
  const double s = wave_sum(e);
  if (l == 0) partial[cb] = s;
}

// Fixed-point plasticity base (Sec. 7, Fixed-Point Plasticity): for every
// centre and material with plasticity, the trial F = (I + dt G_c(v)) S is
// return-mapped (the particles' projection) to F_E and the base becomes
// (I + dt G_c(v))^{-1} F_E; where nothing yields, and for materials without
// plasticity, the reconstructed S itself (9 entries per centre and material).
__global__ __launch_bounds__(64) void k_plastic_base(const double* __restrict__ v, int64_t nnode,
                                                     const int* __restrict__ c_nbr_node,
                                                     const double* __restrict__ Vk,
                                                     const double* __restrict__ Sk, int64_t ncell,
                                                     int K, double dt, double inv4dx,
                                                     double* __restrict__ Seff,
                                                     int32_t* __restrict__ err,
    const MatParams* __restrict__ mats) {
  const int cb = blockIdx.x, l = threadIdx.x;
  const int64_t ci = (int64_t)cb * MPL_BC + l;
  bool need = false;
  for (int k = 0; k < K; ++k)
    need = need || (Vk[k * ncell + ci] != 0.0 && mats[k].plastic != PLASTIC_NONE);
  double A[9], Ai[9];
  if (need) {
    double Gm[9];
    cell_grad(v, nnode, c_nbr_node, cb, l, inv4dx, Gm);
    for (int i = 0; i < 9; ++i) A[i] = dt * Gm[i];
    A[0] += 1.0; A[4] += 1.0; A[8] += 1.0;
    double C[9];
    cofactor(A, C);  // C = det(A) A^{-T}
    const double d = det(A);
    if (!(d != 0.0) || !isfinite(d)) {
      need = false;
      atomicOr(err, 8);
    } else {
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Ai[i * 3 + j] = C[j * 3 + i] / d;
    }
  }
  for (int k = 0; k < K; ++k) {
    double S6[6], S[9];
    for (int j = 0; j < 6; ++j) S6[j] = Sk[(k * 6 + j) * ncell + ci];
    sym_to_full(S6, S);
    double Se[9];
    for (int e = 0; e < 9; ++e) Se[e] = S[e];
    if (need && Vk[k * ncell + ci] != 0.0 && mats[k].plastic != PLASTIC_NONE) {
      double F[9];
      mul(A, S, F);
      if (plastic_project(mats[k], F) > 0.0) mul(Ai, F, Se);
    }
    for (int e = 0; e < 9; ++e) Seff[(k * 9 + e) * ncell + ci] = Se[e];
  }
}

// grad_i = m_i (v_i - vhat_i) + dt sum_c Q_c grad w_ic on the free components
// (0 on the fixed ones); partial sums of the inertia energy (free components)
// and |grad|^2.
template <bool WANT_GRAD>
__global__ __launch_bounds__(64) void k_energy_nodes(const double* __restrict__ v,
                                                     const double* __restrict__ vhat,
                                                     const double* __restrict__ mi,
                                                     const uint8_t* __restrict__ flags,
                                                     const int* __restrict__ n_nbr_cell,
                                                     const double* __restrict__ Qc, int64_t ncell,
                                                     int64_t nnode, double dt, double inv4dx,
                                                     double* __restrict__ g,
                                                     double* __restrict__ pe,
                                                     double* __restrict__ pg) {
  const int nb = blockIdx.x, l = threadIdx.x;
  const int64_t ni = (int64_t)nb * MPL_BC + l;
  const uint8_t fl = flags[ni];
  const bool fr = (fl & MPL_NODE_FREE_ALL) != 0;
  const double m = mi[ni];
  double ein = 0.0, gg = 0.0, gr[3] = {0.0, 0.0, 0.0};
  if (fr) {
    // kinetic term and gradient on the free components only
    double dv[3];
    for (int a = 0; a < 3; ++a) dv[a] = mpl_free(fl, a) ? v[a * nnode + ni] - vhat[a * nnode + ni] : 0.0;
    ein = 0.5 * m * (dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    if (WANT_GRAD) {
      for (int d = 0; d < 8; ++d) {
        const int ci = node_cell(n_nbr_cell, nb, l, d);
        if (ci < 0) continue;
        double gw[3];
        corner_grad(d, inv4dx, gw);
        for (int a = 0; a < 3; ++a)
          gr[a] += Qc[(a * 3) * ncell + ci] * gw[0] + Qc[(a * 3 + 1) * ncell + ci] * gw[1] +
                   Qc[(a * 3 + 2) * ncell + ci] * gw[2];
      }
      for (int a = 0; a < 3; ++a) gr[a] = mpl_free(fl, a) ? m * dv[a] + dt * gr[a] : 0.0;
      gg = gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2];
    }
  }
  if (WANT_GRAD)
    for (int a = 0; a < 3; ++a) g[a * nnode + ni] = gr[a];
  const double se = wave_sum(ein), sg = wave_sum(gg);
  if (l == 0) {
    pe[nb] = se;
    if (WANT_GRAD) pg[nb] = sg;
  }
}

// Deterministic reduction of up to 3 partial arrays (fixed order) into
// scalars, followed by the solver's scalar logic.
enum {
  RED_PLAIN = 0,
  RED_ALPHA = 1,
  RED_BETA = 2,
  RED_PCG_INIT = 3,
  RED_FINIT = 4,   // flexible CG: A = b.b, B = sum Dinv b^2
  RED_FCHECK = 5,  // flexible CG: A = r.r, B = sum Dinv r^2 (convergence, stagnation)
  RED_FBETA = 6,   // flexible CG: A = z.r, B = z.q (Polak-Ribiere beta or fallback)
  RED_FINIT_WARM = 7  // flexible CG from x0: A = b.b, B = sum Dinv r^2, C = r.r
};
template <int MODE>
__global__ __launch_bounds__(1024) void k_reduce(const double* __restrict__ a, int na,
                                                 const double* __restrict__ b, int nb,
                                                 const double* __restrict__ c, int nc,
                                                 SolverScalars* __restrict__ s, int slot) {
  __shared__ double sh[3][16];
  const int t = threadIdx.x;
  if ((MODE == RED_ALPHA || MODE == RED_BETA || MODE == RED_FCHECK || MODE == RED_FBETA) &&
      done_flag(s))
    return;
  // every thread issues all its loads (up to 8 per array) before using any,
  // so arrays of up to 8192 partials cost one memory round trip
  double va[8], vb[8], vc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int i = t + 1024 * k;
    va[k] = i < na ? a[i] : 0.0;
    vb[k] = i < nb ? b[i] : 0.0;
    vc[k] = i < nc ? c[i] : 0.0;
  }
  for (int i = t + 8192; i < na; i += 1024) va[0] += a[i];
  for (int i = t + 8192; i < nb; i += 1024) vb[0] += b[i];
  for (int i = t + 8192; i < nc; i += 1024) vc[0] += c[i];
#pragma unroll
  for (int k = 1; k < 8; ++k) {
    va[0] += va[k];
    vb[0] += vb[k];
    vc[0] += vc[k];
  }
  const double ra = wave_sum(va[0]);
  const double rb = wave_sum(vb[0]);
  const double rc = wave_sum(vc[0]);
  if ((t & 63) == 0) {
    sh[0][t >> 6] = ra;
    sh[1][t >> 6] = rb;
    sh[2][t >> 6] = rc;
  }
  __syncthreads();
  if (t != 0) return;
  double A = 0.0, B = 0.0, C = 0.0;
  for (int w = 0; w < 16; ++w) {
    A += sh[0][w];
    B += sh[1][w];
    C += sh[2][w];
  }
  if (MODE == RED_PLAIN) {
    s->red[slot] = A;
    s->red[slot + 1] = B;
    s->red[slot + 2] = C;
  } else if (MODE == RED_PCG_INIT) {  // A = r.z, B = b.b
    s->rz = A;
    s->bnorm2 = B;
    s->iters = 0;
    s->done = (B == 0.0) ? 1 : 0;
  } else if (MODE == RED_ALPHA) {  // A = p^T K p (cells), B = p^T M p (nodes)
    const double pq = A + B;
    s->pq = pq;
    if (!(pq > 0.0) || !isfinite(pq)) {
      s->done = 2;
      s->nn_off = 1;
      s->alpha = 0.0;
    } else {
      s->alpha = s->rz / pq;
    }
  } else if (MODE == RED_BETA) {  // A = r.z (new), B = r.r
    s->rz_new = A;
    s->rr = B;
    s->iters += 1;
    if (!isfinite(B)) s->done = 2;
    else if (B <= s->tol2) s->done = 1;
    s->beta = A / s->rz;
    s->rz = A;
  } else if (MODE == RED_FINIT) {
    s->bnorm2 = A;
    s->rr = A;
    s->rr_mark = A;
    s->s2 = B;
    s->iters = 0;
    s->done = (A == 0.0) ? 1 : 0;
    s->fallback = 0;
    s->fb_new = 0;
    s->fallbacks = 0;
    s->nn_off = s->done;
  } else if (MODE == RED_FINIT_WARM) {
    // the tolerance stays relative to |b|; stagnation is judged on |r|
    s->bnorm2 = A;
    s->rr = C;
    s->rr_mark = C;
    s->s2 = B;
    s->iters = 0;
    s->done = (A == 0.0 || C == 0.0) ? 1 : 0;
    s->fallback = 0;
    s->fb_new = 0;
    s->fallbacks = 0;
    s->nn_off = s->done;
  } else if (MODE == RED_FCHECK) {
    s->rr = A;
    s->s2 = B;
    s->iters += 1;
    if (!isfinite(A)) s->done = 2;
    else if (A <= s->tol2) s->done = 1;
    // stagnation: less than 10% drop of |r| over the last 10 iterations
    if (s->done == 0 && s->fallback == 0 && s->iters % 10 == 0) {
      if (A > 0.81 * s->rr_mark) {
        s->fallback = 1;
        s->fb_new = 1;
        s->fallbacks += 1;
      }
      s->rr_mark = A;
    }
    s->nn_off = (s->done != 0 || s->fallback != 0) ? 1 : 0;
  } else {  // RED_FBETA
    if (s->fallback) {
      // Jacobi from here on: z = Dinv r, z.r = s2; restart on the switch
      s->beta = s->fb_new ? 0.0 : s->s2 / s->rz;
      s->rz = s->s2;
      s->fb_new = 0;
    } else if (!(A > 0.0) || !isfinite(A) || !isfinite(B)) {
      // the network output is not a descent direction: switch to Jacobi
      s->fallback = 1;
      s->fallbacks += 1;
      s->nn_off = 1;
      s->beta = 0.0;
      s->rz = s->s2;
    } else {
      // flexible (Polak-Ribiere) beta = z_new.(r_new - r_old) / z_old.r_old
      // with r_new - r_old = -alpha q
      s->beta = (s->iters == 0) ? 0.0 : -s->alpha * B / s->rz;
      s->rz = A;
    }
  }
}

__global__ void k_set_tol(SolverScalars* s, double rtol2) { s->tol2 = rtol2 * s->bnorm2; }

// Per-cell projected tangent (Sec. 4.2 Hessian; projection per material):
//   Abar_c = dt^2 sum_k V_k sum_modes max(lam, 0) vec(E S_k) vec(E S_k)^T
// with the analytic eigen-modes E of dP/dF at F_k = (I + dt G_c) S_k.
// FACT (single material, FP32): the modes are E = U e V^T with e diagonal
// (scaling) or a twist/flip pair, so vec(E S) = vec(U e M^T) with M = S V,
// and the cell stores U, M, the projected scaling block and the pair
// coefficients (the layout before MPL_TAN_FACT) instead of the 45 entries.
template <class T, bool FACT, bool MIX>
__global__ __launch_bounds__(64) void k_tangent(const double* __restrict__ v, int64_t nnode,
                                                const int* __restrict__ c_nbr_node,
                                                const double* __restrict__ Vk,
                                                const double* __restrict__ Sk,
                                                const double* __restrict__ Sg, int64_t ncell,
                                                int K, double dt, double inv4dx,
                                                const uint64_t* __restrict__ cmask,
                                                const int32_t* __restrict__ coff,
                                                T* __restrict__ Abar, int32_t* __restrict__ err,
    const MatParams* __restrict__ mats, T* __restrict__ Aoff, const uint8_t* __restrict__ cfmt) {
  const int cb = blockIdx.x, l = threadIdx.x;
  const int64_t ci = (int64_t)cb * MPL_BC + l;
  // factored layout for this block: always (FACT), per block (MIX: blocks
  // whose cells hold at most one material each), or never
  const bool fb = FACT || (MIX && cfmt[cb] != 0);
  const TanSlot ts = tan_slot(cmask, coff, cb, l, FACT ? MPL_TAN_FACT : MPL_TAN_DENSE);
  if (!ts.active) return;
  double Ab[45];
#pragma unroll
  for (int i = 0; i < 45; ++i) Ab[i] = 0.0;
  double fac[MPL_TAN_FACT_READ];
#pragma unroll
  for (int i = 0; i < MPL_TAN_FACT_READ; ++i) fac[i] = 0.0;
  fac[0] = 1.0;  // identity rotation where no material is present
  bool any = false;
  for (int k = 0; k < K; ++k) any = any || (Vk[k * ncell + ci] != 0.0);
  if (any) {
    double Gm[9];
    cell_grad(v, nnode, c_nbr_node, cb, l, inv4dx, Gm);
    double A[9];
    for (int i = 0; i < 9; ++i) A[i] = dt * Gm[i];
    A[0] += 1.0; A[4] += 1.0; A[8] += 1.0;
    for (int k = 0; k < K; ++k) {
      const double V = Vk[k * ncell + ci];
      if (V == 0.0) continue;
      double S6[6], S[9], F[9];
      if (Sg) {  // general base (fixed-point plasticity), 9 entries
        for (int e = 0; e < 9; ++e) S[e] = Sg[(k * 9 + e) * ncell + ci];
      } else {
        for (int j = 0; j < 6; ++j) S6[j] = Sk[(k * 6 + j) * ncell + ci];
        sym_to_full(S6, S);
      }
      mul(A, S, F);
      double U[9], s[3], Vm[9], R[9];
      if (!principal_frame(F, U, s, Vm, R)) {
        atomicOr(err, 8);
        continue;
      }
      double dpsi[3], H[3][3], tw[3], fl[3];
      principal_derivs(mats[k], s, dpsi, H, tw, fl);
      const double coef = dt * dt * V;
      // scaling modes: eigenpairs of the 3x3 Hessian of psi_hat
      double Hs[9] = {H[0][0], H[0][1], H[0][2], H[1][0], H[1][1], H[1][2], H[2][0], H[2][1], H[2][2]};
      double w[3], Qm[9];
      eig_sym3(Hs, w, Qm);
      if (fb) {
        double M[9];
        mul(S, Vm, M);
        rot_to_quat(U, fac);
        for (int i = 0; i < 9; ++i) fac[4 + i] = M[i];
        const int sy[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
        for (int e = 0; e < 6; ++e) {
          double acc = 0.0;
          for (int m = 0; m < 3; ++m)
            if (w[m] > 0.0) acc += coef * w[m] * Qm[sy[e][0] * 3 + m] * Qm[sy[e][1] * 3 + m];
          fac[13 + e] = acc;
        }
        for (int pp = 0; pp < 3; ++pp) {
          const double lt = tw[pp] > 0.0 ? tw[pp] : 0.0, lf = fl[pp] > 0.0 ? fl[pp] : 0.0;
          fac[19 + 2 * pp] = 0.5 * coef * (lt + lf);
          fac[20 + 2 * pp] = 0.5 * coef * (lt - lf);
        }
      }
      for (int mode = 0; mode < 9; ++mode) {
        double lam, E[9];
        if (mode < 3) {
          lam = w[mode];
          if (!(lam > 0.0)) continue;
          // E = U diag(q) V^T
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
              E[i * 3 + j] = U[i * 3] * Qm[mode] * Vm[j * 3] + U[i * 3 + 1] * Qm[3 + mode] * Vm[j * 3 + 1] +
                             U[i * 3 + 2] * Qm[6 + mode] * Vm[j * 3 + 2];
        } else {
          const int p = (mode - 3) >> 1, sign = ((mode - 3) & 1) ? -1 : 1;
          const int pi = (p == 1) ? 1 : 0, pj = (p == 0) ? 1 : 2;
          lam = (sign > 0) ? tw[p] : fl[p];
          if (!(lam > 0.0)) continue;
          // E = (u_i v_j^T +- u_j v_i^T)/sqrt 2
          const double r2 = 0.70710678118654752440;
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
              E[i * 3 + j] = r2 * (U[i * 3 + pi] * Vm[j * 3 + pj] + sign * U[i * 3 + pj] * Vm[j * 3 + pi]);
        }
        double W[9];
        mul(E, S, W);  // vec(E S) is the mode seen in velocity-gradient space
        const double cl = coef * lam;
#pragma unroll
        for (int r = 0; r < 9; ++r) {
          const double wr = cl * W[r];
#pragma unroll
          for (int cc = r; cc < 9; ++cc) Ab[sym9(r, cc)] += wr * W[cc];
        }
      }
    }
  }
  if (fb) {
#pragma unroll
    for (int i = 0; i < MPL_TAN_FACT_READ; ++i) Abar[ts.base + (int64_t)i * ts.n + ts.rank] = (T)fac[i];
    // node-block contributions Q_e(s) = sum_{b,b'} Abar[(a,b),(a',b')]
    // sig_b sig_b' / (4 dx)^2 for the entries e = (a, a') of the 3x3 block
    // (xx, yy, zz, xy, yz, xz; the first three are the Jacobi diagonal, the
    // others are written to Aoff when it is given) and the corner signs
    // sig = (+1, sy, sz), s = 2 (sy < 0) + (sz < 0) (a corner and its
    // opposite share the value)
    const double g2 = inv4dx * inv4dx;
    // (fully unrolled: the entry indices into Ab must be compile-time
    // constants, or Ab leaves registers for scratch memory)
    const TanSlot to = tan_slot(cmask, coff, cb, l, MPL_TAN_OFF);
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      if (e >= 3 && !Aoff) break;
      const int a = e < 3 ? e : (e == 5 ? 0 : e - 3), a2 = e < 3 ? e : (e == 5 ? 2 : e - 2);
#pragma unroll
      for (int sidx = 0; sidx < 4; ++sidx) {
        const double sg[3] = {1.0, (sidx & 2) ? -1.0 : 1.0, (sidx & 1) ? -1.0 : 1.0};
        double q = 0.0;
        for (int b = 0; b < 3; ++b)
          for (int b2 = 0; b2 < 3; ++b2) q += Ab[sym9(a * 3 + b, a2 * 3 + b2)] * sg[b] * sg[b2];
        if (e < 3)
          Abar[ts.base + (int64_t)(MPL_TAN_FACT_READ + e * 4 + sidx) * ts.n + ts.rank] = (T)(q * g2);
        else
          Aoff[to.base + (int64_t)((e - 3) * 4 + sidx) * to.n + to.rank] = (T)(q * g2);
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < 45; ++i) Abar[ts.base + (int64_t)i * ts.n + ts.rank] = (T)Ab[i];
  }
}

// Inverse Jacobi diagonal of H at every node, 1 / (m_i + sum_c sum_{b,b'}
// Abar[(a,b),(a,b')] gw_b gw_b'), and 0 on fixed / massless nodes.
template <class T, bool FACT, bool MIX>
__global__ __launch_bounds__(64) void k_diag(const T* __restrict__ Abar,
                                             const uint64_t* __restrict__ cmask,
                                             const int32_t* __restrict__ coff,
                                             const double* __restrict__ mi,
                                             const uint8_t* __restrict__ flags,
                                             const int* __restrict__ n_nbr_cell, int64_t nnode,
                                             double inv4dx, double* __restrict__ D,
                                             T* __restrict__ Dt, T* __restrict__ mt,
                                             const uint8_t* __restrict__ cfmt) {
  const int nb = blockIdx.x, l = threadIdx.x;
  const int64_t ni = (int64_t)nb * MPL_BC + l;
  double dd[3] = {0.0, 0.0, 0.0};
  const uint8_t fl = flags[ni];
  const bool fr = (fl & MPL_NODE_FREE_ALL) != 0;
  if (fr) {
    for (int d = 0; d < 8; ++d) {
      const int ci = node_cell(n_nbr_cell, nb, l, d);
      if (ci < 0) continue;
      const TanSlot ts = tan_slot(cmask, coff, ci >> 6, ci & 63, FACT ? MPL_TAN_FACT : MPL_TAN_DENSE);
      if (!ts.active) continue;
      if (FACT || (MIX && cfmt[ci >> 6] != 0)) {
        // sign pattern of the node as corner d of that cell, canonical sx = +1
        const int dx = (d >> 2) & 1, dy = (d >> 1) & 1, dz = d & 1;
        const int sy = dx ? (dy ? 0 : 1) : (dy ? 1 : 0), sz = dx ? (dz ? 0 : 1) : (dz ? 1 : 0);
        const int sidx = sy * 2 + sz;
        for (int a = 0; a < 3; ++a)
          dd[a] += (double)Abar[ts.base + (int64_t)(MPL_TAN_FACT_READ + a * 4 + sidx) * ts.n + ts.rank];
        continue;
      }
      double gw[3];
      corner_grad(d, inv4dx, gw);
      for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int b = 0; b < 3; ++b)
          for (int b2 = 0; b2 < 3; ++b2)
            s += (double)Abar[ts.base + (int64_t)sym9(a * 3 + b, a * 3 + b2) * ts.n + ts.rank] * gw[b] *
                 gw[b2];
        dd[a] += s;
      }
    }
    for (int a = 0; a < 3; ++a) dd[a] += mi[ni];
  }
  for (int a = 0; a < 3; ++a) {
    const double di = mpl_free(fl, a) ? 1.0 / dd[a] : 0.0;
    D[a * nnode + ni] = di;
    Dt[a * nnode + ni] = (T)di;
  }
  mt[ni] = (T)mi[ni];
}

// pair index of the symmetric 3x3 block entries (xx, yy, zz, xy, yz, xz)
__host__ __device__ constexpr int blk_a(int e) { return e < 3 ? e : (e == 5 ? 0 : e - 3); }
__host__ __device__ constexpr int blk_b(int e) { return e < 3 ? e : (e == 5 ? 2 : e - 2); }

// 3x3 block-Jacobi preconditioner: at every free node the inverse of its
// diagonal block of H,
//   H_ii[a][a'] = m_i delta_aa' + sum_c sum_{b,b'} Abar[(a,b),(a',b')] gw_b gw_b',
// stored as its six distinct entries (xx, yy, zz, xy, yz, xz) in FP64 (B)
// and in the tangent's precision (Bt); 0 on fixed and massless nodes.  The
// block is m I plus a positive semidefinite sum, so it is invertible
// whenever m > 0; the inverse is the adjugate over the determinant.
template <class T, bool FACT, bool MIX>
__global__ __launch_bounds__(64) void k_block_diag(const T* __restrict__ Abar,
                                                   const uint64_t* __restrict__ cmask,
                                                   const int32_t* __restrict__ coff,
                                                   const double* __restrict__ mi,
                                                   const uint8_t* __restrict__ flags,
                                                   const int* __restrict__ n_nbr_cell, int64_t nnode,
                                                   double inv4dx, double* __restrict__ B,
                                                   T* __restrict__ Bt, const T* __restrict__ Aoff,
                                                   int32_t* __restrict__ err, const uint8_t* __restrict__ cfmt) {
  const int nb = blockIdx.x, l = threadIdx.x;
  const int64_t ni = (int64_t)nb * MPL_BC + l;
  double h[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const uint8_t fl = flags[ni];
  const bool fr = (fl & MPL_NODE_FREE_ALL) != 0;
  if (fr) {
    for (int d = 0; d < 8; ++d) {
      const int ci = node_cell(n_nbr_cell, nb, l, d);
      if (ci < 0) continue;
      const TanSlot ts = tan_slot(cmask, coff, ci >> 6, ci & 63, FACT ? MPL_TAN_FACT : MPL_TAN_DENSE);
      if (!ts.active) continue;
      if (FACT || (MIX && cfmt[ci >> 6] != 0)) {
        const int dx = (d >> 2) & 1, dy = (d >> 1) & 1, dz = d & 1;
        const int sy = dx ? (dy ? 0 : 1) : (dy ? 1 : 0), sz = dx ? (dz ? 0 : 1) : (dz ? 1 : 0);
        const int sidx = sy * 2 + sz;
        const TanSlot to = tan_slot(cmask, coff, ci >> 6, ci & 63, MPL_TAN_OFF);
        for (int e = 0; e < 3; ++e) {
          h[e] += (double)Abar[ts.base + (int64_t)(MPL_TAN_FACT_READ + e * 4 + sidx) * ts.n + ts.rank];
          h[e + 3] += (double)Aoff[to.base + (int64_t)(e * 4 + sidx) * to.n + to.rank];
        }
        continue;
      }
      double gw[3];
      corner_grad(d, inv4dx, gw);
      for (int e = 0; e < 6; ++e) {
        const int a = blk_a(e), a2 = blk_b(e);
        double s = 0.0;
        for (int b = 0; b < 3; ++b)
          for (int b2 = 0; b2 < 3; ++b2)
            s += (double)Abar[ts.base + (int64_t)sym9(a * 3 + b, a2 * 3 + b2) * ts.n + ts.rank] * gw[b] *
                 gw[b2];
        h[e] += s;
      }
    }
    for (int a = 0; a < 3; ++a) h[a] += mi[ni];
    // a node with fixed components takes the block of its free ones: the
    // fixed rows and columns become those of the identity here and 0 in the
    // inverse below
    for (int e = 0; e < 6; ++e) {
      const int a = blk_a(e), a2 = blk_b(e);
      if (!mpl_free(fl, a) || !mpl_free(fl, a2)) h[e] = (a == a2) ? 1.0 : 0.0;
    }
  }
  // a free node's block is m_i I plus PSD cell blocks: positive definite
  // unless a value is not finite; anything else is reported (error bit 128)
  double inv[6];
  const bool ok = sym3_inverse(h, inv);
  if (fr && !ok) atomicOr(err, 128);
  if (!fr || !ok)
    for (int e = 0; e < 6; ++e) inv[e] = 0.0;
  for (int e = 0; e < 6; ++e)
    if (!mpl_free(fl, blk_a(e)) || !mpl_free(fl, blk_b(e))) inv[e] = 0.0;
  for (int e = 0; e < 6; ++e) {
    B[e * nnode + ni] = inv[e];
    Bt[e * nnode + ni] = (T)inv[e];
  }
}

// z = B r with B a symmetric 3x3 block given by its entries (xx, yy, zz, xy,
// yz, xz)
__device__ __forceinline__ void block_apply(const double b[6], const double r[3], double z[3]) {
  z[0] = b[0] * r[0] + b[3] * r[1] + b[5] * r[2];
  z[1] = b[3] * r[0] + b[1] * r[1] + b[4] * r[2];
  z[2] = b[5] * r[0] + b[4] * r[1] + b[2] * r[2];
}

// Vertex block descent (Sec. 5, VBD), one colour: every free node whose index
// parity is `color` takes v_i -= H_ii^{-1} g_i with H_ii = m_i I + sum over its
// cells of the node's 3x3 block of the dense FP64 tangent,
//   H[a][a'] += sum_{b,b'} Abar[(a,b),(a',b')] gw_b gw_b'.
// No two nodes of one colour share a cell, so the updates are independent.
// On a node with fixed components the step is taken on the free ones (their
// rows and columns of H; the gradient is 0 on the fixed ones).
__global__ __launch_bounds__(64) void k_vbd_nodes(const double* __restrict__ Abar,
                                                  const uint64_t* __restrict__ cmask,
                                                  const int32_t* __restrict__ coff,
                                                  const double* __restrict__ mi,
                                                  const uint8_t* __restrict__ flags,
                                                  const int* __restrict__ n_nbr_cell,
                                                  const int4* __restrict__ ncoord, int64_t nnode,
                                                  double inv4dx, int color,
                                                  const double* __restrict__ g,
                                                  double* __restrict__ v, int32_t* __restrict__ err) {
  const int nb = blockIdx.x, l = threadIdx.x;
  const int64_t ni = (int64_t)nb * MPL_BC + l;
  const int4 bc = ncoord[nb];
  const int ix = bc.x * 4 + local_x(l), iy = bc.y * 4 + local_y(l), iz = bc.z * 4 + local_z(l);
  if ((((ix & 1) << 2) | ((iy & 1) << 1) | (iz & 1)) != color) return;
  const uint8_t fl = flags[ni];
  if (!(fl & MPL_NODE_FREE_ALL)) return;
  const double m = mi[ni];
  double H[9] = {m, 0.0, 0.0, 0.0, m, 0.0, 0.0, 0.0, m};
  for (int d = 0; d < 8; ++d) {
    const int ci = node_cell(n_nbr_cell, nb, l, d);
    if (ci < 0) continue;
    const TanSlot ts = tan_slot(cmask, coff, ci >> 6, ci & 63, MPL_TAN_DENSE);
    if (!ts.active) continue;
    double gw[3];
    corner_grad(d, inv4dx, gw);
    for (int a = 0; a < 3; ++a)
      for (int a2 = 0; a2 < 3; ++a2) {
        double s = 0.0;
        for (int b = 0; b < 3; ++b)
          for (int b2 = 0; b2 < 3; ++b2)
            s += Abar[ts.base + (int64_t)sym9(a * 3 + b, a2 * 3 + b2) * ts.n + ts.rank] * gw[b] * gw[b2];
        H[a * 3 + a2] += s;
      }
  }
  for (int a = 0; a < 3; ++a)
    if (!mpl_free(fl, a))
      for (int a2 = 0; a2 < 3; ++a2) H[a * 3 + a2] = H[a2 * 3 + a] = (a == a2) ? 1.0 : 0.0;
  double C[9];
  cofactor(H, C);  // C = det(H) H^{-T}; H is symmetric
  const double dH = det(H);
  if (!(dH > 0.0) || !isfinite(dH)) {
    atomicOr(err, 64);
    return;
  }
  double gi[3];
  for (int a = 0; a < 3; ++a) gi[a] = mpl_free(fl, a) ? g[a * nnode + ni] : 0.0;
  for (int a = 0; a < 3; ++a)
    if (mpl_free(fl, a)) v[a * nnode + ni] -= (C[a] * gi[0] + C[3 + a] * gi[1] + C[6 + a] * gi[2]) / dH;
}

// ---------------------------------------------------------------- Hv
// Fused Hessian-vector product, one wavefront per active cell block:
//   1. stage the 5x5x5 node tile of p (the 2x2x2 corners of all 64 cells) in LDS;
//   2. per cell: dG = sum_d p_{c+d} (x) grad w_d,  y = Abar_c vec(dG),
//      and the cell's share y . vec(dG) of p^T K p;
//   3. put y in LDS; every tile node gathers y_c grad w over its in-block
//      cells in a fixed corner order (race-free, deterministic);
//   4. write the block's own 4x4x4 nodes and its 61 halo nodes (+x/+y/+z
//      faces, which belong to the next node blocks) exactly once.
// The halo pieces are summed into their owner node by the CG update kernel
// (or by k_hv_combine for a stand-alone product), so no node is ever
// written by two workgroups and no atomics are needed.
// Workgroups are mapped XCD-major (xcd_block: consecutive blocks on one XCD)
// so that neighbouring blocks share p tile lines in the same L2.

template <class T, bool DOT, bool FACT, bool MIX>
__global__ __launch_bounds__(256) void k_hv_fused(const T* __restrict__ p, int64_t nnode,
                                                 const int* __restrict__ c_nbr_node,
                                                 const T* __restrict__ Abar,
                                                 const uint64_t* __restrict__ cmask,
                                                 const int32_t* __restrict__ coff, int64_t ncell,
                                                 int n_cblk, T inv4dx, T* __restrict__ Hown,
                                                 T* __restrict__ Hhalo,
                                                 double* __restrict__ partial,
                                                 const SolverScalars* __restrict__ s,
                                                 const uint8_t* __restrict__ cfmt) {
  if (s && done_flag(s)) return;
  // four cell blocks per workgroup, one per wavefront
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int grp = xcd_block(blockIdx.x, (n_cblk + 3) >> 2);
  const int cb = grp * 4 + w;
  const bool valid = cb < n_cblk;
  __shared__ T tp_all[4][3][128];
  __shared__ T ys_all[4][12][64];
  __shared__ double dsum[4];
  T(*tp)[128] = tp_all[w];
  T(*ys)[64] = ys_all[w];
  if (valid) {
    for (int t = l; t < 125; t += 64) {
      const int tx = t / 25, ty = (t / 5) % 5, tz = t % 5;
      const int o = ((tx >> 2) * 2 + (ty >> 2)) * 2 + (tz >> 2);
      const int64_t ni = (int64_t)c_nbr_node[cb * 8 + o] * MPL_BC + local_index(tx & 3, ty & 3, tz & 3);
#pragma unroll
      for (int a = 0; a < 3; ++a) tp[a][t] = p[a * nnode + ni];
    }
  }
  __syncthreads();
  const int64_t ci = (int64_t)cb * MPL_BC + l;
  const int lx = l >> 4, ly = (l >> 2) & 3, lz = l & 3;
  double dot = 0.0;
  if (valid) {
    T g[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) g[e] = T(0);
#pragma unroll
    for (int d = 0; d < 8; ++d) {
      const int dx = (d >> 2) & 1, dy = (d >> 1) & 1, dz = d & 1;
      const int t = ((lx + dx) * 5 + (ly + dy)) * 5 + (lz + dz);
      const T sx = dx ? inv4dx : -inv4dx, sy = dy ? inv4dx : -inv4dx, sz = dz ? inv4dx : -inv4dx;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const T pa = tp[a][t];
        g[a * 3 + 0] += pa * sx;
        g[a * 3 + 1] += pa * sy;
        g[a * 3 + 2] += pa * sz;
      }
    }
    T y[9];
#pragma unroll
    for (int r = 0; r < 9; ++r) y[r] = T(0);
    const TanSlot ts = tan_slot(cmask, coff, cb, l, FACT ? MPL_TAN_FACT : MPL_TAN_DENSE);
    if (ts.active) {
      const T* A = Abar + ts.base + ts.rank;
      // wave-uniform: one cell block per wavefront
      if (FACT || (MIX && cfmt[cb] != 0)) {
        T U[9], M[9], A3[6], pc[6];
        quat_to_rot<T>(A[0], A[ts.n], A[2 * (int64_t)ts.n], A[3 * (int64_t)ts.n], U);
#pragma unroll
        for (int e = 0; e < 9; ++e) M[e] = A[(int64_t)(4 + e) * ts.n];
#pragma unroll
        for (int e = 0; e < 6; ++e) {
          A3[e] = A[(int64_t)(13 + e) * ts.n];
          pc[e] = A[(int64_t)(19 + e) * ts.n];
        }
        // Ghat = U^T g M
        T t1[9], gh[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j)
            t1[i * 3 + j] = U[i] * g[j] + U[3 + i] * g[3 + j] + U[6 + i] * g[6 + j];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j)
            gh[i * 3 + j] = t1[i * 3] * M[j] + t1[i * 3 + 1] * M[3 + j] + t1[i * 3 + 2] * M[6 + j];
        T yh[9];
        yh[0] = A3[0] * gh[0] + A3[1] * gh[4] + A3[2] * gh[8];
        yh[4] = A3[1] * gh[0] + A3[3] * gh[4] + A3[4] * gh[8];
        yh[8] = A3[2] * gh[0] + A3[4] * gh[4] + A3[5] * gh[8];
        // pairs (0,1), (1,2), (0,2)
        yh[1] = pc[0] * gh[1] + pc[1] * gh[3];
        yh[3] = pc[1] * gh[1] + pc[0] * gh[3];
        yh[5] = pc[2] * gh[5] + pc[3] * gh[7];
        yh[7] = pc[3] * gh[5] + pc[2] * gh[7];
        yh[2] = pc[4] * gh[2] + pc[5] * gh[6];
        yh[6] = pc[5] * gh[2] + pc[4] * gh[6];
        // y = U yhat M^T
        T t2[9];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int j = 0; j < 3; ++j)
            t2[a * 3 + j] = U[a * 3] * yh[j] + U[a * 3 + 1] * yh[3 + j] + U[a * 3 + 2] * yh[6 + j];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int b = 0; b < 3; ++b)
            y[a * 3 + b] = t2[a * 3] * M[b * 3] + t2[a * 3 + 1] * M[b * 3 + 1] + t2[a * 3 + 2] * M[b * 3 + 2];
      } else {
#pragma unroll
        for (int r = 0; r < 9; ++r) {
#pragma unroll
          for (int c = r; c < 9; ++c) {
            const T a = A[(int64_t)sym9(r, c) * ts.n];
            y[r] += a * g[c];
            if (c != r) y[c] += a * g[r];
          }
        }
      }
    }
    if (DOT) {
#pragma unroll
      for (int r = 0; r < 9; ++r) dot += (double)y[r] * (double)g[r];
    }
#pragma unroll
    // per component a the four signed sums P_k = y_a0 +- y_a1 +- y_a2 (scaled
    // by 1/(4 dx)): corner sign pattern (sx, sy, sz) contributes
    // sx * P_k with k = 2 (sy != sx) + (sz != sx)
    for (int a = 0; a < 3; ++a) {
      const T y0 = y[a * 3] * inv4dx, y1 = y[a * 3 + 1] * inv4dx, y2 = y[a * 3 + 2] * inv4dx;
      ys[a * 4 + 0][l] = y0 + y1 + y2;
      ys[a * 4 + 1][l] = y0 + y1 - y2;
      ys[a * 4 + 2][l] = y0 - y1 + y2;
      ys[a * 4 + 3][l] = y0 - y1 - y2;
    }
  }
  __syncthreads();
  // Gather: tile node t sums y_c grad w over its in-block cells c = t - d,
  // in corner order d = 0..7 (3 LDS reads per cell).  Round 0: the lane's
  // own node; round 1: halo.
  if (valid) {
    for (int round = 0; round < 2; ++round) {
      int tx, ty, tz;
      if (round == 0) {
        tx = lx; ty = ly; tz = lz;
      } else {
        if (l >= 61) break;
        halo_tile(l, tx, ty, tz);
      }
      T h[3] = {T(0), T(0), T(0)};
#pragma unroll
      for (int d = 0; d < 8; ++d) {
        const int dx = (d >> 2) & 1, dy = (d >> 1) & 1, dz = d & 1;
        const int cx = tx - dx, cy = ty - dy, cz = tz - dz;
        if (cx < 0 || cy < 0 || cz < 0 || cx > 3 || cy > 3 || cz > 3) continue;
        const int cl = local_index(cx, cy, cz);
        const int k = ((dy != dx) << 1) | (dz != dx);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const T v = ys[a * 4 + k][cl];
          h[a] += dx ? v : -v;
        }
      }
      T* out = (round == 0) ? Hown : Hhalo;
#pragma unroll
      for (int a = 0; a < 3; ++a) out[a * ncell + ci] = h[a];
    }
  }
  if (DOT) {
    // one partial per group of four blocks (waves summed in a fixed order)
    const double sdot = wave_sum(dot);
    if (l == 0) dsum[w] = sdot;
    __syncthreads();
    if (threadIdx.x == 0 && grp * 4 < n_cblk) partial[grp] = (dsum[0] + dsum[1]) + (dsum[2] + dsum[3]);
  }
}

// Stand-alone product: Hu = M u + K u on the free components (0 elsewhere).
template <class T>
__global__ __launch_bounds__(64) void k_hv_combine(const T* __restrict__ u,
                                                   const double* __restrict__ mi,
                                                   const uint8_t* __restrict__ flags,
                                                   const int* __restrict__ n_nbr_cell,
                                                   const T* __restrict__ Hown,
                                                   const T* __restrict__ Hhalo, int64_t ncell,
                                                   int64_t nnode, T* __restrict__ Hu) {
  const int nb = blockIdx.x, l = threadIdx.x;
  const int64_t ni = (int64_t)nb * MPL_BC + l;
  const uint8_t fl = flags[ni];
  T h[3];
  gather_kp(Hown, Hhalo, n_nbr_cell, ncell, nb, l, h);
  const T m = (T)mi[ni];
#pragma unroll
  for (int a = 0; a < 3; ++a) Hu[a * nnode + ni] = mpl_free(fl, a) ? h[a] + m * u[a * nnode + ni] : T(0);
}

// ---------------------------------------------------------------- PCG vectors
// Node-vector kernels run 4 node blocks (4 wavefronts) per workgroup and
// emit one partial sum per workgroup (waves combined in a fixed order).
// Dinv holds the inverse Jacobi diagonal (0 on fixed components and
// massless nodes); every vector is 0 on those components.
__device__ __forceinline__ double block4_sum(double v, double* sh) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}

// x = 0, r = b, p = Dinv r; partials r.z, b.b and p^T M p.
template <class T>
__global__ __launch_bounds__(256) void k_pcg_init(const double* __restrict__ b,
                                                  const T* __restrict__ Dinv,
                                                  const T* __restrict__ mi,
                                                  const uint8_t* __restrict__ flags, int64_t nnode,
                                                  int n_nblk, double* __restrict__ x,
                                                  double* __restrict__ r, T* __restrict__ p,
                                                  double* __restrict__ prz, double* __restrict__ pbb,
                                                  double* __restrict__ pmm) {
  __shared__ double sh[4];
  const int nb = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  double rz = 0.0, bb = 0.0, mm = 0.0;
  if (nb < n_nblk) {
    const int64_t ni = (int64_t)nb * MPL_BC + l;
    const uint8_t fl = flags[ni];
    const double m = (double)mi[ni];
    for (int a = 0; a < 3; ++a) {
      const int64_t i = a * nnode + ni;
      const double rv = mpl_free(fl, a) ? b[i] : 0.0;
      const double zv = rv * (double)Dinv[i];
      const T pv = (T)zv;
      x[i] = 0.0;
      r[i] = rv;
      p[i] = pv;
      rz += rv * zv;
      bb += rv * rv;
      mm += m * (double)pv * (double)pv;
    }
  }
  rz = block4_sum(rz, sh);
  bb = block4_sum(bb, sh);
  mm = block4_sum(mm, sh);
  if (threadIdx.x == 0) {
    prz[blockIdx.x] = rz;
    pbb[blockIdx.x] = bb;
    pmm[blockIdx.x] = mm;
  }
}

// q = M p + K p (assembled from the fused product's pieces), x += alpha p,
// r -= alpha q; partials of r.z (z = Dinv r) and r.r.
template <class T>
__global__ __launch_bounds__(256) void k_pcg_update(const T* __restrict__ p,
                                                    const T* __restrict__ Hown,
                                                    const T* __restrict__ Hhalo,
                                                    const int* __restrict__ n_nbr_cell,
                                                    int64_t ncell, const T* __restrict__ mi,
                                                    const T* __restrict__ Dinv,
                                                    const uint8_t* __restrict__ flags, int64_t nnode,
                                                    int n_nblk, double* __restrict__ x,
                                                    double* __restrict__ r, double* __restrict__ prz,
                                                    double* __restrict__ prr,
                                                    const SolverScalars* __restrict__ s,
                                                    T* __restrict__ qout) {
  if (done_flag(s)) return;
  __shared__ double sh[4];
  const int nb = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  const double alpha = s->alpha;
  double rz = 0.0, rr = 0.0;
  if (nb < n_nblk) {
    const int64_t ni = (int64_t)nb * MPL_BC + l;
    const uint8_t fl = flags[ni];
    if (fl & MPL_NODE_FREE_ALL) {
      T h[3];
      gather_kp(Hown, Hhalo, n_nbr_cell, ncell, nb, l, h);
      const T m = mi[ni];
      for (int a = 0; a < 3; ++a) {
        if (!mpl_free(fl, a)) continue;
        const int64_t i = a * nnode + ni;
        const T pv = p[i];
        const T qt = h[a] + m * pv;
        const double q = (double)qt;
        if (qout) qout[i] = qt;
        x[i] += alpha * (double)pv;
        const double rv = r[i] - alpha * q;
        r[i] = rv;
        rz += rv * rv * (double)Dinv[i];
        rr += rv * rv;
      }
    }
  }
  rz = block4_sum(rz, sh);
  rr = block4_sum(rr, sh);
  if (threadIdx.x == 0) {
    prz[blockIdx.x] = rz;
    prr[blockIdx.x] = rr;
  }
}

// p = Dinv r + beta p; partial p^T M p for the next p^T H p.
template <class T>
__global__ __launch_bounds__(256) void k_pcg_direction(const double* __restrict__ r,
                                                       const T* __restrict__ Dinv,
                                                       const T* __restrict__ mi,
                                                       const uint8_t* __restrict__ flags,
                                                       int64_t nnode, int n_nblk,
                                                       T* __restrict__ p, double* __restrict__ pmm,
                                                       const SolverScalars* __restrict__ s) {
  if (done_flag(s)) return;
  __shared__ double sh[4];
  const int nb = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  const double beta = s->beta;
  double mm = 0.0;
  if (nb < n_nblk) {
    const int64_t ni = (int64_t)nb * MPL_BC + l;
    const uint8_t fl = flags[ni];
    const double m = (double)mi[ni];
    for (int a = 0; a < 3; ++a) {
      const int64_t i = a * nnode + ni;
      const T pv = mpl_free(fl, a) ? (T)(r[i] * (double)Dinv[i] + beta * (double)p[i]) : T(0);
      p[i] = pv;
      mm += m * (double)pv * (double)pv;
    }
  }
  mm = block4_sum(mm, sh);
  if (threadIdx.x == 0) pmm[blockIdx.x] = mm;
}

// ---- single-reduction CG (Chronopoulos & Gear) ----
// Mathematically the Jacobi-preconditioned CG above, rearranged so that one
// global reduction per iteration yields both step lengths:
//   p = u + beta p,  s = w + beta s,  x += alpha p,  r -= alpha s,
//   u = Dinv r,  w = H u (next product),
//   gamma = r.u,  delta = u.w,  beta = gamma / gamma_old,
//   alpha = gamma / (delta - beta gamma / alpha_old).
// s carries H p without a second product.  Per iteration: this vector
// kernel, the fused product of u (with its u^T K u partials), one reduction.
// x (FP64) is advanced through an increment dx kept in the tangent's
// precision for at most CG_FLUSH iterations (x += dx every CG_FLUSH-th
// iteration and at the end of the solve), and dx itself only every second
// iteration: with p_j = u_j + beta_j p_{j-1},
//   x_{j+1} = x_{j-1} + alpha_{j-1} p_{j-1} + alpha_j p_j,
// and iteration j (odd) holds both p_{j-1} (the p it reads) and p_j.  After
// an even iteration the term alpha_j p_j is pending (the flush adds it).
// u = Dinv r is stored for the product but not read back by the update,
// which forms it again from r and Dinv (same rounding).
#define CG_FLUSH 8
// BJ: Dinv holds the inverted 3x3 node blocks (block_apply layout, six
// entries per node) instead of the inverse diagonal, and u = B r.
template <class T, bool BJ>
__global__ __launch_bounds__(256) void k_cg_init(const double* __restrict__ b, const T* __restrict__ Dinv,
                                                 const T* __restrict__ mi, const uint8_t* __restrict__ flags,
                                                 int64_t nnode, int n_nblk, double* __restrict__ x,
                                                 T* __restrict__ dx,
                                                 double* __restrict__ r, T* __restrict__ u,
                                                 T* __restrict__ p, T* __restrict__ sv,
                                                 double* __restrict__ pg, double* __restrict__ pbb,
                                                 double* __restrict__ pmu, SolverScalars* __restrict__ s) {
  __shared__ double sh[4];
  const int nb = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  // the first product (next launch) must run even if the previous solve
  // left the done flag set; the reduction after it sets the flag again
  if (blockIdx.x == 0 && threadIdx.x == 0) s->done = 0;
  double g = 0.0, bb = 0.0, mu = 0.0;
  if (nb < n_nblk) {
    const int64_t ni = (int64_t)nb * MPL_BC + l;
    const uint8_t fl = flags[ni];
    const double m = (double)mi[ni];
    if constexpr (BJ) {
      double rb[3], bk[6], z[3];
      for (int a = 0; a < 3; ++a) rb[a] = mpl_free(fl, a) ? b[a * nnode + ni] : 0.0;
      for (int e = 0; e < 6; ++e) bk[e] = (double)Dinv[e * nnode + ni];
      block_apply(bk, rb, z);
      for (int a = 0; a < 3; ++a) {
        const int64_t i = a * nnode + ni;
        const T uv = (T)z[a];
        x[i] = 0.0;
        dx[i] = T(0);
        r[i] = rb[a];
        u[i] = uv;
        p[i] = T(0);
        sv[i] = T(0);
        g += rb[a] * (double)uv;
        bb += rb[a] * rb[a];
        mu += m * (double)uv * (double)uv;
      }
    } else
    for (int a = 0; a < 3; ++a) {
      const int64_t i = a * nnode + ni;
      const double rv = mpl_free(fl, a) ? b[i] : 0.0;
      const T uv = (T)(rv * (double)Dinv[i]);
      x[i] = 0.0;
      dx[i] = T(0);
      r[i] = rv;
      u[i] = uv;
      p[i] = T(0);
      sv[i] = T(0);
      g += rv * (double)uv;
      bb += rv * rv;
      mu += m * (double)uv * (double)uv;
    }
  }
  g = block4_sum(g, sh);
  bb = block4_sum(bb, sh);
  mu = block4_sum(mu, sh);
  if (threadIdx.x == 0) {
    pg[blockIdx.x] = g;
    pbb[blockIdx.x] = bb;
    pmu[blockIdx.x] = mu;
  }
}

// Warm start: u = x0 in the tangent's precision (free components), for the
// product H x0 that gives the initial residual.
template <class T>
__global__ void k_cg_prep(const double* __restrict__ x0, const uint8_t* __restrict__ flags, int64_t nnode,
                          T* __restrict__ u) {
  const int64_t ni = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ni >= nnode) return;
  const uint8_t fl = flags[ni];
  for (int a = 0; a < 3; ++a) u[a * nnode + ni] = mpl_free(fl, a) ? (T)x0[a * nnode + ni] : T(0);
}

// Warm-start variant of k_cg_init: x = x0, r = b - H x0 (the product's
// pieces and u = x0 given), then as k_cg_init; the b.b partial stays the
// tolerance reference.
template <class T, bool BJ>
__global__ __launch_bounds__(256) void k_cg_init_warm(const double* __restrict__ b,
                                                      const double* __restrict__ x0,
                                                      const T* __restrict__ Hown, const T* __restrict__ Hhalo,
                                                      const int* __restrict__ n_nbr_cell, int64_t ncell,
                                                      const T* __restrict__ Dinv, const T* __restrict__ mi,
                                                      const uint8_t* __restrict__ flags, int64_t nnode,
                                                      int n_nblk, double* __restrict__ x, T* __restrict__ dx,
                                                      double* __restrict__ r, T* __restrict__ u,
                                                      T* __restrict__ p, T* __restrict__ sv,
                                                      double* __restrict__ pg, double* __restrict__ pbb,
                                                      double* __restrict__ pmu, SolverScalars* __restrict__ s) {
  __shared__ double sh[4];
  const int nb = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  if (blockIdx.x == 0 && threadIdx.x == 0) s->done = 0;
  double g = 0.0, bb = 0.0, mu = 0.0;
  if (nb < n_nblk) {
    const int64_t ni = (int64_t)nb * MPL_BC + l;
    const uint8_t fl = flags[ni];
    const T m = mi[ni];
    T h[3] = {T(0), T(0), T(0)};
    if (fl & MPL_NODE_FREE_ALL) gather_kp(Hown, Hhalo, n_nbr_cell, ncell, nb, l, h);
    if constexpr (BJ) {
      double bv[3], rb[3], bk[6], z[3];
      for (int a = 0; a < 3; ++a) {
        const int64_t i = a * nnode + ni;
        const bool fa = mpl_free(fl, a);
        bv[a] = fa ? b[i] : 0.0;
        rb[a] = fa ? bv[a] - (double)(h[a] + m * u[i]) : 0.0;
      }
      for (int e = 0; e < 6; ++e) bk[e] = (double)Dinv[e * nnode + ni];
      block_apply(bk, rb, z);
      for (int a = 0; a < 3; ++a) {
        const int64_t i = a * nnode + ni;
        const T uv = (T)z[a];
        x[i] = mpl_free(fl, a) ? x0[i] : 0.0;
        dx[i] = T(0);
        r[i] = rb[a];
        u[i] = uv;
        p[i] = T(0);
        sv[i] = T(0);
        g += rb[a] * (double)uv;
        bb += bv[a] * bv[a];
        mu += (double)m * (double)uv * (double)uv;
      }
    } else
    for (int a = 0; a < 3; ++a) {
      const int64_t i = a * nnode + ni;
      const bool fa = mpl_free(fl, a);
      const double bv = fa ? b[i] : 0.0;
      const double rv = fa ? bv - (double)(h[a] + m * u[i]) : 0.0;
      const T uv = (T)(rv * (double)Dinv[i]);
      x[i] = fa ? x0[i] : 0.0;
      dx[i] = T(0);
      r[i] = rv;
      u[i] = uv;
      p[i] = T(0);
      sv[i] = T(0);
      g += rv * (double)uv;
      bb += bv * bv;
      mu += (double)m * (double)uv * (double)uv;
    }
  }
  g = block4_sum(g, sh);
  bb = block4_sum(bb, sh);
  mu = block4_sum(mu, sh);
  if (threadIdx.x == 0) {
    pg[blockIdx.x] = g;
    pbb[blockIdx.x] = bb;
    pmu[blockIdx.x] = mu;
  }
}

// The FP32 Jacobi variant is held to 80 VGPRs (six waves per SIMD instead of
// five: more of its loads in flight, no spill); the others keep the
// compiler's choice, which a cap would spill.
template <class T, bool BJ>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu((BJ || sizeof(T) == 8) ? 1 : 6))) void k_cg_step(T* __restrict__ u, T* __restrict__ p, T* __restrict__ sv,
                                                 const T* __restrict__ Hown, const T* __restrict__ Hhalo,
                                                 const int* __restrict__ n_nbr_cell, int64_t ncell,
                                                 const T* __restrict__ mi, const T* __restrict__ Dinv,
                                                 const uint8_t* __restrict__ flags, int64_t nnode,
                                                 int n_nblk, double* __restrict__ x, T* __restrict__ dx,
                                                 double* __restrict__ r,
                                                 double* __restrict__ pg, double* __restrict__ prr,
                                                 double* __restrict__ pmu,
                                                 const SolverScalars* __restrict__ s) {
  if (done_flag(s)) return;
  __shared__ double sh3[3][4];
  const int nb = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  const double alpha = s->alpha, beta = s->beta, alpha_last = s->alpha_last;
  const int it = s->iters;
  const bool odd = (it & 1) != 0;
  const bool flush = ((it + 1) % CG_FLUSH) == 0;  // odd iterations only (CG_FLUSH even)
  double g = 0.0, rr = 0.0, mu = 0.0;
  if constexpr (BJ) {
    // block-Jacobi: the same recurrence with u = B r (all three components
    // of r enter each component of u)
    if (nb < n_nblk) {
      const int64_t ni = (int64_t)nb * MPL_BC + l;
      const uint8_t fl = flags[ni];
      T pv[3], svv[3], dxv[3] = {T(0), T(0), T(0)};
      double xv[3] = {0.0, 0.0, 0.0}, rv[3], bk[6];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int64_t i = a * nnode + ni;
        pv[a] = p[i];
        svv[a] = sv[i];
        if (odd) dxv[a] = dx[i];
        if (flush) xv[a] = x[i];
        rv[a] = r[i];
      }
#pragma unroll
      for (int e = 0; e < 6; ++e) bk[e] = (double)Dinv[e * nnode + ni];
      const T m = mi[ni];
      T h[3];
      gather_kp(Hown, Hhalo, n_nbr_cell, ncell, nb, l, h);
      if (fl & MPL_NODE_FREE_ALL) {
        double ud[3], rn[3], und[3];
        block_apply(bk, rv, ud);  // u_j = B r_j as stored for the product
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int64_t i = a * nnode + ni;
          rn[a] = rv[a];
          if (!mpl_free(fl, a)) continue;  // fixed components stay 0
          const T uv = (T)ud[a];
          const T w = h[a] + m * uv;
          const T pn = (T)((double)uv + beta * (double)pv[a]);
          const T sn = (T)((double)w + beta * (double)svv[a]);
          rn[a] = rv[a] - alpha * (double)sn;
          p[i] = pn;
          sv[i] = sn;
          if (odd) {
            const double inc = (double)dxv[a] + (alpha_last * (double)pv[a] + alpha * (double)pn);
            if (flush) {
              x[i] = xv[a] + inc;
              dx[i] = T(0);
            } else {
              dx[i] = (T)inc;
            }
          }
          r[i] = rn[a];
        }
        block_apply(bk, rn, und);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const T un = (T)und[a];
          u[a * nnode + ni] = un;
          g += rn[a] * (double)un;
          rr += rn[a] * rn[a];
          mu += (double)m * (double)un * (double)un;
        }
      }
    }
  } else
  if (nb < n_nblk) {
    const int64_t ni = (int64_t)nb * MPL_BC + l;
    // all loads of the node (three components, the flag, the gathered
    // pieces) are issued at once, also on nodes that are not free (their
    // lines are read by the wave anyway); only free components store
    const uint8_t fl = flags[ni];
    T pv[3], svv[3], dv[3], dxv[3] = {T(0), T(0), T(0)};
    double xv[3] = {0.0, 0.0, 0.0}, rv[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int64_t i = a * nnode + ni;
      pv[a] = p[i];
      svv[a] = sv[i];
      dv[a] = Dinv[i];
      if (odd) dxv[a] = dx[i];
      if (flush) xv[a] = x[i];
      rv[a] = r[i];
    }
    const T m = mi[ni];
    T h[3];
    gather_kp(Hown, Hhalo, n_nbr_cell, ncell, nb, l, h);
    if (fl & MPL_NODE_FREE_ALL) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (!mpl_free(fl, a)) continue;  // fixed components stay 0
        const int64_t i = a * nnode + ni;
        const T uv = (T)(rv[a] * (double)dv[a]);  // u_j = Dinv r_j as stored for the product
        const T w = h[a] + m * uv;                // (H u)_i
        const T pn = (T)((double)uv + beta * (double)pv[a]);
        const T sn = (T)((double)w + beta * (double)svv[a]);
        const double rn = rv[a] - alpha * (double)sn;
        const T un = (T)(rn * (double)dv[a]);
        p[i] = pn;
        sv[i] = sn;
        if (odd) {
          const double inc = (double)dxv[a] + (alpha_last * (double)pv[a] + alpha * (double)pn);
          if (flush) {
            x[i] = xv[a] + inc;
            dx[i] = T(0);
          } else {
            dx[i] = (T)inc;
          }
        }
        r[i] = rn;
        u[i] = un;
        g += rn * (double)un;
        rr += rn * rn;
        mu += (double)m * (double)un * (double)un;
      }
    }
  }
  // the three workgroup sums behind one barrier (same order as a
  // workgroup sum of each: waves paired (0+1) + (2+3))
  g = wave_sum(g);
  rr = wave_sum(rr);
  mu = wave_sum(mu);
  if ((threadIdx.x & 63) == 0) {
    sh3[0][threadIdx.x >> 6] = g;
    sh3[1][threadIdx.x >> 6] = rr;
    sh3[2][threadIdx.x >> 6] = mu;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    pg[blockIdx.x] = (sh3[0][0] + sh3[0][1]) + (sh3[0][2] + sh3[0][3]);
    prr[blockIdx.x] = (sh3[1][0] + sh3[1][1]) + (sh3[1][2] + sh3[1][3]);
    pmu[blockIdx.x] = (sh3[2][0] + sh3[2][1]) + (sh3[2][2] + sh3[2][3]);
  }
}

// Scratch of the two-level CG reduction: per-workgroup sums and the ticket
// counter (zero between launches).
#define CG_RED_MAX 64
struct CgRed {
  double part[4][CG_RED_MAX];
  unsigned ticket;
};
__global__ void k_cg_red_zero(CgRed* __restrict__ red) {
  if (threadIdx.x == 0) red->ticket = 0u;
}
// workgroups of the two-level reduction for arrays of up to nm entries
static int cg_red_groups(int nm) { return red2_groups(nm, CG_RED_MAX); }

// Reduction of the four partial arrays of one single-reduction CG
// iteration, then its scalar logic.  INIT: A = r.u, B = b.b, C = u^T M u,
// D = u^T K u.  STEP: A = r.u, B = r.r, C, D as in INIT.
// Two levels in one launch of G <= CG_RED_MAX workgroups: workgroup g sums
// a contiguous range of every array in a fixed order; the workgroup that
// takes the last ticket (no waiting) sums the G results in workgroup order
// and runs the scalar logic.  The order depends on the array lengths only,
// so the sums are reproducible.
template <bool INIT>
__global__ __launch_bounds__(256) void k_reduce_cg(const double* __restrict__ a,
                                                   const double* __restrict__ b,
                                                   const double* __restrict__ c, int n,
                                                   const double* __restrict__ d, int nd,
                                                   CgRed* __restrict__ red,
                                                   SolverScalars* __restrict__ s) {
  __shared__ double sh[4][4];
  __shared__ int last;
  const int t = threadIdx.x, g = blockIdx.x, G = gridDim.x;
  if (!INIT && done_flag(s)) return;  // every workgroup sees the same flag
  int lo, hi;
  red2_range(g, G, n > nd ? n : nd, lo, hi);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = lo + t; i < hi; i += 256) {
    // the four loads issued together (indices clamped into range, values
    // past an array's end replaced by zero)
    const int ia = min(i, n - 1), id = min(i, nd - 1);
    const double va = n > 0 ? a[ia] : 0.0, vb = n > 0 ? b[ia] : 0.0, vc = n > 0 ? c[ia] : 0.0;
    const double vd = nd > 0 ? d[id] : 0.0;
    acc[0] += i < n ? va : 0.0;
    acc[1] += i < n ? vb : 0.0;
    acc[2] += i < n ? vc : 0.0;
    acc[3] += i < nd ? vd : 0.0;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double w = wave_sum(acc[q]);
    if ((t & 63) == 0) sh[q][t >> 6] = w;
  }
  __syncthreads();
  if (t == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      __hip_atomic_store(&red->part[q][g], ((sh[q][0] + sh[q][1]) + sh[q][2]) + sh[q][3], __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    // the sums above are visible device-wide before the ticket is taken
    const unsigned prev = __hip_atomic_fetch_add(&red->ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    last = prev == (unsigned)(G - 1);
  }
  __syncthreads();
  if (!last || t >= 64) return;
  // the last workgroup: one wave sums the G results in workgroup order
  double v[4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    v[q] = t < G ? __hip_atomic_load(&red->part[q][t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) v[q] = wave_sum(v[q]);
  if (t != 0) return;
  __hip_atomic_store(&red->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);  // ready for the next launch
  const double A = v[0], B = v[1], C = v[2], D = v[3];
  const double s_alpha = s->alpha, s_rz = s->rz, s_tol2 = s->tol2;
  const int s_iters = s->iters;
  const double delta = C + D;
  if (INIT) {
    s->alpha_last = 0.0;
    s->bnorm2 = B;
    s->rr = B;
    s->rz = A;
    s->iters = 0;
    s->beta = 0.0;
    s->done = (B == 0.0) ? 1 : 0;
    if (s->done == 0) {
      if (!(delta > 0.0) || !isfinite(delta)) {
        s->done = 2;
        s->alpha = 0.0;
      } else {
        s->alpha = A / delta;
      }
    }
    return;
  }
  s->alpha_last = s_alpha;  // the step length the completed iteration used
  s->iters = s_iters + 1;
  s->rr = B;
  if (!isfinite(B)) {
    s->done = 2;
    return;
  }
  if (B <= s_tol2) {
    s->done = 1;
    return;
  }
  const double beta = A / s_rz;
  const double denom = delta - beta * A / s_alpha;
  if (!(denom > 0.0) || !isfinite(denom)) {
    s->done = 2;
    return;
  }
  s->beta = beta;
  s->alpha = A / denom;
  s->rz = A;
}

// x += dx (+ alpha_last p when the last iteration's term is pending, i.e.
// an odd number of iterations is complete); dx then carries -alpha_last p so
// that the next (odd) iteration's paired update stays exact.
template <class T>
__global__ __launch_bounds__(256) void k_cg_flush(double* __restrict__ x, T* __restrict__ dx,
                                                  const T* __restrict__ p, int64_t nnode, int64_t nused,
                                                  const SolverScalars* __restrict__ s) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * nnode || i % nnode >= nused) return;
  const bool pending = (s->iters & 1) != 0;
  const double q = pending ? s->alpha_last * (double)p[i] : 0.0;
  x[i] += (double)dx[i] + q;
  dx[i] = (T)(-q);
}

// ---- flexible CG with the learned preconditioner ----
// The preconditioned residual is z = Dinv r + s sqrt(Dinv) o on free nodes,
// o the network output (bf16, 16 channels per box voxel, voxel = node), s^2 =
// s2 / (free DOFs); after a fallback z = Dinv r.
struct NetOut {
  const uint16_t* o;
  int bx, by, bz;
  double inv_nfree;
};
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

__device__ __forceinline__ void learned_z(const NetOut& net, int4 bc, int l, const double* r,
                                          const double* Dinv, int64_t nnode, int64_t ni, double sc,
                                          bool jacobi, double z[3]) {
  const int i = bc.x * 4 + local_x(l), j = bc.y * 4 + local_y(l), k = bc.z * 4 + local_z(l);
  const bool in = !jacobi && i < net.bx && j < net.by && k < net.bz;
  const int64_t v = in ? ((int64_t)i * net.by + j) * net.bz + k : 0;
  for (int a = 0; a < 3; ++a) {
    const double di = Dinv[a * nnode + ni];
    z[a] = di * r[a * nnode + ni];
    if (in) z[a] += sc * sqrt(di) * (double)bf16_to_f32(net.o[v * 16 + a]);
  }
}

// x = 0, r = b on the free components; partials b.b and sum Dinv b^2.
__global__ __launch_bounds__(256) void k_fpcg_init(const double* __restrict__ b,
                                                   const double* __restrict__ Dinv,
                                                   const uint8_t* __restrict__ flags, int64_t nnode,
                                                   int n_nblk, double* __restrict__ x,
                                                   double* __restrict__ r, double* __restrict__ pbb,
                                                   double* __restrict__ ps2) {
  __shared__ double sh[4];
  const int nb = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  double bb = 0.0, s2 = 0.0;
  if (nb < n_nblk) {
    const int64_t ni = (int64_t)nb * MPL_BC + l;
    const uint8_t fl = flags[ni];
    for (int a = 0; a < 3; ++a) {
      const int64_t i = a * nnode + ni;
      const double rv = mpl_free(fl, a) ? b[i] : 0.0;
      x[i] = 0.0;
      r[i] = rv;
      bb += rv * rv;
      s2 += rv * rv * Dinv[i];
    }
  }
  bb = block4_sum(bb, sh);
  s2 = block4_sum(s2, sh);
  if (threadIdx.x == 0) {
    pbb[blockIdx.x] = bb;
    ps2[blockIdx.x] = s2;
  }
}

// Flexible CG from x0: x = x0, r = b - H x0 on the free components (the
// product's pieces of u0 = x0 in the tangent's precision given); partials of
// b.b, sum Dinv r^2 and r.r.
template <class T>
__global__ __launch_bounds__(256) void k_fpcg_init_warm(const double* __restrict__ b,
                                                        const double* __restrict__ x0,
                                                        const T* __restrict__ u0, const T* __restrict__ Hown,
                                                        const T* __restrict__ Hhalo,
                                                        const int* __restrict__ n_nbr_cell, int64_t ncell,
                                                        const T* __restrict__ mi,
                                                        const double* __restrict__ Dinv,
                                                        const uint8_t* __restrict__ flags, int64_t nnode,
                                                        int n_nblk, double* __restrict__ x,
                                                        double* __restrict__ r, double* __restrict__ pbb,
                                                        double* __restrict__ ps2, double* __restrict__ prr) {
  __shared__ double sh[4];
  const int nb = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  double bb = 0.0, s2 = 0.0, rr = 0.0;
  if (nb < n_nblk) {
    const int64_t ni = (int64_t)nb * MPL_BC + l;
    const uint8_t fl = flags[ni];
    T h[3] = {T(0), T(0), T(0)};
    if (fl & MPL_NODE_FREE_ALL) gather_kp(Hown, Hhalo, n_nbr_cell, ncell, nb, l, h);
    const T m = mi[ni];
    for (int a = 0; a < 3; ++a) {
      const int64_t i = a * nnode + ni;
      const bool fa = mpl_free(fl, a);
      const double bv = fa ? b[i] : 0.0;
      const double rv = fa ? bv - (double)(h[a] + m * u0[i]) : 0.0;
      x[i] = fa ? x0[i] : 0.0;
      r[i] = rv;
      bb += bv * bv;
      s2 += rv * rv * Dinv[i];
      rr += rv * rv;
    }
  }
  bb = block4_sum(bb, sh);
  s2 = block4_sum(s2, sh);
  rr = block4_sum(rr, sh);
  if (threadIdx.x == 0) {
    pbb[blockIdx.x] = bb;
    ps2[blockIdx.x] = s2;
    prr[blockIdx.x] = rr;
  }
}

// partials z.r and z.q (q may be null: first iteration)
template <class T>
__global__ __launch_bounds__(256) void k_fpcg_dots(const double* __restrict__ r,
                                                   const T* __restrict__ q,
                                                   const double* __restrict__ Dinv,
                                                   const uint8_t* __restrict__ flags,
                                                   const int4* __restrict__ ncoord, int64_t nnode,
                                                   int n_nblk, NetOut net, double* __restrict__ pzr,
                                                   double* __restrict__ pzq,
                                                   const SolverScalars* __restrict__ s) {
  if (done_flag(s) || s->fallback) return;
  __shared__ double sh[4];
  const int nb = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  const double sc = sqrt(fmax(s->s2 * net.inv_nfree, 1e-300));
  double zr = 0.0, zq = 0.0;
  if (nb < n_nblk) {
    const int64_t ni = (int64_t)nb * MPL_BC + l;
    if (flags[ni] & MPL_NODE_FREE_ALL) {
      double z[3];
      learned_z(net, ncoord[nb], l, r, Dinv, nnode, ni, sc, false, z);
      for (int a = 0; a < 3; ++a) {
        zr += z[a] * r[a * nnode + ni];
        if (q) zq += z[a] * (double)q[a * nnode + ni];
      }
    }
  }
  zr = block4_sum(zr, sh);
  zq = block4_sum(zq, sh);
  if (threadIdx.x == 0) {
    pzr[blockIdx.x] = zr;
    pzq[blockIdx.x] = zq;
  }
}

// p = z + beta p; partial p^T M p.
template <class T>
__global__ __launch_bounds__(256) void k_fpcg_direction(const double* __restrict__ r,
                                                        const double* __restrict__ Dinv,
                                                        const double* __restrict__ mi,
                                                        const uint8_t* __restrict__ flags,
                                                        const int4* __restrict__ ncoord,
                                                        int64_t nnode, int n_nblk, NetOut net,
                                                        T* __restrict__ p, double* __restrict__ pmm,
                                                        const SolverScalars* __restrict__ s) {
  if (done_flag(s)) return;
  __shared__ double sh[4];
  const int nb = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  const double beta = s->beta;
  const bool jacobi = s->fallback != 0;
  const double sc = sqrt(fmax(s->s2 * net.inv_nfree, 1e-300));
  double mm = 0.0;
  if (nb < n_nblk) {
    const int64_t ni = (int64_t)nb * MPL_BC + l;
    const uint8_t fl = flags[ni];
    const double m = mi[ni];
    double z[3] = {0.0, 0.0, 0.0};
    if (fl & MPL_NODE_FREE_ALL) learned_z(net, ncoord[nb], l, r, Dinv, nnode, ni, sc, jacobi, z);
    for (int a = 0; a < 3; ++a) {
      const int64_t i = a * nnode + ni;
      // beta = 0 (first iteration, restart after a fallback) does not read
      // the previous direction, which may hold anything on the first call
      const double pold = (beta != 0.0) ? (double)p[i] : 0.0;
      const T pv = mpl_free(fl, a) ? (T)(z[a] + beta * pold) : T(0);
      p[i] = pv;
      mm += m * (double)pv * (double)pv;
    }
  }
  mm = block4_sum(mm, sh);
  if (threadIdx.x == 0) pmm[blockIdx.x] = mm;
}

// z = learned preconditioner applied to r (block layout, FP64 output).
__global__ __launch_bounds__(256) void k_precond_z(const double* __restrict__ r,
                                                   const double* __restrict__ Dinv,
                                                   const uint8_t* __restrict__ flags,
                                                   const int4* __restrict__ ncoord, int64_t nnode,
                                                   int n_nblk, NetOut net,
                                                   const SolverScalars* __restrict__ s,
                                                   double* __restrict__ z) {
  const int nb = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  if (nb >= n_nblk) return;
  const int64_t ni = (int64_t)nb * MPL_BC + l;
  double zz[3] = {0.0, 0.0, 0.0};
  if (flags[ni] & MPL_NODE_FREE_ALL)
    learned_z(net, ncoord[nb], l, r, Dinv, nnode, ni, sqrt(fmax(s->s2 * net.inv_nfree, 1e-300)), false,
              zz);
  for (int a = 0; a < 3; ++a) z[a * nnode + ni] = zz[a];
}

// ---- online training of the learned preconditioner ----
// Energy-norm loss on the solver's residual r:
//   L(z) = (1/2 z^T H z - z^T r) / (r^T Dinv r),
// minimised by z = H^{-1} r; L - L(H^{-1} r) is half the squared H-norm
// error of z over r^T Dinv r.  With z = Dinv r + s sqrt(Dinv) o:
//   dL/do = s sqrt(Dinv) (H z - r) / (r^T Dinv r).
__global__ __launch_bounds__(256) void k_online_rdr(const double* __restrict__ r,
                                                    const double* __restrict__ Dinv,
                                                    const uint8_t* __restrict__ flags, int64_t nnode,
                                                    int n_nblk, double* __restrict__ part) {
  __shared__ double sh[4];
  const int nb = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  double acc = 0.0;
  if (nb < n_nblk) {
    const int64_t ni = (int64_t)nb * MPL_BC + l;
    if (flags[ni] & MPL_NODE_FREE_ALL)
      for (int a = 0; a < 3; ++a) {
        const double rv = r[a * nnode + ni];
        acc += rv * rv * Dinv[a * nnode + ni];
      }
  }
  acc = block4_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

template <class T>
__global__ __launch_bounds__(256) void k_online_z(const double* __restrict__ r,
                                                  const double* __restrict__ Dinv,
                                                  const uint8_t* __restrict__ flags,
                                                  const int4* __restrict__ ncoord, int64_t nnode,
                                                  int n_nblk, NetOut net, const double* __restrict__ rdr,
                                                  T* __restrict__ z, int jacobi) {
  const int nb = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  if (nb >= n_nblk) return;
  const int64_t ni = (int64_t)nb * MPL_BC + l;
  double zz[3] = {0.0, 0.0, 0.0};
  if (flags[ni] & MPL_NODE_FREE_ALL)
    learned_z(net, ncoord[nb], l, r, Dinv, nnode, ni, sqrt(fmax(rdr[0] * net.inv_nfree, 1e-300)),
              jacobi != 0, zz);
  for (int a = 0; a < 3; ++a) z[a * nnode + ni] = (T)zz[a];
}

// partials z.Hz and z.r
template <class T>
__global__ __launch_bounds__(256) void k_online_dots(const double* __restrict__ r,
                                                     const T* __restrict__ z,
                                                     const T* __restrict__ hz,
                                                     const uint8_t* __restrict__ flags, int64_t nnode,
                                                     int n_nblk, double* __restrict__ pzhz,
                                                     double* __restrict__ pzr) {
  __shared__ double sh[4];
  const int nb = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  double a1 = 0.0, a2 = 0.0;
  if (nb < n_nblk) {
    const int64_t ni = (int64_t)nb * MPL_BC + l;
    if (flags[ni] & MPL_NODE_FREE_ALL)
      for (int a = 0; a < 3; ++a) {
        const int64_t i = a * nnode + ni;
        a1 += (double)z[i] * (double)hz[i];
        a2 += (double)z[i] * r[i];
      }
  }
  a1 = block4_sum(a1, sh);
  a2 = block4_sum(a2, sh);
  if (threadIdx.x == 0) {
    pzhz[blockIdx.x] = a1;
    pzr[blockIdx.x] = a2;
  }
}

// node-layout output gradient s sqrt(Dinv) (Hz - r) / rdr; loss into *loss
template <class T>
__global__ __launch_bounds__(256) void k_online_grad(const double* __restrict__ r,
                                                     const T* __restrict__ hz,
                                                     const double* __restrict__ Dinv,
                                                     const uint8_t* __restrict__ flags, int64_t nnode,
                                                     int n_nblk, double inv_nfree,
                                                     const double* __restrict__ red,
                                                     double* __restrict__ g, double* __restrict__ loss) {
  const int nb = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  const double rdr = red[0];
  if (blockIdx.x == 0 && threadIdx.x == 0) *loss = rdr > 0.0 ? (0.5 * red[1] - red[2]) / rdr : 0.0;
  if (nb >= n_nblk) return;
  const int64_t ni = (int64_t)nb * MPL_BC + l;
  const uint8_t fl = flags[ni];
  const double sc = sqrt(fmax(rdr * inv_nfree, 1e-300));
  for (int a = 0; a < 3; ++a) {
    const int64_t i = a * nnode + ni;
    g[i] = (mpl_free(fl, a) && rdr > 0.0) ? sc * sqrt(Dinv[i]) * ((double)hz[i] - r[i]) / rdr : 0.0;
  }
}

__global__ __launch_bounds__(64) void k_axpy_dot(const double* __restrict__ v,
                                                 const double* __restrict__ dir, double alpha,
                                                 const double* __restrict__ g,
                                                 const uint8_t* __restrict__ flags, int64_t nnode,
                                                 double* __restrict__ out, double* __restrict__ pdot) {
  const int nb = blockIdx.x, l = threadIdx.x;
  const int64_t ni = (int64_t)nb * MPL_BC + l;
  const uint8_t fl = flags[ni];
  double dt = 0.0;
  for (int a = 0; a < 3; ++a) {
    const int64_t i = a * nnode + ni;
    const bool fa = mpl_free(fl, a);
    out[i] = fa ? v[i] + alpha * dir[i] : v[i];
    if (g) dt += fa ? g[i] * dir[i] : 0.0;
  }
  if (pdot) {
    dt = wave_sum(dt);
    if (l == 0) pdot[nb] = dt;
  }
}

__global__ __launch_bounds__(64) void k_escale(const double* __restrict__ Vk, int64_t ncell, int K,
                                               double* __restrict__ partial,
    const MatParams* __restrict__ mats) {
  const int cb = blockIdx.x, l = threadIdx.x;
  const int64_t ci = (int64_t)cb * MPL_BC + l;
  double s = 0.0;
  for (int k = 0; k < K; ++k) s += Vk[k * ncell + ci] * (mats[k].mu + fabs(mats[k].lambda));
  s = wave_sum(s);
  if (l == 0) partial[cb] = s;
}

template <class T>
__global__ void k_mask_free(T* __restrict__ u, const uint8_t* __restrict__ flags, int64_t nnode) {
  int64_t ni = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ni >= nnode) return;
  const uint8_t fl = flags[ni];
  for (int a = 0; a < 3; ++a)
    if (!mpl_free(fl, a)) u[a * nnode + ni] = T(0);
}

__global__ void k_neg(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = -a[i];
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

}  // namespace

// ======================================================================
// The materials live in the context's own device table (copied at creation),
// so contexts on one GPU never share them.
static mpl_status upload_mats(mpl_ctx*) { return MPL_OK; }

static mpl_status ensure_partials(mpl_ctx* c) {
  size_t n = std::max(c->n_cblk, c->n_nblk) + 64;
  return mpl_ensure(c, c->partials, sizeof(double) * 8 * n);
}
static double* partial_slot(mpl_ctx* c, int k) {
  size_t n = std::max(c->n_cblk, c->n_nblk) + 64;
  return P<double>(c->partials) + k * n;
}

// The base the energy and tangent kernels read: the return-mapped one under
// fixed-point plasticity, else the symmetric stretch (null).
static const double* sgen(mpl_ctx* c) { return c->s_general ? P<double>(c->Seff) : nullptr; }

// Fixed-point plasticity: the base at the node velocity v (block layout).
// ---- Anderson acceleration of fixed-point plasticity ----
struct AAVecs {
  const double* p[10];
};
struct AACoef {
  double a[10];
};

// v_hist = v, f_hist = vt - v (the accepted Newton update), all slots.
__global__ void k_aa_push(const double* __restrict__ v, const double* __restrict__ vt,
                          double* __restrict__ vh, double* __restrict__ fh, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  vh[i] = v[i];
  fh[i] = vt[i] - v[i];
}

// Partial dot products f_i . f_j (i <= j < nv) over free DOFs, one partial per
// workgroup of four node blocks: part[pair * nwg + wg].
__global__ __launch_bounds__(256) void k_aa_gram(AAVecs f, int nv, const uint8_t* __restrict__ flags,
                                                 int64_t nnode, int n_nblk, double* __restrict__ part, int nwg) {
  __shared__ double sh[4];
  const int nb = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  const int64_t ni = (int64_t)nb * MPL_BC + l;
  const uint8_t fl = nb < n_nblk ? flags[ni] : (uint8_t)0;
  double x[5][3];
  for (int k = 0; k < nv; ++k)
    for (int a = 0; a < 3; ++a) x[k][a] = mpl_free(fl, a) ? f.p[k][a * nnode + ni] : 0.0;
  int pair = 0;
  for (int i = 0; i < nv; ++i)
    for (int j = i; j < nv; ++j, ++pair) {
      double d = x[i][0] * x[j][0] + x[i][1] * x[j][1] + x[i][2] * x[j][2];
      d = block4_sum(d, sh);
      if (threadIdx.x == 0) part[(int64_t)pair * nwg + blockIdx.x] = d;
      __syncthreads();
    }
}

// out[pair] = sum of that pair's partials, fixed order, one workgroup.
__global__ __launch_bounds__(1024) void k_aa_reduce(const double* __restrict__ part, int npair, int nwg,
                                                    double* __restrict__ out) {
  __shared__ double sh[16];
  const int t = threadIdx.x;
  for (int p = 0; p < npair; ++p) {
    double acc = 0.0;
    for (int i = t; i < nwg; i += 1024) acc += part[(int64_t)p * nwg + i];
    acc = wave_sum(acc);
    if ((t & 63) == 0) sh[t >> 6] = acc;
    __syncthreads();
    if (t == 0) {
      double s2 = 0.0;
      for (int w = 0; w < 16; ++w) s2 += sh[w];
      out[p] = s2;
    }
    __syncthreads();
  }
}

// out = sum_k coef_k vec_k over all slots.
__global__ void k_aa_combine(AAVecs vec, AACoef coef, int nv, double* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s2 = 0.0;
  for (int k = 0; k < nv; ++k) s2 += coef.a[k] * vec.p[k][i];
  out[i] = s2;
}

static mpl_status plastic_base(mpl_ctx* c, const double* v) {
  const int64_t ncell = (int64_t)c->ncell_alloc(), nnode = (int64_t)c->nnode_alloc();
  MPL_TRY(upload_mats(c));
  MPL_TRY(mpl_ensure(c, c->Seff, sizeof(double) * 9 * c->nmat * ncell));
  MPL_LAUNCH(c, k_plastic_base, c->n_cblk, 64, v, nnode, P<int>(c->c_nbr_node), P<double>(c->Vk),
             P<double>(c->Sk), ncell, c->nmat, c->dt, 0.25 * c->inv_dx, P<double>(c->Seff),
             &c->dscal()->err, P<MatParams>(c->matbuf));
  c->s_general = true;
  return MPL_OK;
}

mpl_status mpl_stage_reconstruct(mpl_ctx* c) {
  if (!c->unloaded) return mpl_fail(c, MPL_ERR_STATE, "reconstruct before unload");
  MPL_TRY(upload_mats(c));
  const int64_t ncell = (int64_t)c->ncell_alloc();
  MPL_HIP(c, hipMemsetAsync(&c->dscal()->domain_count, 0, sizeof(int32_t), c->stream));
  MPL_LAUNCH(c, k_reconstruct, (int)((ncell + 127) / 128), 128, P<double>(c->Vk), P<double>(c->Tk),
             P<double>(c->Sk), ncell, c->nmat, &c->dscal()->domain_count, P<MatParams>(c->matbuf));
  c->reconstructed = true;
  c->s_general = false;
  return MPL_OK;
}

// energy (and gradient into c->g) at v (block layout); gnorm2 may be null.
mpl_status mpl_stage_energy(mpl_ctx* c, const double* v, bool want_grad, double* energy,
                            double* gnorm2) {
  if (!c->reconstructed) return mpl_fail(c, MPL_ERR_STATE, "energy before reconstruction");
  MPL_TRY(upload_mats(c));
  MPL_TRY(ensure_partials(c));
  const int64_t ncell = (int64_t)c->ncell_alloc(), nnode = (int64_t)c->nnode_alloc();
  const double inv4dx = 0.25 * c->inv_dx;
  double* pc = partial_slot(c, 0);
  double* pe = partial_slot(c, 1);
  double* pg = partial_slot(c, 2);
  if (want_grad) {
    MPL_TRY(mpl_ensure(c, c->Qc, 8 * 9 * ncell));
    MPL_TRY(mpl_ensure(c, c->g, 8 * 3 * nnode));
    MPL_LAUNCH(c, k_energy_cells<true>, c->n_cblk, 64, v, nnode, P<int>(c->c_nbr_node),
               P<double>(c->Vk), P<double>(c->Sk), sgen(c), ncell, c->nmat, c->dt, inv4dx, P<double>(c->Qc), pc, P<MatParams>(c->matbuf));
    MPL_LAUNCH(c, k_energy_nodes<true>, c->n_nblk, 64, v, P<double>(c->vhat), P<double>(c->mi),
               P<uint8_t>(c->flags), P<int>(c->n_nbr_cell), P<double>(c->Qc), ncell, nnode, c->dt,
               inv4dx, P<double>(c->g), pe, pg);
    // with no scalar wanted (vertex block descent needs the gradient only)
    // skip the reduction and the host synchronisation
    if (!energy && !gnorm2) return MPL_OK;
    MPL_LAUNCH(c, k_reduce<RED_PLAIN>, 1, 1024, pc, c->n_cblk, pe, c->n_nblk, pg, c->n_nblk,
               c->dscal(), 0);
  } else {
    MPL_LAUNCH(c, k_energy_cells<false>, c->n_cblk, 64, v, nnode, P<int>(c->c_nbr_node),
               P<double>(c->Vk), P<double>(c->Sk), sgen(c), ncell, c->nmat, c->dt, inv4dx, (double*)nullptr, pc, P<MatParams>(c->matbuf));
    MPL_LAUNCH(c, k_energy_nodes<false>, c->n_nblk, 64, v, P<double>(c->vhat), P<double>(c->mi),
               P<uint8_t>(c->flags), P<int>(c->n_nbr_cell), (const double*)nullptr, ncell, nnode,
               c->dt, inv4dx, (double*)nullptr, pe, (double*)nullptr);
    MPL_LAUNCH(c, k_reduce<RED_PLAIN>, 1, 1024, pc, c->n_cblk, pe, c->n_nblk, pe, 0, c->dscal(), 0);
  }
  MPL_TRY(mpl_sync_scalars(c));
  if (energy) *energy = c->hscal.red[0] + c->hscal.red[1];
  if (gnorm2) *gnorm2 = c->hscal.red[2];
  return MPL_OK;
}

// Tangent layout per cell block for several materials in FP32: factored
// (1) when every cell of the block holds at most one material (V_{c,k} > 0 for
// at most one k), dense (0) otherwise; part[cb] = the block's factored cells.
__global__ __launch_bounds__(64) void k_tan_format(const double* __restrict__ Vk, int64_t ncell, int K,
                                                   const uint64_t* __restrict__ cmask,
                                                   uint8_t* __restrict__ cfmt, int32_t* __restrict__ part) {
  const int cb = blockIdx.x, l = threadIdx.x;
  const int64_t ci = (int64_t)cb * MPL_BC + l;
  const uint64_t m = cmask[cb];
  int cnt = 0;
  if ((m >> l) & 1ull)
    for (int k = 0; k < K; ++k) cnt += Vk[k * ncell + ci] != 0.0 ? 1 : 0;
  const bool fact = !__any(cnt > 1);
  if (l == 0) {
    cfmt[cb] = fact ? 1 : 0;
    part[cb] = fact ? __popcll(m) : 0;
  }
}

// Sum of n int32 values by one workgroup in a fixed order into *out.
__global__ __launch_bounds__(1024) void k_sum_i32(const int32_t* __restrict__ a, int n, int32_t* __restrict__ out) {
  __shared__ int32_t sh[16];
  const int t = threadIdx.x;
  int32_t acc = 0;
  for (int i = t; i < n; i += 1024) acc += a[i];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((t & 63) == 0) sh[t >> 6] = acc;
  __syncthreads();
  if (t == 0) {
    int32_t s = 0;
    for (int k = 0; k < 16; ++k) s += sh[k];
    *out = s;
  }
}

mpl_status mpl_stage_tangent(mpl_ctx* c, const double* v, int precision) {
  if (!c->reconstructed) return mpl_fail(c, MPL_ERR_STATE, "tangent before reconstruction");
  MPL_TRY(upload_mats(c));
  const int64_t ncell = (int64_t)c->ncell_alloc(), nnode = (int64_t)c->nnode_alloc();
  const double inv4dx = 0.25 * c->inv_dx;
  MPL_TRY(mpl_ensure(c, c->D, 8 * 3 * nnode));
  const int64_t ntan = (int64_t)c->hscal.n_tan_cells + 64;
  const uint64_t* cm = P<uint64_t>(c->cmask);
  const int32_t* co = P<int32_t>(c->coff);
  // FP32 layouts: with one material the tangent is stored factored (37
  // entries per cell, 25 of them read by the Hessian-vector product, 12
  // Jacobi-diagonal sums); with several materials each cell block is
  // factored when none of its cells holds two materials, dense (45 entries)
  // otherwise, in blocks of 45 slots per cell.  With block-Jacobi the
  // factored cells' 12 off-diagonal node-block sums go to Aoff.
  const bool fp32 = precision == MPL_F32 && c->factored_enabled;
  const bool fact = fp32 && c->nmat == 1;
  const bool mixed = fp32 && c->nmat > 1;
  const bool bj = c->opts.precond == MPL_PRECOND_BLOCK_JACOBI;
  c->tan_factored = fact;
  c->tan_mixed = mixed;
  const uint8_t* fmt = nullptr;
  if (mixed) {
    MPL_TRY(mpl_ensure(c, c->cfmt, (size_t)c->n_cblk + 64));
    MPL_TRY(mpl_ensure(c, c->fcnt, 4 * ((size_t)c->n_cblk + 64)));
    MPL_LAUNCH(c, k_tan_format, c->n_cblk, 64, P<double>(c->Vk), ncell, c->nmat, cm, P<uint8_t>(c->cfmt),
               P<int32_t>(c->fcnt));
    MPL_LAUNCH(c, k_sum_i32, 1, 1024, P<int32_t>(c->fcnt), c->n_cblk, &c->dscal()->n_fact_cells);
    fmt = P<uint8_t>(c->cfmt);
  }
  if ((fact || mixed) && bj) MPL_TRY(mpl_ensure(c, c->Aoff, 4 * MPL_TAN_OFF * ntan));
  float* aoff = (fact || mixed) && bj ? P<float>(c->Aoff) : nullptr;
  if (precision == MPL_F32) {
    MPL_TRY(mpl_ensure(c, c->Abar32, 4 * (fact ? MPL_TAN_FACT : MPL_TAN_DENSE) * ntan));
    MPL_TRY(mpl_ensure(c, c->Dt, 4 * 3 * nnode));
    MPL_TRY(mpl_ensure(c, c->mt, 4 * nnode));
#define MPL_TAN_LAUNCH(FA, MI, AO)                                                                    \
  MPL_LAUNCH(c, (k_tangent<float, FA, MI>), c->n_cblk, 64, v, nnode, P<int>(c->c_nbr_node),           \
             P<double>(c->Vk), P<double>(c->Sk), sgen(c), ncell, c->nmat, c->dt, inv4dx, cm, co,     \
             P<float>(c->Abar32), &c->dscal()->err, P<MatParams>(c->matbuf), AO, fmt);               \
  MPL_LAUNCH(c, (k_diag<float, FA, MI>), c->n_nblk, 64, P<float>(c->Abar32), cm, co, P<double>(c->mi), \
             P<uint8_t>(c->flags), P<int>(c->n_nbr_cell), nnode, inv4dx, P<double>(c->D),            \
             P<float>(c->Dt), P<float>(c->mt), fmt)
    if (fact) {
      MPL_TAN_LAUNCH(true, false, aoff);
    } else if (mixed) {
      MPL_TAN_LAUNCH(false, true, aoff);
    } else {
      MPL_TAN_LAUNCH(false, false, (float*)nullptr);
    }
#undef MPL_TAN_LAUNCH
  } else {
    MPL_TRY(mpl_ensure(c, c->Abar64, 8 * MPL_TAN_DENSE * ntan));
    MPL_LAUNCH(c, (k_tangent<double, false, false>), c->n_cblk, 64, v, nnode, P<int>(c->c_nbr_node),
               P<double>(c->Vk), P<double>(c->Sk), sgen(c), ncell, c->nmat, c->dt, inv4dx, cm, co,
               P<double>(c->Abar64), &c->dscal()->err, P<MatParams>(c->matbuf), (double*)nullptr,
               (const uint8_t*)nullptr);
    MPL_TRY(mpl_ensure(c, c->Dt, 8 * 3 * nnode));
    MPL_TRY(mpl_ensure(c, c->mt, 8 * nnode));
    MPL_LAUNCH(c, (k_diag<double, false, false>), c->n_nblk, 64, P<double>(c->Abar64), cm, co, P<double>(c->mi),
               P<uint8_t>(c->flags), P<int>(c->n_nbr_cell), nnode, inv4dx, P<double>(c->D),
               P<double>(c->Dt), P<double>(c->mt), (const uint8_t*)nullptr);
  }
  c->bj_built = false;
  if (bj) {
    MPL_TRY(mpl_ensure(c, c->Bj, 8 * 6 * nnode));
    if (precision == MPL_F32) {
      MPL_TRY(mpl_ensure(c, c->Bjt, 4 * 6 * nnode));
#define MPL_BJ_LAUNCH(FA, MI, AO)                                                                        \
  MPL_LAUNCH(c, (k_block_diag<float, FA, MI>), c->n_nblk, 64, P<float>(c->Abar32), cm, co, P<double>(c->mi), \
             P<uint8_t>(c->flags), P<int>(c->n_nbr_cell), nnode, inv4dx, P<double>(c->Bj), P<float>(c->Bjt), \
             (const float*)AO, &c->dscal()->err, fmt)
      if (fact) {
        MPL_BJ_LAUNCH(true, false, aoff);
      } else if (mixed) {
        MPL_BJ_LAUNCH(false, true, aoff);
      } else {
        MPL_BJ_LAUNCH(false, false, nullptr);
      }
#undef MPL_BJ_LAUNCH
    } else {
      MPL_TRY(mpl_ensure(c, c->Bjt, 8 * 6 * nnode));
      MPL_LAUNCH(c, (k_block_diag<double, false, false>), c->n_nblk, 64, P<double>(c->Abar64), cm, co, P<double>(c->mi),
                 P<uint8_t>(c->flags), P<int>(c->n_nbr_cell), nnode, inv4dx, P<double>(c->Bj), P<double>(c->Bjt), (const double*)nullptr,
                 &c->dscal()->err, (const uint8_t*)nullptr);
    }
    // the node blocks are read by every CG iteration: check them once here
    MPL_TRY(mpl_sync_scalars(c));
    if (c->hscal.err & 128)
      return mpl_fail(c, MPL_ERR_NONFINITE, "a 3x3 node block of the Newton matrix is not positive definite");
    c->bj_built = true;
  }
  c->tangent_built = true;
  ++c->tangent_serial;
  c->tangent_precision = precision;
  return MPL_OK;
}

static hipEvent_t next_event_in(std::vector<hipEvent_t>& pool, int& used) {
  if (used >= (int)pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    pool.push_back(e);
  }
  return pool[used++];
}
static hipEvent_t next_event(mpl_ctx* c) { return next_event_in(c->hv_events, c->hv_event_used); }
// Reads the elapsed times of the recorded event pairs (products and CG
// updates) into the per-solve totals.
static mpl_status flush_hv_events(mpl_ctx* c) {
  if (c->hv_event_used == 0 && c->up_event_used == 0) return MPL_OK;
  MPL_HIP(c, hipStreamSynchronize(c->stream));
  for (int i = 0; i + 1 < c->hv_event_used; i += 2) {
    float ms = 0.f;
    MPL_HIP(c, hipEventElapsedTime(&ms, c->hv_events[i], c->hv_events[i + 1]));
    c->hv_ms_total += ms;
    c->hv_calls += 1;
  }
  for (int i = 0; i + 1 < c->up_event_used; i += 2) {
    float ms = 0.f;
    MPL_HIP(c, hipEventElapsedTime(&ms, c->up_events[i], c->up_events[i + 1]));
    c->up_ms_total += ms;
    c->up_calls += 1;
  }
  c->hv_event_used = 0;
  c->up_event_used = 0;
  return MPL_OK;
}

template <class T> static DevBuf& abar_buf(mpl_ctx* c) { return c->Abar32; }
template <> DevBuf& abar_buf<double>(mpl_ctx* c) { return c->Abar64; }
template <class T> static DevBuf& pieces_buf(mpl_ctx* c) { return c->Y32; }
template <> DevBuf& pieces_buf<double>(mpl_ctx* c) { return c->Y64; }
template <class T> static DevBuf& pvec_buf(mpl_ctx* c) { return c->p32; }
template <> DevBuf& pvec_buf<double>(mpl_ctx* c) { return c->p64; }

// The fused cell-block product: own and halo node pieces of K p (and, with
// dot, the per-block partial sums of p^T K p), timed with HIP events when
// time_kernels is 1 (every launch) or 2 (one iteration's product per CG
// chunk).
template <class T>
static mpl_status hv_pieces(mpl_ctx* c, const T* p, bool dot, T* out = nullptr) {
  const int64_t ncell = (int64_t)c->ncell_alloc(), nnode = (int64_t)c->nnode_alloc();
  if (!out) {
    DevBuf& pieces = pieces_buf<T>(c);
    MPL_TRY(mpl_ensure(c, pieces, sizeof(T) * 6 * ncell));
    out = P<T>(pieces);
  }
  T* Hown = out;
  T* Hhalo = Hown + 3 * ncell;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->opts.time_kernels == 1 || (c->opts.time_kernels == 2 && c->hv_sample)) {
    if (c->hv_event_used + 2 > 4096) MPL_TRY(flush_hv_events(c));
    e0 = next_event(c);
    e1 = next_event(c);
    if (e0) MPL_HIP(c, hipEventRecord(e0, c->stream));
  }
  const T inv4 = (T)(0.25 * c->inv_dx);
  const int grid = (((c->n_cblk + 3) / 4 + 7) / 8) * 8;
#define MPL_HV_LAUNCH(DOT, FACT, MIX, PART, SCAL)                                                       \
  MPL_LAUNCH(c, (k_hv_fused<T, DOT, FACT, MIX>), grid, 256, p, nnode, P<int>(c->c_nbr_node),     \
             P<T>(abar_buf<T>(c)), P<uint64_t>(c->cmask), P<int32_t>(c->coff), ncell, c->n_cblk, inv4, \
             Hown, Hhalo, PART, SCAL, (const uint8_t*)(MIX ? c->cfmt.p : nullptr))
  const bool fact = c->tan_factored;
  const bool mixed = c->tan_mixed && sizeof(T) == 4;
  if (dot && fact) MPL_HV_LAUNCH(true, true, false, partial_slot(c, 0), (const SolverScalars*)c->dscal());
  else if (dot && mixed) MPL_HV_LAUNCH(true, false, true, partial_slot(c, 0), (const SolverScalars*)c->dscal());
  else if (dot) MPL_HV_LAUNCH(true, false, false, partial_slot(c, 0), (const SolverScalars*)c->dscal());
  else if (fact) MPL_HV_LAUNCH(false, true, false, (double*)nullptr, (const SolverScalars*)nullptr);
  else if (mixed) MPL_HV_LAUNCH(false, false, true, (double*)nullptr, (const SolverScalars*)nullptr);
  else MPL_HV_LAUNCH(false, false, false, (double*)nullptr, (const SolverScalars*)nullptr);
#undef MPL_HV_LAUNCH
  if (e1) MPL_HIP(c, hipEventRecord(e1, c->stream));
  return MPL_OK;
}

// u, Hu in block layout, precision of the stored tangent.
mpl_status mpl_stage_hv(mpl_ctx* c, const void* u, void* Hu, int precision, bool dot) {
  if (!c->tangent_built || c->tangent_precision != precision)
    return mpl_fail(c, MPL_ERR_STATE, "Hv needs a tangent built in the same precision");
  const int64_t ncell = (int64_t)c->ncell_alloc(), nnode = (int64_t)c->nnode_alloc();
  MPL_TRY(ensure_partials(c));
  if (precision == MPL_F32) {
    MPL_TRY(hv_pieces<float>(c, (const float*)u, dot));
    const float* Hown = P<float>(c->Y32);
    MPL_LAUNCH(c, k_hv_combine<float>, c->n_nblk, 64, (const float*)u, P<double>(c->mi),
               P<uint8_t>(c->flags), P<int>(c->n_nbr_cell), Hown, Hown + 3 * ncell, ncell, nnode,
               (float*)Hu);
  } else {
    MPL_TRY(hv_pieces<double>(c, (const double*)u, dot));
    const double* Hown = P<double>(c->Y64);
    MPL_LAUNCH(c, k_hv_combine<double>, c->n_nblk, 64, (const double*)u, P<double>(c->mi),
               P<uint8_t>(c->flags), P<int>(c->n_nbr_cell), Hown, Hown + 3 * ncell, ncell, nnode,
               (double*)Hu);
  }
  return MPL_OK;
}

mpl_status mpl_mask_free_nodes(mpl_ctx* c, void* u, int is_f32) {
  const int64_t nnode = (int64_t)c->nnode_alloc();
  if (is_f32)
    MPL_LAUNCH(c, k_mask_free<float>, (int)((nnode + 255) / 256), 256, (float*)u, P<uint8_t>(c->flags), nnode);
  else
    MPL_LAUNCH(c, k_mask_free<double>, (int)((nnode + 255) / 256), 256, (double*)u, P<uint8_t>(c->flags), nnode);
  return MPL_OK;
}

mpl_status mpl_stage_hv_into(mpl_ctx* c, const void* u, void* Hu, void* pieces, int precision) {
  if (!c->tangent_built || c->tangent_precision != precision)
    return mpl_fail(c, MPL_ERR_STATE, "Hv needs a tangent built in the same precision");
  const int64_t ncell = (int64_t)c->ncell_alloc(), nnode = (int64_t)c->nnode_alloc();
  if (precision == MPL_F32) {
    float* Hown = (float*)pieces;
    MPL_TRY(hv_pieces<float>(c, (const float*)u, false, Hown));
    MPL_LAUNCH(c, k_hv_combine<float>, c->n_nblk, 64, (const float*)u, P<double>(c->mi),
               P<uint8_t>(c->flags), P<int>(c->n_nbr_cell), (const float*)Hown,
               (const float*)Hown + 3 * ncell, ncell, nnode, (float*)Hu);
  } else {
    double* Hown = (double*)pieces;
    MPL_TRY(hv_pieces<double>(c, (const double*)u, false, Hown));
    MPL_LAUNCH(c, k_hv_combine<double>, c->n_nblk, 64, (const double*)u, P<double>(c->mi),
               P<uint8_t>(c->flags), P<int>(c->n_nbr_cell), (const double*)Hown,
               (const double*)Hown + 3 * ncell, ncell, nnode, (double*)Hu);
  }
  return MPL_OK;
}

template <class T>
LevelArrays mpl_level0(const mpl_ctx* c) {
  LevelArrays L;
  L.n_cblk = c->n_cblk;
  L.n_nblk = c->n_nblk;
  L.ncell = (int64_t)c->ncell_alloc();
  L.nnode = (int64_t)c->nnode_alloc();
  L.c_nbr_node = P<int>(c->c_nbr_node);
  L.n_nbr_cell = P<int>(c->n_nbr_cell);
  L.cmask = P<uint64_t>(c->cmask);
  L.coff = P<int32_t>(c->coff);
  L.Abar = sizeof(T) == 4 ? c->Abar32.p : c->Abar64.p;
  L.fact = c->tan_factored && sizeof(T) == 4;
  L.mixed = c->tan_mixed && sizeof(T) == 4;
  L.cfmt = P<uint8_t>(c->cfmt);
  L.mi = P<double>(c->mi);
  L.flags = P<uint8_t>(c->flags);
  L.inv_dx = c->inv_dx;
  return L;
}

template <class T>
mpl_status mpl_level_hv_pieces(mpl_ctx* c, const LevelArrays& L, const T* p, T* pieces,
                               const SolverScalars* s, double* partial) {
  const T inv4 = (T)(0.25 * L.inv_dx);
  const int grid = (((L.n_cblk + 3) / 4 + 7) / 8) * 8;
  T* Hown = pieces;
  T* Hhalo = pieces + 3 * L.ncell;
  const T* A = (const T*)L.Abar;
  const uint8_t* fmt = L.mixed ? L.cfmt : nullptr;
#define MPL_LV_HV(DOT, FACT, MIX)                                                                  \
  MPL_LAUNCH(c, (k_hv_fused<T, DOT, FACT, MIX>), grid, 256, p, L.nnode, L.c_nbr_node, A, L.cmask, \
             L.coff, L.ncell, L.n_cblk, inv4, Hown, Hhalo, partial, s, fmt)
  if (partial) {
    if (L.fact) MPL_LV_HV(true, true, false);
    else if (L.mixed) MPL_LV_HV(true, false, true);
    else MPL_LV_HV(true, false, false);
  } else {
    if (L.fact) MPL_LV_HV(false, true, false);
    else if (L.mixed) MPL_LV_HV(false, false, true);
    else MPL_LV_HV(false, false, false);
  }
#undef MPL_LV_HV
  return MPL_OK;
}

template <class T>
mpl_status mpl_level_diag(mpl_ctx* c, const LevelArrays& L, double* D, T* Dt, T* mt) {
  const T* A = (const T*)L.Abar;
  const double inv4 = 0.25 * L.inv_dx;
  if (L.fact)
    MPL_LAUNCH(c, (k_diag<T, true, false>), L.n_nblk, 64, A, L.cmask, L.coff, L.mi, L.flags,
               L.n_nbr_cell, L.nnode, inv4, D, Dt, mt, L.cfmt);
  else if (L.mixed)
    MPL_LAUNCH(c, (k_diag<T, false, true>), L.n_nblk, 64, A, L.cmask, L.coff, L.mi, L.flags,
               L.n_nbr_cell, L.nnode, inv4, D, Dt, mt, L.cfmt);
  else
    MPL_LAUNCH(c, (k_diag<T, false, false>), L.n_nblk, 64, A, L.cmask, L.coff, L.mi, L.flags,
               L.n_nbr_cell, L.nnode, inv4, D, Dt, mt, L.cfmt);
  return MPL_OK;
}

template LevelArrays mpl_level0<float>(const mpl_ctx*);
template LevelArrays mpl_level0<double>(const mpl_ctx*);
template mpl_status mpl_level_hv_pieces<float>(mpl_ctx*, const LevelArrays&, const float*, float*,
                                               const SolverScalars*, double*);
template mpl_status mpl_level_hv_pieces<double>(mpl_ctx*, const LevelArrays&, const double*, double*,
                                                const SolverScalars*, double*);
template mpl_status mpl_level_diag<float>(mpl_ctx*, const LevelArrays&, double*, float*, float*);
template mpl_status mpl_level_diag<double>(mpl_ctx*, const LevelArrays&, double*, double*, double*);

// Runs PCG iterations in chunks of `check` until the device flag reports
// convergence or breakdown or max_pcg iterations have been launched.  A
// chunk is captured into a HIP graph once and replayed while the buffers and
// sizes it was captured with (key, keyn) are unchanged; iterations past
// convergence are device-side no-ops, so replaying a whole chunk is exact.
// Without graph support the chunk is launched eagerly.  hook (may be null)
// runs on the host after every chunk that leaves the iteration running,
// with the iteration count.
static mpl_status run_chunks(mpl_ctx* c, GraphCache& gc, const void* const key[24], const int keyn[8],
                             int check, const std::function<mpl_status()>& launch_iteration,
                             const std::function<mpl_status(int)>* hook, int expect = 0) {
  // Events recorded inside a captured graph cannot be timed, so products are
  // timed on eager launches: time_kernels 1 runs every iteration eagerly;
  // time_kernels 2 replays check - 1 iterations from the graph and runs the
  // chunk's last iteration eagerly with events around its product.
  const bool sample = c->opts.time_kernels == 2;
  const int ncap = sample ? check - 1 : check;
  bool use_graph = c->graphs_enabled && c->opts.time_kernels != 1 && ncap > 0;
  if (use_graph) {
    bool same = gc.exec != nullptr;
    for (int i = 0; i < 24 && same; ++i) same = gc.key[i] == key[i];
    for (int i = 0; i < 8 && same; ++i) same = gc.keyn[i] == keyn[i];
    if (same && gc.time_mode != c->opts.time_kernels) same = false;
    if (!same) {
      if (gc.exec) (void)hipGraphExecDestroy(gc.exec);
      if (gc.graph) (void)hipGraphDestroy(gc.graph);
      gc.exec = nullptr;
      gc.graph = nullptr;
      // capture on the private stream (nothing runs while capturing)
      bool ok = c->cap_stream != nullptr ||
                hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) == hipSuccess;
      for (int i = 0; i < 2 && ok; ++i)
        ok = c->cap_order[i] != nullptr ||
             hipEventCreateWithFlags(&c->cap_order[i], hipEventDisableTiming) == hipSuccess;
      const hipStream_t user = c->stream;
      if (ok) {
        c->stream = c->cap_stream;
        ok = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
      }
      mpl_status lst = MPL_OK;
      if (ok) {
        for (int k = 0; k < ncap && lst == MPL_OK; ++k) lst = launch_iteration();
        hipGraph_t g = nullptr;
        ok = (hipStreamEndCapture(c->stream, &g) == hipSuccess) && lst == MPL_OK && g != nullptr;
        if (ok) ok = hipGraphInstantiate(&gc.exec, g, nullptr, nullptr, 0) == hipSuccess;
        if (g && !ok) (void)hipGraphDestroy(g);
        if (ok) gc.graph = g;
      }
      c->stream = user;
      (void)hipGetLastError();
      gc.time_mode = c->opts.time_kernels;
      if (!ok) {
        gc.exec = nullptr;
        c->graphs_enabled = false;
        use_graph = false;
      } else {
        for (int i = 0; i < 24; ++i) gc.key[i] = key[i];
        for (int i = 0; i < 8; ++i) gc.keyn[i] = keyn[i];
      }
    }
  }
  // expect: iterations the solve is expected to take at least; chunks that
  // end before it are queued without a poll (without a hook only: a chunk
  // past convergence costs only its no-op launches)
  if (hook) expect = 0;
  int it = 0;
  for (;;) {
    if (use_graph && it + check <= c->opts.max_pcg) {
      // the replay runs on the private stream, ordered after everything
      // queued on the caller's stream and before everything queued after it
      MPL_HIP(c, hipEventRecord(c->cap_order[0], c->stream));
      MPL_HIP(c, hipStreamWaitEvent(c->cap_stream, c->cap_order[0], 0));
      MPL_HIP(c, hipGraphLaunch(gc.exec, c->cap_stream));
      MPL_HIP(c, hipEventRecord(c->cap_order[1], c->cap_stream));
      MPL_HIP(c, hipStreamWaitEvent(c->stream, c->cap_order[1], 0));
      c->graph_replays += 1;
      if (sample) {
        c->hv_sample = true;
        const mpl_status lst = launch_iteration();
        c->hv_sample = false;
        MPL_TRY(lst);
      }
      it += check;
    } else {
      // the timed iteration's position rotates from chunk to chunk so that
      // the samples cover the update kernel's iteration-dependent work (dx
      // every second, x every eighth iteration) evenly
      const int pos = (int)(c->sample_rot++ % (uint32_t)check);
      for (int k = 0; k < check && it < c->opts.max_pcg; ++k, ++it) {
        c->hv_sample = k == pos;
        const mpl_status lst = launch_iteration();
        c->hv_sample = false;
        MPL_TRY(lst);
      }
    }
    if (it < expect && it < c->opts.max_pcg) continue;
    MPL_TRY(mpl_sync_scalars(c));
    if (c->opts.time_kernels) MPL_TRY(flush_hv_events(c));
    if (c->hscal.done != 0 || it >= c->opts.max_pcg) break;
    if (hook) MPL_TRY((*hook)(it));
  }
  if (c->opts.time_kernels) MPL_TRY(flush_hv_events(c));
  return MPL_OK;
}

// Jacobi-PCG on H x = b over free DOFs (b, x block layout FP64).  Per
// iteration: fused product (p^T K p partials), alpha, update (x, r and the
// assembled Hp), beta / convergence, new direction (p^T M p partials).
// Iterations past convergence are no-ops on the device, so the host polls
// the done flag only every pcg_check_every iterations.
template <class T>
static mpl_status pcg_impl(mpl_ctx* c, const double* b, double* x, int* iters, double* rel,
                           const std::function<mpl_status(int)>* hook = nullptr,
                           bool hook_reads_x = false, const double* x0 = nullptr) {
  const int64_t ncell = (int64_t)c->ncell_alloc(), nnode = (int64_t)c->nnode_alloc();
  MPL_TRY(ensure_partials(c));
  MPL_TRY(mpl_ensure(c, c->r, 8 * 3 * nnode));
  DevBuf& pb_ = pvec_buf<T>(c);
  MPL_TRY(mpl_ensure(c, pb_, sizeof(T) * 3 * nnode));
  MPL_TRY(mpl_ensure(c, pieces_buf<T>(c), sizeof(T) * 6 * ncell));
  T* p = P<T>(pb_);
  const T* Hown = P<T>(pieces_buf<T>(c));
  const T* Hhalo = Hown + 3 * ncell;
  SolverScalars* s = c->dscal();
  double* pk = partial_slot(c, 0);
  double* pa = partial_slot(c, 1);
  double* pb = partial_slot(c, 2);
  double* pm = partial_slot(c, 3);
  const int nwg = (c->n_nblk + 3) / 4;
  if (c->cg_single) {
    // single-reduction form (see k_cg_step)
    MPL_TRY(mpl_ensure(c, c->cg_u, sizeof(T) * 3 * nnode));
    MPL_TRY(mpl_ensure(c, c->cg_s, sizeof(T) * 3 * nnode));
    MPL_TRY(mpl_ensure(c, c->cg_dx, sizeof(T) * 3 * nnode));
    T* u = P<T>(c->cg_u);
    T* sv = P<T>(c->cg_s);
    T* dx = P<T>(c->cg_dx);
    const int nflush = (int)((3 * nnode + 255) / 256);
    const int ngrp = (c->n_cblk + 3) / 4;
    const int nred = cg_red_groups(std::max(nwg, ngrp));
    if (!c->cg_red.p) {
      MPL_TRY(mpl_ensure(c, c->cg_red, sizeof(CgRed)));
      MPL_LAUNCH(c, k_cg_red_zero, 1, 64, P<CgRed>(c->cg_red));
    }
    CgRed* red = P<CgRed>(c->cg_red);
    // Jacobi (inverse diagonal) or block-Jacobi (inverted node blocks)
    const bool bj = c->opts.precond == MPL_PRECOND_BLOCK_JACOBI;
    if (bj && !c->bj_built) return mpl_fail(c, MPL_ERR_STATE, "block-Jacobi blocks not built with the tangent");
    const T* pre = bj ? P<T>(c->Bjt) : P<T>(c->Dt);
    auto* kinit = bj ? &k_cg_init<T, true> : &k_cg_init<T, false>;
    auto* kwarm = bj ? &k_cg_init_warm<T, true> : &k_cg_init_warm<T, false>;
    auto* kstep = bj ? &k_cg_step<T, true> : &k_cg_step<T, false>;
    if (x0) {
      MPL_LAUNCH(c, k_cg_prep<T>, (int)((nnode + 255) / 256), 256, x0, P<uint8_t>(c->flags), nnode, u);
      MPL_TRY(hv_pieces<T>(c, u, false));
      MPL_LAUNCH(c, kwarm, nwg, 256, b, x0, Hown, Hhalo, P<int>(c->n_nbr_cell), ncell,
                 pre, P<T>(c->mt), P<uint8_t>(c->flags), nnode, c->n_nblk, x, dx, P<double>(c->r),
                 u, p, sv, pa, pb, pm, s);
    } else {
      MPL_LAUNCH(c, kinit, nwg, 256, b, pre, P<T>(c->mt), P<uint8_t>(c->flags), nnode,
                 c->n_nblk, x, dx, P<double>(c->r), u, p, sv, pa, pb, pm, s);
    }
    MPL_TRY(hv_pieces<T>(c, u, true));
    MPL_LAUNCH(c, k_reduce_cg<true>, nred, 256, pa, pb, pm, nwg, pk, ngrp, red, s);
    MPL_LAUNCH(c, k_set_tol, 1, 1, s, c->opts.pcg_rtol * c->opts.pcg_rtol);
    const int check = std::max(1, c->opts.pcg_check_every);
    auto launch_iteration = [&]() -> mpl_status {
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (c->opts.time_kernels == 1 || (c->opts.time_kernels == 2 && c->hv_sample)) {
        if (c->up_event_used + 2 > 4096) MPL_TRY(flush_hv_events(c));
        e0 = next_event_in(c->up_events, c->up_event_used);
        e1 = next_event_in(c->up_events, c->up_event_used);
        if (e0) MPL_HIP(c, hipEventRecord(e0, c->stream));
      }
      MPL_LAUNCH(c, kstep, nwg, 256, u, p, sv, Hown, Hhalo, P<int>(c->n_nbr_cell), ncell,
                 P<T>(c->mt), pre, P<uint8_t>(c->flags), nnode, c->n_nblk, x, dx, P<double>(c->r),
                 pa, pb, pm, s);
      if (e1) MPL_HIP(c, hipEventRecord(e1, c->stream));
      MPL_TRY(hv_pieces<T>(c, u, true));
      MPL_LAUNCH(c, k_reduce_cg<false>, nred, 256, pa, pb, pm, nwg, pk, ngrp, red, s);
      return MPL_OK;
    };
    const void* key[24] = {x,           p,           c->r.p,          pre,
                           abar_buf<T>(c).p, c->partials.p, pieces_buf<T>(c).p, c->mt.p,
                           c->flags.p,  c->n_nbr_cell.p, c->c_nbr_node.p, c->scal.p,
                           c->cmask.p,  c->coff.p,   u,               sv,
                           dx,          c->cg_red.p};
    const int keyn[8] = {c->n_cblk, c->n_nblk, check, (int)bj, 0, 0, (int)c->tan_factored + 2 * (int)c->tan_mixed, 2};
    // a hook that reads x sees the full solution vector (flushing changes
    // the rounding of x, so it is done only for such hooks)
    std::function<mpl_status(int)> flushed_hook;
    if (hook && hook_reads_x) {
      flushed_hook = [&](int it) -> mpl_status {
        MPL_LAUNCH(c, k_cg_flush<T>, nflush, 256, x, dx, p, nnode, (int64_t)c->n_nblk * MPL_BC, s);
        return (*hook)(it);
      };
    }
    MPL_TRY(run_chunks(c, c->pcg_cache[2], key, keyn, check, launch_iteration,
                       hook ? (hook_reads_x ? &flushed_hook : hook) : nullptr, c->pcg_expect));
    MPL_LAUNCH(c, k_cg_flush<T>, nflush, 256, x, dx, p, nnode, (int64_t)c->n_nblk * MPL_BC, s);
    if (iters) *iters = c->hscal.iters;
    if (rel) *rel = c->hscal.bnorm2 > 0.0 ? std::sqrt(c->hscal.rr / c->hscal.bnorm2) : 0.0;
    if (c->hscal.done == 2 && c->hscal.iters == 0 && c->hscal.bnorm2 > 0.0)
      return mpl_fail(c, MPL_ERR_NONFINITE, "PCG breakdown (u.Hu <= 0 or not finite)");
    return MPL_OK;
  }
  MPL_LAUNCH(c, k_pcg_init<T>, nwg, 256, b, P<T>(c->Dt), P<T>(c->mt), P<uint8_t>(c->flags),
             nnode, c->n_nblk, x, P<double>(c->r), p, pa, pb, pm);
  MPL_LAUNCH(c, k_reduce<RED_PCG_INIT>, 1, 1024, pa, nwg, pb, nwg, pb, 0, s, 0);
  MPL_LAUNCH(c, k_set_tol, 1, 1, s, c->opts.pcg_rtol * c->opts.pcg_rtol);
  const int check = std::max(1, c->opts.pcg_check_every);
  auto launch_iteration = [&]() -> mpl_status {
    MPL_TRY(hv_pieces<T>(c, p, true));
    MPL_LAUNCH(c, k_reduce<RED_ALPHA>, 1, 1024, pk, (c->n_cblk + 3) / 4, pm, nwg, pm, 0, s, 0);
    MPL_LAUNCH(c, k_pcg_update<T>, nwg, 256, p, Hown, Hhalo, P<int>(c->n_nbr_cell), ncell,
               P<T>(c->mt), P<T>(c->Dt), P<uint8_t>(c->flags), nnode, c->n_nblk, x,
               P<double>(c->r), pa, pb, s, (T*)nullptr);
    MPL_LAUNCH(c, k_reduce<RED_BETA>, 1, 1024, pa, nwg, pb, nwg, pb, 0, s, 0);
    MPL_LAUNCH(c, k_pcg_direction<T>, nwg, 256, P<double>(c->r), P<T>(c->Dt), P<T>(c->mt),
               P<uint8_t>(c->flags), nnode, c->n_nblk, p, pm, s);
    return MPL_OK;
  };
  const void* key[24] = {x,           p,           c->r.p,          c->Dt.p,
                         abar_buf<T>(c).p, c->partials.p, pieces_buf<T>(c).p, c->mt.p,
                         c->flags.p,  c->n_nbr_cell.p, c->c_nbr_node.p, c->scal.p,
                         c->cmask.p,  c->coff.p};
  const int keyn[8] = {c->n_cblk, c->n_nblk, check, 0, 0, 0, (int)c->tan_factored + 2 * (int)c->tan_mixed, 0};
  MPL_TRY(run_chunks(c, c->pcg_cache[0], key, keyn, check, launch_iteration, hook));
  if (iters) *iters = c->hscal.iters;
  if (rel) *rel = c->hscal.bnorm2 > 0.0 ? std::sqrt(c->hscal.rr / c->hscal.bnorm2) : 0.0;
  if (c->hscal.done == 2 && c->hscal.iters == 0 && c->hscal.bnorm2 > 0.0)
    return mpl_fail(c, MPL_ERR_NONFINITE, "PCG breakdown (p.Hp <= 0 or not finite)");
  return MPL_OK;
}

// Flexible CG preconditioned by the network (Polak-Ribiere beta, so that a
// preconditioner that varies from iteration to iteration still yields a
// descent method), falling back to Jacobi when z.r <= 0, on NaN/Inf, or when
// |r| drops by less than 10% over 10 iterations.  Per iteration: fused
// product, alpha, update (x, r, q = Hp stored), convergence/stagnation
// check, network input, network forward, z.r and z.q, beta, new direction.
template <class T>
static mpl_status pcg_learned(mpl_ctx* c, const double* b, double* x, int* iters, double* rel,
                              const std::function<mpl_status(int)>* hook = nullptr,
                              const double* x0 = nullptr) {
  if (!c->nn || !c->nn->ready) return mpl_fail(c, MPL_ERR_STATE, "learned preconditioner has no weights");
  NNState& nn = *c->nn;
  const int64_t ncell = (int64_t)c->ncell_alloc(), nnode = (int64_t)c->nnode_alloc();
  MPL_TRY(ensure_partials(c));
  MPL_TRY(mpl_ensure(c, c->r, 8 * 3 * nnode));
  DevBuf& pb_ = pvec_buf<T>(c);
  DevBuf& qb_ = (sizeof(T) == 4) ? c->q32 : c->q64;
  MPL_TRY(mpl_ensure(c, pb_, sizeof(T) * 3 * nnode));
  MPL_TRY(mpl_ensure(c, qb_, sizeof(T) * 3 * nnode));
  MPL_TRY(mpl_ensure(c, pieces_buf<T>(c), sizeof(T) * 6 * ncell));
  MPL_TRY(nn_prepare_box(c, false));
  MPL_TRY(nn_set_dref(c, P<double>(c->D)));
  T* p = P<T>(pb_);
  T* q = P<T>(qb_);
  const T* Hown = P<T>(pieces_buf<T>(c));
  const T* Hhalo = Hown + 3 * ncell;
  SolverScalars* s = c->dscal();
  const double* s2 = &s->s2;
  nn.skip = &s->nn_off;
  double* pk = partial_slot(c, 0);
  double* pa = partial_slot(c, 1);
  double* pb = partial_slot(c, 2);
  double* pm = partial_slot(c, 3);
  const int nwg = (c->n_nblk + 3) / 4;
  const NetOut net{(const uint16_t*)nn.act.p + nn.t_out, nn.box[0], nn.box[1], nn.box[2],
                   nn_inv_free_dofs(c)};
  const double* r = P<double>(c->r);
  const double* D = P<double>(c->D);
  auto precondition = [&](const T* qv) -> mpl_status {
    MPL_TRY(nn_stage_features(c, r, D, s2));
    MPL_TRY(nn_forward(c, nn));
    MPL_LAUNCH(c, k_fpcg_dots<T>, nwg, 256, r, qv, D, P<uint8_t>(c->flags), P<int4>(c->ncoord), nnode,
               c->n_nblk, net, pa, pb, s);
    MPL_LAUNCH(c, k_reduce<RED_FBETA>, 1, 1024, pa, nwg, pb, nwg, pb, 0, s, 0);
    MPL_LAUNCH(c, k_fpcg_direction<T>, nwg, 256, r, D, P<double>(c->mi), P<uint8_t>(c->flags),
               P<int4>(c->ncoord), nnode, c->n_nblk, net, p, pm, s);
    return MPL_OK;
  };
  if (x0) {
    // start from x0 (the q buffer holds x0 in the tangent's precision for its product)
    MPL_LAUNCH(c, k_cg_prep<T>, (int)((nnode + 255) / 256), 256, x0, P<uint8_t>(c->flags), nnode, q);
    MPL_TRY(hv_pieces<T>(c, q, false));
    MPL_LAUNCH(c, k_fpcg_init_warm<T>, nwg, 256, b, x0, (const T*)q, Hown, Hhalo, P<int>(c->n_nbr_cell), ncell,
               P<T>(c->mt), D, P<uint8_t>(c->flags), nnode, c->n_nblk, x, P<double>(c->r), pa, pb, pk);
    MPL_LAUNCH(c, k_reduce<RED_FINIT_WARM>, 1, 1024, pa, nwg, pb, nwg, pk, nwg, s, 0);
  } else {
    MPL_LAUNCH(c, k_fpcg_init, nwg, 256, b, D, P<uint8_t>(c->flags), nnode, c->n_nblk, x, P<double>(c->r),
               pa, pb);
    MPL_LAUNCH(c, k_reduce<RED_FINIT>, 1, 1024, pa, nwg, pb, nwg, pb, 0, s, 0);
  }
  MPL_LAUNCH(c, k_set_tol, 1, 1, s, c->opts.pcg_rtol * c->opts.pcg_rtol);
  mpl_status st = precondition((const T*)nullptr);
  const int check = std::max(1, c->opts.pcg_check_every);
  auto launch_iteration = [&]() -> mpl_status {
    MPL_TRY(hv_pieces<T>(c, p, true));
    MPL_LAUNCH(c, k_reduce<RED_ALPHA>, 1, 1024, pk, (c->n_cblk + 3) / 4, pm, nwg, pm, 0, s, 0);
    MPL_LAUNCH(c, k_pcg_update<T>, nwg, 256, p, Hown, Hhalo, P<int>(c->n_nbr_cell), ncell,
               P<T>(c->mt), P<T>(c->Dt), P<uint8_t>(c->flags), nnode, c->n_nblk, x, P<double>(c->r), pa, pb,
               s, q);
    // pa = sum Dinv r^2, pb = r.r
    MPL_LAUNCH(c, k_reduce<RED_FCHECK>, 1, 1024, pb, nwg, pa, nwg, pa, 0, s, 0);
    return precondition(q);
  };
  if (st == MPL_OK) {
    const void* key[24] = {x,           p,           c->r.p,          c->D.p,
                           abar_buf<T>(c).p, c->partials.p, pieces_buf<T>(c).p, c->mi.p,
                           c->flags.p,  c->n_nbr_cell.p, c->c_nbr_node.p, c->scal.p,
                           q,           nn.act.p,    nn.wsw.p,        c->ncoord.p,
                           c->cmask.p,  c->coff.p,   nn.params.p,     c->nmap.p,
                           c->Dt.p,     c->mt.p};
    const int keyn[8] = {c->n_cblk, c->n_nblk, check, nn.box[0], nn.box[1], nn.box[2], (int)c->tan_factored + 2 * (int)c->tan_mixed, 1};
    st = run_chunks(c, c->pcg_cache[1], key, keyn, check, launch_iteration, hook);
  }
  nn.skip = nullptr;
  MPL_TRY(st);
  c->fallbacks_total += c->hscal.fallbacks;
  if (iters) *iters = c->hscal.iters;
  if (rel) *rel = c->hscal.bnorm2 > 0.0 ? std::sqrt(c->hscal.rr / c->hscal.bnorm2) : 0.0;
  if (c->hscal.done == 2 && c->hscal.iters == 0 && c->hscal.bnorm2 > 0.0)
    return mpl_fail(c, MPL_ERR_NONFINITE, "PCG breakdown (p.Hp <= 0 or not finite)");
  return MPL_OK;
}

// Buffers of the energy-norm loss kernels (online training and
// mpl_precond_energy_loss).
template <class T>
static mpl_status online_buffers(mpl_ctx* c, int n_losses) {
  NNState& nn = *c->nn;
  const int64_t ncell = (int64_t)c->ncell_alloc(), nnode = (int64_t)c->nnode_alloc();
  MPL_TRY(nn_prepare_box(c, true));
  MPL_TRY(ensure_partials(c));
  MPL_TRY(mpl_ensure(c, c->ozt, sizeof(T) * 3 * nnode));
  MPL_TRY(mpl_ensure(c, c->ohz, sizeof(T) * 3 * nnode));
  MPL_TRY(mpl_ensure(c, c->ogr, sizeof(double) * 3 * nnode));
  MPL_TRY(mpl_ensure(c, c->opieces, sizeof(T) * 6 * ncell));
  MPL_TRY(mpl_ensure(c, nn.tmp, sizeof(double) * (n_losses + 64) + 2 * sizeof(double) * (c->n_nblk + 64)));
  return nn_set_dref(c, P<double>(c->D));
}

// r^T Dinv r of the residual r (block layout) into red[0].
static mpl_status online_rdr(mpl_ctx* c, const double* r) {
  const int nwg = (c->n_nblk + 3) / 4;
  double* p4 = partial_slot(c, 4);
  MPL_LAUNCH(c, k_online_rdr, nwg, 256, r, P<double>(c->D), P<uint8_t>(c->flags), (int64_t)c->nnode_alloc(),
             c->n_nblk, p4);
  MPL_LAUNCH(c, k_reduce<RED_PLAIN>, 1, 1024, p4, nwg, p4, 0, p4, 0, c->dscal(), 0);
  return MPL_OK;
}

// Energy-norm loss of z = preconditioner(r) (the network output staged in
// the activation arena or, with jacobi = 1, z = Dinv r): z into ozt, H z into
// ohz, the loss into *loss (device) and dL/do into ogr.  Needs red[0] =
// r^T Dinv r (online_rdr); uses red[1..3] and partial slots 4-5.
template <class T>
static mpl_status online_loss(mpl_ctx* c, const double* r, int jacobi, double* loss) {
  NNState& nn = *c->nn;
  const int64_t ncell = (int64_t)c->ncell_alloc(), nnode = (int64_t)c->nnode_alloc();
  SolverScalars* s = c->dscal();
  const int nwg = (c->n_nblk + 3) / 4;
  double* p4 = partial_slot(c, 4);
  double* p5 = partial_slot(c, 5);
  const double* D = P<double>(c->D);
  T* z = P<T>(c->ozt);
  T* hz = P<T>(c->ohz);
  const NetOut net{(const uint16_t*)nn.act.p + nn.t_out, nn.box[0], nn.box[1], nn.box[2],
                   nn_inv_free_dofs(c)};
  MPL_LAUNCH(c, k_online_z<T>, nwg, 256, r, D, P<uint8_t>(c->flags), P<int4>(c->ncoord), nnode,
             c->n_nblk, net, &s->red[0], z, jacobi);
  MPL_TRY(hv_pieces<T>(c, z, false, P<T>(c->opieces)));
  const T* Hown = P<T>(c->opieces);
  MPL_LAUNCH(c, k_hv_combine<T>, c->n_nblk, 64, (const T*)z, P<double>(c->mi), P<uint8_t>(c->flags),
             P<int>(c->n_nbr_cell), Hown, Hown + 3 * ncell, ncell, nnode, hz);
  MPL_LAUNCH(c, k_online_dots<T>, nwg, 256, r, (const T*)z, (const T*)hz, P<uint8_t>(c->flags), nnode,
             c->n_nblk, p4, p5);
  MPL_LAUNCH(c, k_reduce<RED_PLAIN>, 1, 1024, p4, nwg, p5, nwg, p5, 0, s, 1);
  MPL_LAUNCH(c, k_online_grad<T>, nwg, 256, r, (const T*)hz, D, P<uint8_t>(c->flags), nnode, c->n_nblk,
             nn_inv_free_dofs(c), (const double*)&s->red[0], P<double>(c->ogr), loss);
  return MPL_OK;
}

// Online training: `steps` Adam steps of the network on the energy-norm
// loss of the current residual c->r under the current tangent.  Runs
// between PCG chunks; touches neither the iteration's vectors nor its
// control scalars (its reductions use red[0..3] and partial slots 4-6).
template <class T>
static mpl_status online_train(mpl_ctx* c) {
  NNState& nn = *c->nn;
  MPL_TRY(online_buffers<T>(c, c->online_steps));
  const int32_t* saved_skip = nn.skip;
  const int saved_tk = c->opts.time_kernels;
  nn.skip = nullptr;
  c->opts.time_kernels = 0;
  const double* r = P<double>(c->r);
  const double* D = P<double>(c->D);
  // losses go after the dref partials in nn.tmp
  double* losses = P<double>(nn.tmp) + 2 * (c->n_nblk + 64);
  mpl_status st = MPL_OK;
  auto run = [&]() -> mpl_status {
    MPL_TRY(online_rdr(c, r));
    // reference: the same loss for the Jacobi preconditioner
    MPL_TRY(online_loss<T>(c, r, 1, losses + c->online_steps));
    for (int k = 0; k < c->online_steps; ++k) {
      MPL_TRY(nn_stage_features(c, r, D, &c->dscal()->red[0]));
      MPL_TRY(nn_forward(c, nn));
      MPL_TRY(online_loss<T>(c, r, 0, losses + k));
      MPL_TRY(nn_stage_output_grad(c, P<double>(c->ogr)));
      MPL_TRY(nn_backward_update(c, nn, c->online_lr));
    }
    return MPL_OK;
  };
  st = run();
  nn.skip = saved_skip;
  c->opts.time_kernels = saved_tk;
  MPL_TRY(st);
  double first = 0.0, ref = 0.0;
  MPL_HIP(c, hipMemcpyAsync(&first, losses, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  MPL_HIP(c, hipMemcpyAsync(&ref, losses + c->online_steps, sizeof(double), hipMemcpyDeviceToHost,
                            c->stream));
  MPL_HIP(c, hipStreamSynchronize(c->stream));
  c->online_done += c->online_steps;
  if (std::isfinite(first) && std::isfinite(ref)) {
    c->online_loss_sum += first;
    c->online_ref_sum += ref;
    c->online_loss_n += 1;
  }
  return MPL_OK;
}

// Energy-norm loss of the learned preconditioner on a given residual r
// (block layout in c->r): the network output o is the caller's box tensor
// (FP32, rounded to BF16 like the network's own output) or, when o_box is
// NULL, the network's forward on the features of r.  Loss and Jacobi loss
// to the host, dL/do (block layout) in c->ogr.
template <class T>
static mpl_status energy_loss_on(mpl_ctx* c, const float* o_box, double* loss, double* loss_jacobi) {
  NNState& nn = *c->nn;
  MPL_TRY(online_buffers<T>(c, 2));
  const int32_t* saved_skip = nn.skip;
  nn.skip = nullptr;
  const double* r = P<double>(c->r);
  double* losses = P<double>(nn.tmp) + 2 * (c->n_nblk + 64);
  auto run = [&]() -> mpl_status {
    MPL_TRY(online_rdr(c, r));
    MPL_TRY(online_loss<T>(c, r, 1, losses + 1));
    if (o_box) {
      MPL_TRY(nn_stage_output_f32(c, o_box));
    } else {
      MPL_TRY(nn_stage_features(c, r, P<double>(c->D), &c->dscal()->red[0]));
      MPL_TRY(nn_forward(c, nn));
    }
    return online_loss<T>(c, r, 0, losses);
  };
  mpl_status st = run();
  nn.skip = saved_skip;
  MPL_TRY(st);
  double h[2] = {0.0, 0.0};
  MPL_HIP(c, hipMemcpyAsync(h, losses, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  MPL_HIP(c, hipStreamSynchronize(c->stream));
  if (loss) *loss = h[0];
  if (loss_jacobi) *loss_jacobi = h[1];
  return MPL_OK;
}

// Training pairs for the learned preconditioner: solve H x* = b to
// collect_rtol with Jacobi PCG, then run the solver's own iteration (Jacobi
// PCG, or flexible CG with the current network when the learned
// preconditioner is selected, so that later pairs follow the residuals the
// trained solver meets) and record (r_k, x* - x_k) every collect_every
// iterations until the sample store is full.  x* is left in c->xstar.
template <class T>
static mpl_status collect_pairs(mpl_ctx* c, const double* b, int* iters) {
  const int64_t nnode = (int64_t)c->nnode_alloc();
  MPL_TRY(mpl_ensure(c, c->xstar, 8 * 3 * nnode));
  MPL_TRY(mpl_ensure(c, c->x, 8 * 3 * nnode));
  MPL_TRY(nn_prepare_box(c, true));
  MPL_TRY(nn_set_dref(c, P<double>(c->D)));
  const mpl_solver_opts saved = c->opts;
  c->opts.pcg_rtol = c->collect_rtol;
  c->opts.pcg_check_every = c->collect_every;
  double rel = 0.0;
  mpl_status st = pcg_impl<T>(c, b, P<double>(c->xstar), iters, &rel);
  NNSampleStore& store = nn_samples(c);
  const bool learned = saved.precond == MPL_PRECOND_LEARNED;
  // sum Dinv r^2 of the current residual: r.z in Jacobi PCG, s2 in flexible CG
  const double* s2 = learned ? &c->dscal()->s2 : &c->dscal()->rz;
  std::function<mpl_status(int)> hook = [&](int) -> mpl_status {
    if (store.count >= store.capacity) return MPL_OK;
    return nn_record_sample(c, P<double>(c->r), P<double>(c->x), P<double>(c->xstar), P<double>(c->D), s2);
  };
  if (st == MPL_OK && store.count < store.capacity) {
    // stop the replay at the exact solve's length
    c->opts.max_pcg = std::max(1, std::min(c->opts.max_pcg, *iters));
    st = learned ? pcg_learned<T>(c, b, P<double>(c->x), nullptr, nullptr, &hook)
                 : pcg_impl<T>(c, b, P<double>(c->x), nullptr, nullptr, &hook, true);
  }
  c->opts = saved;
  return st;
}

// z = P(r) with the learned preconditioner at the current tangent's
// diagonal (block layout, FP64).  Uses the solver's r, x and scalars as scratch.
mpl_status mpl_stage_precond_apply(mpl_ctx* c, const double* rin, double* z) {
  if (!c->tangent_built) return mpl_fail(c, MPL_ERR_STATE, "preconditioner before tangent");
  if (!c->nn || !c->nn->ready) return mpl_fail(c, MPL_ERR_STATE, "learned preconditioner has no weights");
  NNState& nn = *c->nn;
  const int64_t nnode = (int64_t)c->nnode_alloc();
  MPL_TRY(ensure_partials(c));
  MPL_TRY(mpl_ensure(c, c->r, 8 * 3 * nnode));
  MPL_TRY(mpl_ensure(c, c->x, 8 * 3 * nnode));
  MPL_TRY(nn_prepare_box(c, false));
  MPL_TRY(nn_set_dref(c, P<double>(c->D)));
  SolverScalars* s = c->dscal();
  const int nwg = (c->n_nblk + 3) / 4;
  double* pa = partial_slot(c, 1);
  double* pb = partial_slot(c, 2);
  MPL_LAUNCH(c, k_fpcg_init, nwg, 256, rin, P<double>(c->D), P<uint8_t>(c->flags), nnode, c->n_nblk,
             P<double>(c->x), P<double>(c->r), pa, pb);
  MPL_LAUNCH(c, k_reduce<RED_FINIT>, 1, 1024, pa, nwg, pb, nwg, pb, 0, s, 0);
  MPL_TRY(nn_stage_features(c, P<double>(c->r), P<double>(c->D), &s->s2));
  nn.skip = nullptr;
  MPL_TRY(nn_forward(c, nn));
  const NetOut net{(const uint16_t*)nn.act.p + nn.t_out, nn.box[0], nn.box[1], nn.box[2],
                   nn_inv_free_dofs(c)};
  MPL_LAUNCH(c, k_precond_z, nwg, 256, P<double>(c->r), P<double>(c->D), P<uint8_t>(c->flags),
             P<int4>(c->ncoord), nnode, c->n_nblk, net, s, z);
  return MPL_OK;
}

mpl_status mpl_stage_pcg(mpl_ctx* c, const double* b, double* x, int* iters, double* rel,
                         const double* x0) {
  if (!c->tangent_built) return mpl_fail(c, MPL_ERR_STATE, "PCG before tangent");
  // online training of the network at the first chunk boundary and then
  // every online_every iterations
  const bool online = c->online_every > 0 && c->online_steps > 0 && c->nn && c->nn->ready;
  int last = -1;
  std::function<mpl_status(int)> hook = [&](int it) -> mpl_status {
    if (last >= 0 && it - last < c->online_every) return MPL_OK;
    last = it;
    return c->tangent_precision == MPL_F32 ? online_train<float>(c) : online_train<double>(c);
  };
  const std::function<mpl_status(int)>* h = online ? &hook : nullptr;
  if (c->opts.precond == MPL_PRECOND_LEARNED) {
    if (c->tangent_precision == MPL_F32) return pcg_learned<float>(c, b, x, iters, rel, h, x0);
    return pcg_learned<double>(c, b, x, iters, rel, h, x0);
  }
  if (c->opts.precond == MPL_PRECOND_MULTIGRID) return mpl_stage_pcg_mg(c, b, x, iters, rel, x0);
  // (a warm start applies to the single-reduction Jacobi loop)
  if (!c->cg_single) x0 = nullptr;
  if (c->tangent_precision == MPL_F32) return pcg_impl<float>(c, b, x, iters, rel, h, false, x0);
  return pcg_impl<double>(c, b, x, iters, rel, h, false, x0);
}

namespace {
// out = 2 x1 - x2 (dense node arrays)
__global__ void k_extrapolate(const double* __restrict__ x1, const double* __restrict__ x2,
                              double* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = 2.0 * x1[i] - x2[i];
}
// Galerkin start: per node block, the partial sums over free components of
// w_k . (H w_l) for k <= l (packed row by row) and then of w_k . b, for up to
// GAL_MAX vectors (block layout, vector k at w + k * 3 nnode).
#define GAL_MAX 3
static_assert(GAL_MAX <= mpl_ctx::kHist, "the Galerkin basis comes from the history ring");
#define GAL_SUMS (GAL_MAX * (GAL_MAX + 1) / 2 + GAL_MAX)
template <class T>
__global__ __launch_bounds__(64) void k_gram(const double* __restrict__ w, const T* __restrict__ y,
                                             const double* __restrict__ b, const uint8_t* __restrict__ flags,
                                             int64_t nnode, int nv, int n_nblk, double* __restrict__ part) {
  const int nb = blockIdx.x, l = threadIdx.x;
  const int64_t ni = (int64_t)nb * MPL_BC + l;
  const uint8_t fl = flags[ni];
  const int64_t n3 = 3 * nnode;
  const int ng = nv * (nv + 1) / 2;
  double acc[GAL_SUMS];
#pragma unroll
  for (int q = 0; q < GAL_SUMS; ++q) acc[q] = 0.0;
  if (fl & MPL_NODE_FREE_ALL) {
    for (int a = 0; a < 3; ++a) {
      if (!mpl_free(fl, a)) continue;
      const int64_t i = a * nnode + ni;
      double wv[GAL_MAX], yv[GAL_MAX];
#pragma unroll
      for (int k = 0; k < GAL_MAX; ++k) {
        wv[k] = k < nv ? w[k * n3 + i] : 0.0;
        yv[k] = k < nv ? (double)y[k * n3 + i] : 0.0;
      }
      const double bv = b[i];
      int q = 0;
#pragma unroll
      for (int k = 0; k < GAL_MAX; ++k)
#pragma unroll
        for (int m = k; m < GAL_MAX; ++m) {
          acc[q] += wv[k] * yv[m];
          ++q;
        }
#pragma unroll
      for (int k = 0; k < GAL_MAX; ++k) acc[q + k] += wv[k] * bv;
    }
  }
  // store the nv-vector layout: pairs (k <= m < nv) row by row, then w_k . b
  int q = 0, o = 0;
#pragma unroll
  for (int k = 0; k < GAL_MAX; ++k)
#pragma unroll
    for (int m = k; m < GAL_MAX; ++m) {
      const double sum = wave_sum(acc[q]);
      if (k < nv && m < nv) {
        if (l == 0) part[(int64_t)o * n_nblk + nb] = sum;
        ++o;
      }
      ++q;
    }
#pragma unroll
  for (int k = 0; k < GAL_MAX; ++k) {
    const double sum = wave_sum(acc[q + k]);
    if (k < nv && l == 0) part[(int64_t)(ng + k) * n_nblk + nb] = sum;
  }
}
// fixed-order sums of the rows of k_gram partials, one 1024-thread
// workgroup per row (grid = number of rows)
__global__ __launch_bounds__(1024) void k_gram_reduce(const double* __restrict__ part, int n,
                                                      double* __restrict__ out) {
  __shared__ double sh[16];
  const int t = threadIdx.x, q = blockIdx.x;
  double v = 0.0;
  for (int i = t; i < n; i += 1024) v += part[(int64_t)q * n + i];
  v = wave_sum(v);
  if ((t & 63) == 0) sh[t >> 6] = v;
  __syncthreads();
  if (t == 0) {
    double r = 0.0;
    for (int w = 0; w < 16; ++w) r += sh[w];
    out[q] = r;
  }
}
// u = (T) w (block layout, 3 components)
template <class T>
__global__ void k_to_prec(const double* __restrict__ w, T* __restrict__ u, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) u[i] = (T)w[i];
}
struct GalCoef {
  double c[GAL_MAX];
};
// x0 = sum_k c_k w_k on the free components, 0 elsewhere (block layout)
__global__ __launch_bounds__(64) void k_lincomb(const double* __restrict__ w, GalCoef cf, int nv,
                                                const uint8_t* __restrict__ flags, int64_t nnode,
                                                double* __restrict__ x0) {
  const int64_t ni = (int64_t)blockIdx.x * MPL_BC + threadIdx.x;
  const uint8_t fl = flags[ni];
  const int64_t n3 = 3 * nnode;
  for (int a = 0; a < 3; ++a) {
    const int64_t i = a * nnode + ni;
    double v = 0.0;
    for (int k = 0; k < nv; ++k) v += cf.c[k] * w[k * n3 + i];
    x0[i] = mpl_free(fl, a) ? v : 0.0;
  }
}
// out = 3 x1 - 3 x2 + x3 (dense node arrays)
__global__ void k_extrapolate2(const double* __restrict__ x1, const double* __restrict__ x2,
                               const double* __restrict__ x3, double* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = 3.0 * (x1[i] - x2[i]) + x3[i];
}
}  // namespace

// warm_start 4: the start x0 = W c that minimises the energy norm of the
// error over the span W of earlier solutions (the last GAL_MAX of this
// Newton index, newest first; five instead of three gained nothing, adding
// the other indices' solutions cost iterations), from
// (W^T H W) c = W^T b with H the current tangent.  A vector whose Cholesky
// pivot falls below 1e-10 of the largest diagonal entry is left out; *used
// stays false when no vector is left.
template <class T>
static mpl_status galerkin_start(mpl_ctx* c, const DevBuf* const* hist, int nv, const double* b,
                                 double* x0, bool* used) {
  *used = false;
  nv = std::min(nv, GAL_MAX);
  if (nv <= 0) return MPL_OK;
  const int64_t nnode = (int64_t)c->nnode_alloc(), n3 = 3 * nnode;
  const int ng = nv * (nv + 1) / 2, nq = ng + nv;
  MPL_TRY(mpl_ensure(c, c->gal_w, 8 * (size_t)GAL_MAX * n3));
  MPL_TRY(mpl_ensure(c, c->gal_u, sizeof(T) * n3));
  MPL_TRY(mpl_ensure(c, c->gal_y, sizeof(T) * (size_t)GAL_MAX * n3));
  MPL_TRY(mpl_ensure(c, c->gal_part, 8 * ((size_t)GAL_SUMS * c->n_nblk + GAL_SUMS)));
  double* w = P<double>(c->gal_w);
  T* y = P<T>(c->gal_y);
  for (int k = 0; k < nv; ++k) {
    MPL_TRY(mpl_dense_to_block_nodes(c, hist[k]->p, w + k * n3, 3, 0));
    MPL_LAUNCH(c, k_to_prec<T>, (int)((n3 + 255) / 256), 256, (const double*)(w + k * n3), P<T>(c->gal_u), n3);
    MPL_TRY(mpl_stage_hv(c, c->gal_u.p, y + k * n3, c->tangent_precision, false));
  }
  double* part = P<double>(c->gal_part);
  double* sums = part + (size_t)GAL_SUMS * c->n_nblk;
  MPL_LAUNCH(c, k_gram<T>, c->n_nblk, 64, (const double*)w, (const T*)y, b, P<uint8_t>(c->flags), nnode, nv,
             c->n_nblk, part);
  MPL_LAUNCH(c, k_gram_reduce, nq, 1024, (const double*)part, c->n_nblk, sums);
  double h[GAL_SUMS];
  MPL_HIP(c, hipMemcpyAsync(h, sums, sizeof(double) * nq, hipMemcpyDeviceToHost, c->stream));
  MPL_HIP(c, hipStreamSynchronize(c->stream));
  // G_km from the packed upper triangle (the product is symmetric up to
  // rounding; the upper entry is used for both)
  double G[GAL_MAX][GAL_MAX];
  {
    int q = 0;
    for (int k = 0; k < nv; ++k)
      for (int m = k; m < nv; ++m, ++q) G[k][m] = G[m][k] = h[q];
  }
  double dmax = 0.0;
  for (int k = 0; k < nv; ++k)
    if (std::isfinite(G[k][k])) dmax = std::max(dmax, G[k][k]);
  if (!(dmax > 0.0)) return MPL_OK;
  // Cholesky over the kept vectors, in order
  int keep[GAL_MAX], m = 0;
  double L[GAL_MAX][GAL_MAX] = {};
  for (int k = 0; k < nv; ++k) {
    double row[GAL_MAX];
    bool ok = true;
    for (int j = 0; j < m && ok; ++j) {
      double v = G[k][keep[j]];
      for (int t = 0; t < j; ++t) v -= row[t] * L[j][t];
      row[j] = v / L[j][j];
      ok = std::isfinite(row[j]);
    }
    if (!ok) continue;
    double d = G[k][k];
    for (int t = 0; t < m; ++t) d -= row[t] * row[t];
    if (!(d > 1e-10 * dmax) || !std::isfinite(d)) continue;
    for (int t = 0; t < m; ++t) L[m][t] = row[t];
    L[m][m] = std::sqrt(d);
    keep[m++] = k;
  }
  if (m == 0) return MPL_OK;
  double z[GAL_MAX], cm[GAL_MAX];
  for (int i = 0; i < m; ++i) {
    double v = h[ng + keep[i]];
    for (int t = 0; t < i; ++t) v -= L[i][t] * z[t];
    z[i] = v / L[i][i];
  }
  for (int i = m - 1; i >= 0; --i) {
    double v = z[i];
    for (int t = i + 1; t < m; ++t) v -= L[t][i] * cm[t];
    cm[i] = v / L[i][i];
  }
  GalCoef cf;
  for (int k = 0; k < GAL_MAX; ++k) cf.c[k] = 0.0;
  for (int i = 0; i < m; ++i) cf.c[keep[i]] = cm[i];
  MPL_LAUNCH(c, k_lincomb, c->n_nblk, 64, (const double*)w, cf, nv, P<uint8_t>(c->flags), nnode, x0);
  *used = true;
  return MPL_OK;
}

// One Anderson step of the fixed-point plasticity iteration (see the
// plastic_anderson option): history push, least-squares fit, candidate
// iterate in aa_tmp with its plastic base, energy and gradient (in c->g).
// *accepted tells whether the candidate is taken; when it is not, the
// history restarts from the pair just pushed.
static mpl_status anderson_step(mpl_ctx* c, const double* v, const double* vt, double gn_k, bool* accepted,
                                double* E_out, double* gn2_out) {
  *accepted = false;
  const int m = c->opts.plastic_anderson;
  const int64_t nnode = (int64_t)c->nnode_alloc();
  const int64_t n3 = 3 * nnode;
  // push: drop the oldest pair when m + 1 are stored
  if (c->aa_n == m + 1) {
    DevBuf v0 = c->aa_v[0], f0 = c->aa_f[0];
    for (int k = 0; k < m; ++k) {
      c->aa_v[k] = c->aa_v[k + 1];
      c->aa_f[k] = c->aa_f[k + 1];
    }
    c->aa_v[m] = v0;
    c->aa_f[m] = f0;
    c->aa_n = m;
  }
  const int slot = c->aa_n;
  MPL_TRY(mpl_ensure(c, c->aa_v[slot], 8 * n3));
  MPL_TRY(mpl_ensure(c, c->aa_f[slot], 8 * n3));
  MPL_LAUNCH(c, k_aa_push, (int)((n3 + 255) / 256), 256, v, vt, P<double>(c->aa_v[slot]), P<double>(c->aa_f[slot]), n3);
  c->aa_n += 1;
  const int nv = c->aa_n;
  if (nv < 2) return MPL_OK;
  // Gram matrix of the stored updates
  const int nwg = (c->n_nblk + 3) / 4;
  const int npair = nv * (nv + 1) / 2;
  MPL_TRY(mpl_ensure(c, c->aa_part, 8 * ((size_t)npair * nwg + 64)));
  MPL_TRY(mpl_ensure(c, c->aa_tmp, 8 * n3));
  AAVecs fv{};
  for (int k = 0; k < nv; ++k) fv.p[k] = P<double>(c->aa_f[k]);
  MPL_LAUNCH(c, k_aa_gram, nwg, 256, fv, nv, P<uint8_t>(c->flags), nnode, c->n_nblk, P<double>(c->aa_part), nwg);
  MPL_LAUNCH(c, k_aa_reduce, 1, 1024, P<double>(c->aa_part), npair, nwg, P<double>(c->aa_part) + (size_t)npair * nwg);
  double g[15];
  MPL_HIP(c, hipMemcpyAsync(g, P<double>(c->aa_part) + (size_t)npair * nwg, 8 * npair, hipMemcpyDeviceToHost,
                            c->stream));
  MPL_HIP(c, hipStreamSynchronize(c->stream));
  double G[5][5];
  for (int i = 0, q = 0; i < nv; ++i)
    for (int j = i; j < nv; ++j, ++q) G[i][j] = G[j][i] = g[q];
  // normal equations of min |f_k - dF gamma|, dF_j = f_{j+1} - f_j
  const int h = nv - 1, k = nv - 1;
  double M[4][4], r[4], tr = 0.0;
  for (int i = 0; i < h; ++i) {
    for (int j = 0; j < h; ++j) M[i][j] = G[i + 1][j + 1] - G[i + 1][j] - G[i][j + 1] + G[i][j];
    r[i] = G[i + 1][k] - G[i][k];
    tr += M[i][i];
  }
  if (!(tr > 0.0) || !std::isfinite(tr)) return MPL_OK;
  for (int i = 0; i < h; ++i) M[i][i] += 1e-12 * tr / h;
  // Cholesky solve of the small symmetric positive definite system
  double L[4][4] = {}, y[4], gam[4];
  for (int i = 0; i < h; ++i) {
    for (int j = 0; j <= i; ++j) {
      double s2 = M[i][j];
      for (int q = 0; q < j; ++q) s2 -= L[i][q] * L[j][q];
      if (i == j) {
        if (!(s2 > 0.0)) return MPL_OK;
        L[i][i] = std::sqrt(s2);
      } else {
        L[i][j] = s2 / L[j][j];
      }
    }
  }
  for (int i = 0; i < h; ++i) {
    double s2 = r[i];
    for (int q = 0; q < i; ++q) s2 -= L[i][q] * y[q];
    y[i] = s2 / L[i][i];
  }
  for (int i = h - 1; i >= 0; --i) {
    double s2 = y[i];
    for (int q = i + 1; q < h; ++q) s2 -= L[q][i] * gam[q];
    gam[i] = s2 / L[i][i];
  }
  // v_new = v_k + f_k - sum_j gamma_j (dv_j + df_j) as a combination of the
  // stored v and f
  AAVecs vec{};
  AACoef co{};
  for (int i = 0; i < nv; ++i) {
    vec.p[i] = P<double>(c->aa_v[i]);
    vec.p[nv + i] = P<double>(c->aa_f[i]);
  }
  co.a[k] += 1.0;
  co.a[nv + k] += 1.0;
  for (int j = 0; j < h; ++j) {
    co.a[j + 1] -= gam[j];
    co.a[j] += gam[j];
    co.a[nv + j + 1] -= gam[j];
    co.a[nv + j] += gam[j];
  }
  MPL_LAUNCH(c, k_aa_combine, (int)((n3 + 255) / 256), 256, vec, co, 2 * nv, P<double>(c->aa_tmp), n3);
  MPL_TRY(plastic_base(c, P<double>(c->aa_tmp)));
  double E = 0.0, gn2 = 0.0;
  MPL_TRY(mpl_stage_energy(c, P<double>(c->aa_tmp), true, &E, &gn2));
  if (std::isfinite(E) && std::isfinite(gn2) && std::sqrt(gn2) < gn_k) {
    *accepted = true;
    *E_out = E;
    *gn2_out = gn2;
    return MPL_OK;
  }
  // restart the history from the pair just pushed (buffers swapped, never
  // shared, so each stays owned by one slot)
  std::swap(c->aa_v[0], c->aa_v[k]);
  std::swap(c->aa_f[0], c->aa_f[k]);
  c->aa_n = 1;
  return MPL_OK;
}

mpl_status mpl_stage_solve(mpl_ctx* c, mpl_stats* st) {
  if (!c->reconstructed) return mpl_fail(c, MPL_ERR_STATE, "solve before reconstruction");
  const int64_t nnode = (int64_t)c->nnode_alloc();
  MPL_TRY(mpl_ensure(c, c->dir, 8 * 3 * nnode));
  MPL_TRY(mpl_ensure(c, c->vt, 8 * 3 * nnode));
  MPL_TRY(mpl_ensure(c, c->g, 8 * 3 * nnode));
  MPL_TRY(mpl_ensure(c, c->x, 8 * 3 * nnode));
  MPL_TRY(ensure_partials(c));
  double* v = P<double>(c->v);
  // energy rounding scale sum V (mu + |lambda|) for the line-search allowance
  MPL_LAUNCH(c, k_escale, c->n_cblk, 64, P<double>(c->Vk), (int64_t)c->ncell_alloc(), c->nmat,
             partial_slot(c, 3), P<MatParams>(c->matbuf));
  MPL_LAUNCH(c, k_reduce<RED_PLAIN>, 1, 1024, partial_slot(c, 3), c->n_cblk, partial_slot(c, 3), 0,
             partial_slot(c, 3), 0, c->dscal(), 4);
  MPL_TRY(mpl_sync_scalars(c));
  const double escale = c->hscal.red[4];
  double E = 0.0, gn2 = 0.0;
  if (c->opts.vbd_sweeps > 0) {
    // vertex block descent instead of Newton-PCG (Sec. 5, VBD)
    MPL_TRY(mpl_stage_energy(c, v, true, &E, &gn2));
    if (!std::isfinite(E)) return mpl_fail(c, MPL_ERR_DOMAIN, "initial state outside the model domain");
    const double g0v = std::sqrt(gn2);
    for (int sw = 0; sw < c->opts.vbd_sweeps; ++sw)
      for (int color = 0; color < 8; ++color) {
        MPL_TRY(mpl_stage_energy(c, v, true, nullptr, nullptr));
        MPL_TRY(mpl_stage_tangent(c, v, MPL_F64));
        MPL_LAUNCH(c, k_vbd_nodes, c->n_nblk, 64, P<double>(c->Abar64), P<uint64_t>(c->cmask),
                   P<int32_t>(c->coff), P<double>(c->mi), P<uint8_t>(c->flags), P<int>(c->n_nbr_cell),
                   P<int4>(c->ncoord), nnode, 0.25 * c->inv_dx, color, P<double>(c->g), v,
                   &c->dscal()->err);
      }
    MPL_TRY(mpl_stage_energy(c, v, true, &E, &gn2));
    if (c->hscal.err & 64) {
      c->solved = false;
      return mpl_fail(c, MPL_ERR_NONFINITE, "a vertex block is not positive definite");
    }
    if (st) {
      *st = mpl_stats{};
      st->newton_iters = c->opts.vbd_sweeps;
      st->g0_norm = g0v;
      st->g_norm = std::sqrt(gn2);
      st->energy = E;
    }
    c->solved = std::isfinite(E);
    return c->solved ? MPL_OK : mpl_fail(c, MPL_ERR_NONFINITE, "non-finite energy after the sweeps");
  }
  const bool fixed_point = c->opts.plasticity == MPL_PLASTICITY_FIXED_POINT;
  if (fixed_point) MPL_TRY(plastic_base(c, v));
  MPL_TRY(mpl_stage_energy(c, v, true, &E, &gn2));
  if (!std::isfinite(E)) return mpl_fail(c, MPL_ERR_DOMAIN, "initial state outside the model domain");
  const double g0 = std::sqrt(gn2);
  double gn = g0;
  int pcg_total = 0, ls_total = 0, it = 0;
  int per_newton[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  mpl_status result = MPL_OK;
  c->hv_ms_total = 0.0;
  c->hv_calls = 0;
  c->up_ms_total = 0.0;
  c->up_calls = 0;
  c->graph_replays = 0;
  c->fallbacks_total = 0;
  c->aa_n = 0;  // a new fixed-point iteration
  double gn_prev = gn, eta_prev = c->opts.newton_forcing;
  const double pcg_rtol = c->opts.pcg_rtol;
  for (;; ++it) {
    if (gn == 0.0 || gn <= c->opts.newton_rtol * g0) break;
    if (it >= c->opts.max_newton) {
      result = mpl_fail(c, MPL_ERR_NOT_CONVERGED, "Newton iteration cap reached");
      break;
    }
    // inexact Newton: forcing term of this iteration (Eisenstat-Walker, choice 2)
    double rtol_k = pcg_rtol;
    if (c->opts.newton_forcing > 0.0) {
      double eta = c->opts.newton_forcing;
      if (it > 0) {
        const double q = gn / gn_prev;
        eta = 0.9 * q * q;
        const double guard = 0.9 * eta_prev * eta_prev;
        if (guard > 0.1) eta = std::max(eta, guard);
        eta = std::min(eta, c->opts.newton_forcing);
      }
      eta = std::max(eta, 0.5 * c->opts.newton_rtol * g0 / gn);
      eta_prev = eta;
      rtol_k = std::max(pcg_rtol, eta);
    }
    MPL_TRY(mpl_stage_tangent(c, v, c->opts.hv_precision));
    // b = -g
    MPL_LAUNCH(c, k_neg, (int)((3 * nnode + 255) / 256), 256, P<double>(c->g), P<double>(c->dir),
               3 * nnode);
    int iters = 0;
    double rel = 0.0;
    if (c->collect_every > 0 && c->nn && c->nn->store && c->nn->store->count < c->nn->store->capacity) {
      // collection mode: the exact solution is the Newton direction
      if (c->tangent_precision == MPL_F32) MPL_TRY(collect_pairs<float>(c, P<double>(c->dir), &iters));
      else MPL_TRY(collect_pairs<double>(c, P<double>(c->dir), &iters));
      MPL_HIP(c, hipMemcpyAsync(c->x.p, c->xstar.p, 8 * 3 * nnode, hipMemcpyDeviceToDevice, c->stream));
    } else {
      const double* x0 = nullptr;
      const bool warm = c->opts.warm_start && it < mpl_ctx::kWarm;
      // ring length of the mode: 1 (previous), 2 (linear), 3 (quadratic),
      // GAL_MAX (Galerkin); a change of mode starts the histories afresh
      const int wm = c->opts.warm_start;
      const int len = wm >= 4 ? GAL_MAX : std::max(wm, 1);
      if (len != c->whist_len) {
        for (int j = 0; j < mpl_ctx::kWarm; ++j) c->wcount[j] = c->whead[j] = 0;
        c->whist_len = len;
      }
      const int64_t nd3 = 3 * (int64_t)(c->dims[0] + 1) * (c->dims[1] + 1) * (c->dims[2] + 1);
      auto hist = [&](int k) -> DevBuf& {  // k-th newest solution of this Newton index
        return c->whist[it][((c->whead[it] - k) % len + len) % len];
      };
      if (warm && c->wcount[it] > 0) {
        MPL_TRY(mpl_ensure(c, c->warm_x0, 8 * 3 * nnode));
        const int have = c->wcount[it];
        bool done_x0 = false;
        if (wm == 4) {
          const DevBuf* h[GAL_MAX];
          for (int k = 0; k < have; ++k) h[k] = &hist(k);
          if (c->tangent_precision == MPL_F32)
            MPL_TRY(galerkin_start<float>(c, h, have, P<double>(c->dir), P<double>(c->warm_x0), &done_x0));
          else
            MPL_TRY(galerkin_start<double>(c, h, have, P<double>(c->dir), P<double>(c->warm_x0), &done_x0));
        }
        if (!done_x0) {
          // polynomial extrapolation of the newest solutions: constant, linear
          // (2 x_{n-1} - x_{n-2}) or quadratic (3 x_{n-1} - 3 x_{n-2} + x_{n-3})
          const int order = std::min(have, std::min(std::max(wm, 1), 3));
          if (order == 1) {
            MPL_TRY(mpl_dense_to_block_nodes(c, hist(0).p, c->warm_x0.p, 3, 0));
          } else {
            MPL_TRY(mpl_ensure(c, c->wtmp, 8 * nd3));
            if (order == 2)
              MPL_LAUNCH(c, k_extrapolate, (int)((nd3 + 255) / 256), 256, P<double>(hist(0)),
                         P<double>(hist(1)), P<double>(c->wtmp), nd3);
            else
              MPL_LAUNCH(c, k_extrapolate2, (int)((nd3 + 255) / 256), 256, P<double>(hist(0)),
                         P<double>(hist(1)), P<double>(hist(2)), P<double>(c->wtmp), nd3);
            MPL_TRY(mpl_dense_to_block_nodes(c, c->wtmp.p, c->warm_x0.p, 3, 0));
          }
        }
        x0 = P<double>(c->warm_x0);
      }
      // three quarters of the previous step's count for this Newton index
      // are run before the first convergence poll
      c->pcg_expect = it < 8 ? (3 * c->last_pcg[it]) / 4 : 0;
      c->opts.pcg_rtol = rtol_k;
      const mpl_status pst = mpl_stage_pcg(c, P<double>(c->dir), P<double>(c->x), &iters, &rel, x0);
      c->opts.pcg_rtol = pcg_rtol;
      c->pcg_expect = 0;
      MPL_TRY(pst);
      if (it < 8) c->last_pcg[it] = iters;
      if (warm) {
        // the solution becomes the newest entry of the ring
        c->whead[it] = (c->whead[it] + 1) % len;
        DevBuf& dst = c->whist[it][c->whead[it]];
        MPL_TRY(mpl_ensure(c, dst, 8 * nd3));
        // nodes outside this solve's active blocks start the next one from 0
        MPL_HIP(c, hipMemsetAsync(dst.p, 0, 8 * nd3, c->stream));
        MPL_TRY(mpl_block_to_dense_nodes(c, c->x.p, dst.p, 3, 0));
        c->wcount[it] = std::min(c->wcount[it] + 1, len);
      }
    }
    pcg_total += iters;
    if (it < 8) per_newton[it] = iters;
    // g . x for the Armijo test
    MPL_LAUNCH(c, k_axpy_dot, c->n_nblk, 64, v, P<double>(c->x), 0.0, P<double>(c->g),
               P<uint8_t>(c->flags), nnode, P<double>(c->vt), partial_slot(c, 3));
    MPL_LAUNCH(c, k_reduce<RED_PLAIN>, 1, 1024, partial_slot(c, 3), c->n_nblk, partial_slot(c, 3), 0,
               partial_slot(c, 3), 0, c->dscal(), 4);
    MPL_TRY(mpl_sync_scalars(c));
    const double gtp = c->hscal.red[4];
    const double allowance = 1e-14 * escale + 1e-13 * std::fabs(E);
    double alpha = 1.0, Et = 0.0;
    bool ok = false;
    int ls = 0;
    for (; ls <= c->opts.max_ls; ++ls) {
      MPL_LAUNCH(c, k_axpy_dot, c->n_nblk, 64, v, P<double>(c->x), alpha, (const double*)nullptr,
                 P<uint8_t>(c->flags), nnode, P<double>(c->vt), (double*)nullptr);
      MPL_TRY(mpl_stage_energy(c, P<double>(c->vt), false, &Et, nullptr));
      if (std::isfinite(Et) && Et <= E + c->opts.armijo_c * alpha * gtp + allowance) {
        ok = true;
        break;
      }
      alpha *= 0.5;
    }
    ls_total += ls;
    if (!ok) {
      result = mpl_fail(c, MPL_ERR_LINESEARCH, "no step length passed the line search");
      break;
    }
    bool accel = false;
    if (fixed_point && c->opts.plastic_anderson > 0) {
      // Anderson acceleration: push (v_k, f_k = vt - v_k), fit f_k by the
      // differences of the stored updates, take the extrapolated iterate if
      // its gradient (with its own plastic base) is finite and below |g(v_k)|
      double Eaa = 0.0, gaa2 = 0.0;
      MPL_TRY(anderson_step(c, v, P<double>(c->vt), gn, &accel, &Eaa, &gaa2));
      if (accel) {
        MPL_HIP(c, hipMemcpyAsync(v, c->aa_tmp.p, 8 * 3 * nnode, hipMemcpyDeviceToDevice, c->stream));
        E = Eaa;
        gn2 = gaa2;
      }
    }
    if (!accel) {
      MPL_HIP(c, hipMemcpyAsync(v, c->vt.p, 8 * 3 * nnode, hipMemcpyDeviceToDevice, c->stream));
      // fixed-point plasticity: re-project at the new iterate before its energy
      if (fixed_point) MPL_TRY(plastic_base(c, v));
      MPL_TRY(mpl_stage_energy(c, v, true, &E, &gn2));
    }
    gn_prev = gn;
    gn = std::sqrt(gn2);
    if (!std::isfinite(gn)) {
      result = mpl_fail(c, MPL_ERR_NONFINITE, "gradient is not finite");
      break;
    }
  }
  if (st) {
    st->newton_iters = it;
    st->pcg_iters = pcg_total;
    st->ls_halvings = ls_total;
    st->g0_norm = g0;
    st->g_norm = gn;
    st->energy = E;
    st->hv_ms_total = c->hv_ms_total;
    st->hv_calls = c->hv_calls;
    st->upd_ms_total = c->up_ms_total;
    st->upd_calls = c->up_calls;
    // per free node: reads p, s, Dinv, m and the two product pieces (tangent
    // precision), r (FP64), the flag byte, dx every second and x every eighth
    // iteration; writes p, s, u, r, dx every second and x every eighth
    {
      const double e = c->tangent_precision == MPL_F32 ? 4.0 : 8.0;
      st->upd_model_bytes = (28.0 * e + 55.0) / 3.0 * c->hscal.n_free_dofs;
    }
    st->graph_replays = c->graph_replays;
    st->fallbacks = c->fallbacks_total;
    for (int k = 0; k < 8; ++k) st->pcg_per_newton[k] = per_newton[k];
  }
  c->solved = (result == MPL_OK);
  return result;
}

// ======================================================================
extern "C" {

mpl_status mpl_reconstruct_stretch(mpl_ctx* c) {
  if (!c) return MPL_ERR_INVALID_ARG;
  return mpl_stage_reconstruct(c);
}

mpl_status mpl_energy_grad(mpl_ctx* c, const double* v, double* energy, double* grad) {
  if (!c) return MPL_ERR_INVALID_ARG;
  if (!c->reconstructed) return mpl_fail(c, MPL_ERR_STATE, "energy before reconstruction");
  const int64_t nnode = (int64_t)c->nnode_alloc();
  const double* vb = P<double>(c->v);
  if (v) {
    MPL_TRY(mpl_ensure(c, c->vt, 8 * 3 * nnode));
    MPL_TRY(mpl_dense_to_block_nodes(c, v, c->vt.p, 3, 0));
    vb = P<double>(c->vt);
  }
  double E = 0.0;
  MPL_TRY(mpl_stage_energy(c, vb, grad != nullptr, &E, nullptr));
  if (energy) *energy = E;
  if (grad) MPL_TRY(mpl_block_to_dense_nodes(c, c->g.p, grad, 3, 0));
  return MPL_OK;
}

mpl_status mpl_build_tangent(mpl_ctx* c, const double* v, int32_t precision) {
  if (!c) return MPL_ERR_INVALID_ARG;
  if (precision != MPL_F32 && precision != MPL_F64) return mpl_fail(c, MPL_ERR_INVALID_ARG, "precision");
  if (!c->reconstructed) return mpl_fail(c, MPL_ERR_STATE, "tangent before reconstruction");
  const double* vb = P<double>(c->v);
  if (v) {
    MPL_TRY(mpl_ensure(c, c->vt, 8 * 3 * (int64_t)c->nnode_alloc()));
    MPL_TRY(mpl_dense_to_block_nodes(c, v, c->vt.p, 3, 0));
    vb = P<double>(c->vt);
  }
  return mpl_stage_tangent(c, vb, precision);
}

mpl_status mpl_hv(mpl_ctx* c, const void* u, void* Hu, int32_t precision) {
  if (!c || !u || !Hu) return MPL_ERR_INVALID_ARG;
  if (!c->tangent_built || c->tangent_precision != precision)
    return mpl_fail(c, MPL_ERR_STATE, "mpl_hv needs a tangent built in the same precision");
  const int64_t nnode = (int64_t)c->nnode_alloc();
  const int f32 = precision == MPL_F32;
  DevBuf& bin = f32 ? c->p32 : c->p64;
  DevBuf& bout = f32 ? c->q32 : c->q64;
  MPL_TRY(mpl_ensure(c, bin, (f32 ? 4 : 8) * 3 * nnode));
  MPL_TRY(mpl_ensure(c, bout, (f32 ? 4 : 8) * 3 * nnode));
  MPL_TRY(mpl_dense_to_block_nodes(c, u, bin.p, 3, f32));
  if (f32)
    MPL_LAUNCH(c, k_mask_free<float>, (int)((nnode + 255) / 256), 256, (float*)bin.p,
               P<uint8_t>(c->flags), nnode);
  else
    MPL_LAUNCH(c, k_mask_free<double>, (int)((nnode + 255) / 256), 256, (double*)bin.p,
               P<uint8_t>(c->flags), nnode);
  MPL_TRY(mpl_stage_hv(c, bin.p, bout.p, precision, false));
  MPL_TRY(mpl_block_to_dense_nodes(c, bout.p, Hu, 3, f32));
  if (c->opts.time_kernels) MPL_TRY(flush_hv_events(c));
  return MPL_OK;
}

mpl_status mpl_precond_apply(mpl_ctx* c, const double* r, double* z) {
  if (!c || !r || !z) return MPL_ERR_INVALID_ARG;
  const int64_t nnode = (int64_t)c->nnode_alloc();
  MPL_TRY(mpl_ensure(c, c->dir, 8 * 3 * nnode));
  MPL_TRY(mpl_ensure(c, c->vt, 8 * 3 * nnode));
  MPL_TRY(mpl_dense_to_block_nodes(c, r, c->dir.p, 3, 0));
  MPL_TRY(mpl_stage_precond_apply(c, P<double>(c->dir), P<double>(c->vt)));
  MPL_TRY(mpl_block_to_dense_nodes(c, c->vt.p, z, 3, 0));
  MPL_HIP(c, hipStreamSynchronize(c->stream));
  return MPL_OK;
}

mpl_status mpl_precond_energy_loss(mpl_ctx* c, const double* r, const float* o_box, double* loss,
                                   double* loss_jacobi, double* grad_o) {
  if (!c || !r) return MPL_ERR_INVALID_ARG;
  if (!c->tangent_built) return mpl_fail(c, MPL_ERR_STATE, "energy loss needs a tangent");
  if (!c->nn || !c->nn->ready) return mpl_fail(c, MPL_ERR_STATE, "learned preconditioner has no weights");
  const int64_t nnode = (int64_t)c->nnode_alloc();
  MPL_TRY(mpl_ensure(c, c->r, 8 * 3 * nnode));
  MPL_TRY(mpl_dense_to_block_nodes(c, r, c->r.p, 3, 0));
  if (c->tangent_precision == MPL_F32) MPL_TRY(energy_loss_on<float>(c, o_box, loss, loss_jacobi));
  else MPL_TRY(energy_loss_on<double>(c, o_box, loss, loss_jacobi));
  if (grad_o) MPL_TRY(mpl_block_to_dense_nodes(c, c->ogr.p, grad_o, 3, 0));
  MPL_HIP(c, hipStreamSynchronize(c->stream));
  return MPL_OK;
}

mpl_status mpl_precond_record_pair(mpl_ctx* c, const double* r, const double* x, const double* xstar) {
  if (!c || !r || !x || !xstar) return MPL_ERR_INVALID_ARG;
  if (!c->tangent_built) return mpl_fail(c, MPL_ERR_STATE, "a training pair needs a tangent");
  if (!c->nn || !c->nn->ready) return mpl_fail(c, MPL_ERR_STATE, "learned preconditioner has no weights");
  const int64_t nnode = (int64_t)c->nnode_alloc();
  MPL_TRY(ensure_partials(c));
  MPL_TRY(nn_prepare_box(c, true));
  NNSampleStore& store = nn_samples(c);
  if (store.count >= store.capacity) return mpl_fail(c, MPL_ERR_OOM, "training sample store is full (mpl_precond_reserve)");
  MPL_TRY(mpl_ensure(c, c->r, 8 * 3 * nnode));
  MPL_TRY(mpl_ensure(c, c->x, 8 * 3 * nnode));
  MPL_TRY(mpl_ensure(c, c->xstar, 8 * 3 * nnode));
  MPL_TRY(mpl_dense_to_block_nodes(c, r, c->r.p, 3, 0));
  MPL_TRY(mpl_dense_to_block_nodes(c, x, c->x.p, 3, 0));
  MPL_TRY(mpl_dense_to_block_nodes(c, xstar, c->xstar.p, 3, 0));
  MPL_TRY(nn_set_dref(c, P<double>(c->D)));
  MPL_TRY(online_rdr(c, P<double>(c->r)));
  MPL_TRY(nn_record_sample(c, P<double>(c->r), P<double>(c->x), P<double>(c->xstar), P<double>(c->D),
                           &c->dscal()->red[0]));
  MPL_HIP(c, hipStreamSynchronize(c->stream));
  return MPL_OK;
}

mpl_status mpl_pcg(mpl_ctx* c, const double* b, double* x, int32_t* iters, double* rel_resid) {
  if (!c || !b || !x) return MPL_ERR_INVALID_ARG;
  if (!c->tangent_built) return mpl_fail(c, MPL_ERR_STATE, "mpl_pcg needs a tangent");
  const int64_t nnode = (int64_t)c->nnode_alloc();
  MPL_TRY(mpl_ensure(c, c->dir, 8 * 3 * nnode));
  MPL_TRY(mpl_ensure(c, c->x, 8 * 3 * nnode));
  MPL_TRY(mpl_dense_to_block_nodes(c, b, c->dir.p, 3, 0));
  int it = 0;
  double rel = 0.0;
  MPL_TRY(mpl_stage_pcg(c, P<double>(c->dir), P<double>(c->x), &it, &rel));
  MPL_TRY(mpl_block_to_dense_nodes(c, c->x.p, x, 3, 0));
  if (iters) *iters = it;
  if (rel_resid) *rel_resid = rel;
  return MPL_OK;
}

mpl_status mpl_solve(mpl_ctx* c, double* v_out, mpl_stats* st) {
  if (!c) return MPL_ERR_INVALID_ARG;
  mpl_status s = mpl_stage_solve(c, st);
  if (v_out) MPL_TRY(mpl_block_to_dense_nodes(c, c->v.p, v_out, 3, 0));
  return s;
}

}  // extern "C"
