// Multigrid-preconditioned CG on the incremental potential.  The paper
// names multigrid-preconditioned CG beside plain PCG as an off-the-shelf
// solver of the same potential (Sec. 7, the vertex block descent
// comparison) without defining it; this is the textbook geometric V-cycle
// on the voxel mesh (symmetric, damped-Jacobi smoothing, trilinear
// transfer), with the definitions stated in mpmlite.h ("multigrid"):
//
//   * level l + 1 halves every axis of level l; its cells carry the sum of
//     their eight children's tangents and are multiplied by the same
//     one-point Q1 product (k_hv_fused, dense 45-value layout) with the
//     coarse spacing; coarse masses are the restricted fine masses;
//   * every level lives in the same block-sparse layout as the step's grid
//     (4^3 cell and node blocks, compact ids, neighbour tables), built on
//     the device from the level above: a coarse cell block is active when
//     one of its (at most eight) child cell blocks carries a tangent;
//   * restriction and prolongation are gathers (every coarse node sums its
//     27 fine nodes, every fine node its 1, 2, 4 or 8 coarse nodes), so no
//     two lanes write one value and the sums have a fixed order;
//   * the damping of each level's sweeps comes from power iterations on the
//     device, started from SplitMix64 signs so that the start carries no
//     hourglass pattern.
//
// PCG (Hestenes-Stiefel) keeps x and r in FP64 like the Jacobi solver; the
// cycle runs in the tangent's precision.
#include <algorithm>
#include <cmath>
#include <vector>

#include "mpl_grid.h"

using namespace mpl;

struct MGLevel {
  int dims[3] = {0, 0, 0}, cbd[3] = {0, 0, 0}, nbd[3] = {0, 0, 0};
  double dx = 0.0, inv_dx = 0.0;
  int n_cblk = 0, n_nblk = 0;
  // structure (levels >= 1; level 0 is the context's grid)
  DevBuf cflag, cmap, nflag, nmap, ccoord, ncoord, c_nbr_node, n_nbr_cell, scan;
  DevBuf cmask, ccnt, coff, Abar, mi, flags, D, Dt, mt;
  // cycle vectors in the tangent's precision and the product's pieces
  DevBuf x, b, res, pieces, part;
  double omega = 0.0, lambda = 0.0;
  int64_t ncell() const { return (int64_t)n_cblk * MPL_BC; }
  int64_t nnode() const { return (int64_t)n_nblk * MPL_BC; }
};

struct MGState {
  int nlev = 0;
  MGLevel lev[MPL_MG_MAX_LEVELS];
  // the hierarchy matches this tangent build, precision and options
  int serial = -1, precision = -1, levels_opt = 0;
  double omega_opt = 0.0;
  DevBuf counts;  // int32 scratch: block counts of a level build
  DevBuf pw;      // FP64 scalars of the power iterations, 4 per level
  DevBuf rblk;    // FP64 block-layout input of mpl_mg_apply
  // PCG vectors and partial sums
  DevBuf p, partials;
};

namespace {

// Device view of a level's geometry for the transfer and build kernels.
struct GeoDev {
  int dims[3], cbd[3], nbd[3];
  const int32_t* cmap;  // dense cell-block map (-1 inactive)
  const int32_t* nmap;  // dense node-block map
  const int4* ccoord;
  const int4* ncoord;
  const uint64_t* cmask;
  const double* mi;
  const uint8_t* flags;
};

// compact node slot of level node (x, y, z), -1 when outside the level or in
// an inactive node block
__device__ __forceinline__ int64_t node_slot(const GeoDev& g, int x, int y, int z) {
  if (x < 0 || y < 0 || z < 0 || x > g.dims[0] || y > g.dims[1] || z > g.dims[2]) return -1;
  const int bx = x >> 2, by = y >> 2, bz = z >> 2;
  const int id = g.nmap[(bx * g.nbd[1] + by) * g.nbd[2] + bz];
  return id < 0 ? -1 : (int64_t)id * MPL_BC + local_index(x & 3, y & 3, z & 3);
}

__device__ __forceinline__ double block4_sum(double v, double* sh) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------- hierarchy

// coarse cell block of every fine cell block that carries a tangent
__global__ void k_mg_mark(GeoDev F, int f_ncblk, int cb1, int cb2, int32_t* __restrict__ cflag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= f_ncblk || F.cmask[i] == 0ull) return;
  const int4 b = F.ccoord[i];
  cflag[((b.x >> 1) * cb1 + (b.y >> 1)) * cb2 + (b.z >> 1)] = 1;
}

// tangent-carrying coarse cells: those with a tangent-carrying child
__global__ __launch_bounds__(64) void k_mg_cell_mask(GeoDev F, const int4* __restrict__ ccoord,
                                                     uint64_t* __restrict__ cmask,
                                                     int32_t* __restrict__ ccnt) {
  const int cb = blockIdx.x, l = threadIdx.x;
  const int4 b = ccoord[cb];
  const int X = b.x * 4 + local_x(l), Y = b.y * 4 + local_y(l), Z = b.z * 4 + local_z(l);
  bool act = false;
  for (int d = 0; d < 8; ++d) {
    const int fx = 2 * X + ((d >> 2) & 1), fy = 2 * Y + ((d >> 1) & 1), fz = 2 * Z + (d & 1);
    const int bx = fx >> 2, by = fy >> 2, bz = fz >> 2;
    if (bx >= F.cbd[0] || by >= F.cbd[1] || bz >= F.cbd[2]) continue;
    const int id = F.cmap[(bx * F.cbd[1] + by) * F.cbd[2] + bz];
    if (id < 0) continue;
    act = act || ((F.cmask[id] >> local_index(fx & 3, fy & 3, fz & 3)) & 1ull);
  }
  const uint64_t m = __ballot(act);
  if (l == 0) {
    cmask[cb] = m;
    ccnt[cb] = __popcll(m);
  }
}

// Column col of a factored FP32 cell tangent (layout in mpl_grid.h):
// y = Abar e_col with Abar vec(g) = vec(U yhat M^T), Ghat = U^T g M.
__device__ __forceinline__ void fact_column(const float* f, int col, float* y) {
  float U[9];
  quat_to_rot<float>(f[0], f[1], f[2], f[3], U);
  const float* M = f + 4;
  const float* A3 = f + 13;
  const float* pc = f + 19;
  // g = e_col: row a = col / 3, column b = col % 3
  const int ga = col / 3, gb = col % 3;
  float gh[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) gh[i * 3 + j] = U[ga * 3 + i] * M[gb * 3 + j];
  float yh[9];
  yh[0] = A3[0] * gh[0] + A3[1] * gh[4] + A3[2] * gh[8];
  yh[4] = A3[1] * gh[0] + A3[3] * gh[4] + A3[4] * gh[8];
  yh[8] = A3[2] * gh[0] + A3[4] * gh[4] + A3[5] * gh[8];
  yh[1] = pc[0] * gh[1] + pc[1] * gh[3];
  yh[3] = pc[1] * gh[1] + pc[0] * gh[3];
  yh[5] = pc[2] * gh[5] + pc[3] * gh[7];
  yh[7] = pc[3] * gh[5] + pc[2] * gh[7];
  yh[2] = pc[4] * gh[2] + pc[5] * gh[6];
  yh[6] = pc[5] * gh[2] + pc[4] * gh[6];
  float t2[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int j = 0; j < 3; ++j) t2[a * 3 + j] = U[a * 3] * yh[j] + U[a * 3 + 1] * yh[3 + j] + U[a * 3 + 2] * yh[6 + j];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) y[a * 3 + c] = t2[a * 3] * M[c * 3] + t2[a * 3 + 1] * M[c * 3 + 1] + t2[a * 3 + 2] * M[c * 3 + 2];
}

// Coarse cell tangent = sum of its children's (dense 45 values; children
// in the factored FP32 layout are expanded column by column).  Children are
// added in a fixed order (corner d = 0..7).
template <class T, bool PFACT, bool PMIX>
__global__ __launch_bounds__(64) void k_mg_tangent(GeoDev F, const T* __restrict__ Ap,
                                                   const int32_t* __restrict__ pcoff,
                                                   const uint8_t* __restrict__ pcfmt,
                                                   const int4* __restrict__ ccoord,
                                                   const uint64_t* __restrict__ cmask,
                                                   const int32_t* __restrict__ coff, T* __restrict__ Ac) {
  const int cb = blockIdx.x, l = threadIdx.x;
  const TanSlot cs = tan_slot(cmask, coff, cb, l, MPL_TAN_DENSE);
  if (!cs.active) return;
  const int4 b = ccoord[cb];
  const int X = b.x * 4 + local_x(l), Y = b.y * 4 + local_y(l), Z = b.z * 4 + local_z(l);
  T acc[MPL_TAN_DENSE];
#pragma unroll
  for (int e = 0; e < MPL_TAN_DENSE; ++e) acc[e] = T(0);
  for (int d = 0; d < 8; ++d) {
    const int fx = 2 * X + ((d >> 2) & 1), fy = 2 * Y + ((d >> 1) & 1), fz = 2 * Z + (d & 1);
    const int bx = fx >> 2, by = fy >> 2, bz = fz >> 2;
    if (bx >= F.cbd[0] || by >= F.cbd[1] || bz >= F.cbd[2]) continue;
    const int id = F.cmap[(bx * F.cbd[1] + by) * F.cbd[2] + bz];
    if (id < 0) continue;
    const int fl = local_index(fx & 3, fy & 3, fz & 3);
    const TanSlot ts = tan_slot(F.cmask, pcoff, id, fl, PFACT ? MPL_TAN_FACT : MPL_TAN_DENSE);
    if (!ts.active) continue;
    const T* A = Ap + ts.base + ts.rank;
    if constexpr (sizeof(T) == 4) {
      if (PFACT || (PMIX && pcfmt[id] != 0)) {
        float f[MPL_TAN_FACT_READ];
#pragma unroll
        for (int e = 0; e < MPL_TAN_FACT_READ; ++e) f[e] = (float)A[(int64_t)e * ts.n];
#pragma unroll
        for (int col = 0; col < 9; ++col) {
          float y[9];
          fact_column(f, col, y);
#pragma unroll
          for (int r = 0; r <= col; ++r) acc[sym9(r, col)] += (T)y[r];
        }
        continue;
      }
    }
#pragma unroll
    for (int e = 0; e < MPL_TAN_DENSE; ++e) acc[e] += A[(int64_t)e * ts.n];
  }
  T* out = Ac + cs.base + cs.rank;
#pragma unroll
  for (int e = 0; e < MPL_TAN_DENSE; ++e) out[(int64_t)e * cs.n] = acc[e];
}

// Coarse node mass m_C = P^T m (27 fine nodes, weights 1, 1/2, 1/4, 1/8 in a
// fixed order) and flags: component a fixed when the co-located fine node
// has mass and that component fixed; free when the coarse node has mass and
// the component is not fixed.
__global__ __launch_bounds__(64) void k_mg_nodes(GeoDev F, const int4* __restrict__ ncoord, int cd0,
                                                 int cd1, int cd2, double* __restrict__ mi,
                                                 uint8_t* __restrict__ flags) {
  const int nb = blockIdx.x, l = threadIdx.x;
  const int64_t ni = (int64_t)nb * MPL_BC + l;
  const int4 b = ncoord[nb];
  const int X = b.x * 4 + local_x(l), Y = b.y * 4 + local_y(l), Z = b.z * 4 + local_z(l);
  double m = 0.0;
  uint8_t fl = 0;
  if (X <= cd0 && Y <= cd1 && Z <= cd2) {
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dz = -1; dz <= 1; ++dz) {
          const int64_t s = node_slot(F, 2 * X + dx, 2 * Y + dy, 2 * Z + dz);
          if (s < 0) continue;
          const double w = (dx ? 0.5 : 1.0) * (dy ? 0.5 : 1.0) * (dz ? 0.5 : 1.0);
          m += w * F.mi[s];
        }
    const int64_t s0 = node_slot(F, 2 * X, 2 * Y, 2 * Z);
    const uint8_t f0 = s0 >= 0 ? F.flags[s0] : uint8_t(0);
    if (m > 0.0) {
      fl = MPL_NODE_ACTIVE;
      for (int a = 0; a < 3; ++a) {
        const bool fixed_a = (f0 & MPL_NODE_ACTIVE) && !mpl_free(f0, a);
        if (fixed_a) fl |= MPL_NODE_FIXED;
        else fl |= (uint8_t)(MPL_NODE_FREE_X << a);
      }
    }
  }
  mi[ni] = m;
  flags[ni] = fl;
}

// ---------------------------------------------------------------- power iteration
// Node vectors below: 4 node blocks (waves) per 256-thread workgroup, one
// partial sum per workgroup.

template <class T>
__global__ __launch_bounds__(256) void k_mg_pw_start(const uint8_t* __restrict__ flags,
                                                     const int4* __restrict__ ncoord, int d1, int d2,
                                                     int64_t nnode, int n_nblk, T* __restrict__ x,
                                                     double* __restrict__ part) {
  __shared__ double sh[4];
  const int nb = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  double xx = 0.0;
  if (nb < n_nblk) {
    const int64_t ni = (int64_t)nb * MPL_BC + l;
    const int4 b = ncoord[nb];
    const int64_t i = b.x * 4 + local_x(l), j = b.y * 4 + local_y(l), k = b.z * 4 + local_z(l);
    const uint64_t node = (uint64_t)((i * (d1 + 1) + j) * (d2 + 1) + k);
    const uint8_t fl = flags[ni];
    for (int a = 0; a < 3; ++a) {
      const double v = mpl_free(fl, a) ? ((splitmix64(3ull * node + a) >> 63) ? -1.0 : 1.0) : 0.0;
      x[a * nnode + ni] = (T)v;
      xx += v * v;
    }
  }
  xx = block4_sum(xx, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = xx;
}

// u = D^-1/2 x / |x| (D holds the inverse diagonal)
template <class T>
__global__ __launch_bounds__(256) void k_mg_pw_scale(const T* __restrict__ x, const double* __restrict__ D,
                                                     const double* __restrict__ xx, int64_t nnode, int n_nblk,
                                                     T* __restrict__ u) {
  const int nb = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  if (nb >= n_nblk) return;
  const int64_t ni = (int64_t)nb * MPL_BC + l;
  const double inv = *xx > 0.0 ? 1.0 / sqrt(*xx) : 0.0;
  for (int a = 0; a < 3; ++a) {
    const int64_t i = a * nnode + ni;
    u[i] = (T)(sqrt(D[i]) * (double)x[i] * inv);
  }
}

// y = D^-1/2 A u on the free components; partials of (x / |x|) . y and y . y;
// x <- y
template <class T>
__global__ __launch_bounds__(256) void k_mg_pw_apply(const T* __restrict__ u, const T* __restrict__ Hown,
                                                     const T* __restrict__ Hhalo,
                                                     const int* __restrict__ n_nbr_cell, int64_t ncell,
                                                     const double* __restrict__ mi,
                                                     const uint8_t* __restrict__ flags,
                                                     const double* __restrict__ D,
                                                     const double* __restrict__ xx, int64_t nnode,
                                                     int n_nblk, T* __restrict__ x,
                                                     double* __restrict__ pxy, double* __restrict__ pyy) {
  __shared__ double sh[4];
  const int nb = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  double sxy = 0.0, syy = 0.0;
  if (nb < n_nblk) {
    const int64_t ni = (int64_t)nb * MPL_BC + l;
    const uint8_t fl = flags[ni];
    T h[3];
    gather_kp(Hown, Hhalo, n_nbr_cell, ncell, nb, l, h);
    const double m = mi[ni];
    const double inv = *xx > 0.0 ? 1.0 / sqrt(*xx) : 0.0;
    for (int a = 0; a < 3; ++a) {
      const int64_t i = a * nnode + ni;
      const double y = mpl_free(fl, a) ? sqrt(D[i]) * ((double)h[a] + m * (double)u[i]) : 0.0;
      sxy += (double)x[i] * inv * y;
      syy += y * y;
      x[i] = (T)y;
    }
  }
  sxy = block4_sum(sxy, sh);
  syy = block4_sum(syy, sh);
  if (threadIdx.x == 0) {
    pxy[blockIdx.x] = sxy;
    pyy[blockIdx.x] = syy;
  }
}

// Fixed-order sum of one or two partial arrays by one workgroup into out[0..1]
// (out[1] untouched when b is null).
__global__ __launch_bounds__(1024) void k_mg_sum(const double* __restrict__ a, const double* __restrict__ b,
                                                 int n, double* __restrict__ out) {
  __shared__ double sh[2][16];
  const int t = threadIdx.x;
  double va = 0.0, vb = 0.0;
  for (int i = t; i < n; i += 1024) {
    va += a[i];
    if (b) vb += b[i];
  }
  va = wave_sum(va);
  vb = wave_sum(vb);
  if ((t & 63) == 0) {
    sh[0][t >> 6] = va;
    sh[1][t >> 6] = vb;
  }
  __syncthreads();
  if (t == 0) {
    double A = 0.0, B = 0.0;
    for (int w = 0; w < 16; ++w) {
      A += sh[0][w];
      B += sh[1][w];
    }
    out[0] = A;
    if (b) out[1] = B;
  }
}

// ---------------------------------------------------------------- V-cycle kernels

// Damped-Jacobi sweep on the free components: FIRST x = omega Dinv b, else
// x += omega Dinv (b - (K x + M x)) with K x gathered from the pieces.
template <class T, class BT, bool FIRST>
__global__ __launch_bounds__(256) void k_mg_jacobi(const BT* __restrict__ b, const T* __restrict__ Dinv,
                                                   const T* __restrict__ Hown, const T* __restrict__ Hhalo,
                                                   const int* __restrict__ n_nbr_cell, int64_t ncell,
                                                   const double* __restrict__ mi,
                                                   const uint8_t* __restrict__ flags, int64_t nnode,
                                                   int n_nblk, double omega, T* __restrict__ x,
                                                   const SolverScalars* __restrict__ s) {
  if (s && done_flag(s)) return;
  const int nb = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  if (nb >= n_nblk) return;
  const int64_t ni = (int64_t)nb * MPL_BC + l;
  const uint8_t fl = flags[ni];
  T h[3] = {T(0), T(0), T(0)};
  if (!FIRST) gather_kp(Hown, Hhalo, n_nbr_cell, ncell, nb, l, h);
  const T m = (T)mi[ni];
  const T w = (T)omega;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int64_t i = a * nnode + ni;
    T v = T(0);
    if (mpl_free(fl, a)) {
      const T bv = (T)b[i];
      if (FIRST) {
        v = w * Dinv[i] * bv;
      } else {
        const T xv = x[i];
        v = xv + w * Dinv[i] * (bv - (h[a] + m * xv));
      }
    }
    x[i] = v;
  }
}

// res = b - (K x + M x) on the free components
template <class T, class BT>
__global__ __launch_bounds__(256) void k_mg_residual(const BT* __restrict__ b, const T* __restrict__ Hown,
                                                     const T* __restrict__ Hhalo,
                                                     const int* __restrict__ n_nbr_cell, int64_t ncell,
                                                     const double* __restrict__ mi,
                                                     const uint8_t* __restrict__ flags, int64_t nnode,
                                                     int n_nblk, const T* __restrict__ x, T* __restrict__ res,
                                                     const SolverScalars* __restrict__ s) {
  if (s && done_flag(s)) return;
  const int nb = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  if (nb >= n_nblk) return;
  const int64_t ni = (int64_t)nb * MPL_BC + l;
  const uint8_t fl = flags[ni];
  T h[3];
  gather_kp(Hown, Hhalo, n_nbr_cell, ncell, nb, l, h);
  const T m = (T)mi[ni];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int64_t i = a * nnode + ni;
    res[i] = mpl_free(fl, a) ? (T)b[i] - (h[a] + m * x[i]) : T(0);
  }
}

// coarse b = P^T res on the coarse free components (27 fine nodes per coarse
// node in a fixed order; the fine residual is zero off the fine free DOFs)
template <class T>
__global__ __launch_bounds__(256) void k_mg_restrict(GeoDev F, const T* __restrict__ fres, int64_t f_nnode,
                                                     const int4* __restrict__ ncoord,
                                                     const uint8_t* __restrict__ flags, int64_t nnode,
                                                     int n_nblk, T* __restrict__ bc,
                                                     const SolverScalars* __restrict__ s) {
  if (s && done_flag(s)) return;
  const int nb = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  if (nb >= n_nblk) return;
  const int64_t ni = (int64_t)nb * MPL_BC + l;
  const uint8_t fl = flags[ni];
  T acc[3] = {T(0), T(0), T(0)};
  if (fl & MPL_NODE_FREE_ALL) {
    const int4 b = ncoord[nb];
    const int X = b.x * 4 + local_x(l), Y = b.y * 4 + local_y(l), Z = b.z * 4 + local_z(l);
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dz = -1; dz <= 1; ++dz) {
          const int64_t sl = node_slot(F, 2 * X + dx, 2 * Y + dy, 2 * Z + dz);
          if (sl < 0) continue;
          const T w = (T)((dx ? 0.5 : 1.0) * (dy ? 0.5 : 1.0) * (dz ? 0.5 : 1.0));
#pragma unroll
          for (int a = 0; a < 3; ++a) acc[a] += w * fres[a * f_nnode + sl];
        }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) bc[a * nnode + ni] = mpl_free(fl, a) ? acc[a] : T(0);
}

// fine x += P xc on the fine free components (1, 2, 4 or 8 coarse nodes per
// fine node; the coarse vector is zero off the coarse free DOFs)
template <class T>
__global__ __launch_bounds__(256) void k_mg_prolong(GeoDev Cg, const T* __restrict__ xc, int64_t c_nnode,
                                                    const int4* __restrict__ ncoord,
                                                    const uint8_t* __restrict__ flags, int64_t nnode,
                                                    int n_nblk, T* __restrict__ x,
                                                    const SolverScalars* __restrict__ s) {
  if (s && done_flag(s)) return;
  const int nb = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  if (nb >= n_nblk) return;
  const int64_t ni = (int64_t)nb * MPL_BC + l;
  const uint8_t fl = flags[ni];
  if (!(fl & MPL_NODE_FREE_ALL)) return;
  const int4 b = ncoord[nb];
  const int p[3] = {b.x * 4 + local_x(l), b.y * 4 + local_y(l), b.z * 4 + local_z(l)};
  int lo[3], cnt[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = p[a] >> 1;
    cnt[a] = (p[a] & 1) ? 2 : 1;
  }
  T acc[3] = {T(0), T(0), T(0)};
  for (int i = 0; i < cnt[0]; ++i)
    for (int j = 0; j < cnt[1]; ++j)
      for (int k = 0; k < cnt[2]; ++k) {
        const int64_t sl = node_slot(Cg, lo[0] + i, lo[1] + j, lo[2] + k);
        if (sl < 0) continue;
        const T w = (T)((cnt[0] == 2 ? 0.5 : 1.0) * (cnt[1] == 2 ? 0.5 : 1.0) * (cnt[2] == 2 ? 0.5 : 1.0));
#pragma unroll
        for (int a = 0; a < 3; ++a) acc[a] += w * xc[a * c_nnode + sl];
      }
#pragma unroll
  for (int a = 0; a < 3; ++a)
    if (mpl_free(fl, a)) x[a * nnode + ni] += acc[a];
}

// ---------------------------------------------------------------- PCG kernels

// x = x0 (or 0), r = b - A x0 (or b) on the free components; partials of b.b
// and r.r.  Hown/Hhalo: pieces of the product of x0 (ignored without x0).
template <class T>
__global__ __launch_bounds__(256) void k_mgpcg_init(const double* __restrict__ b,
                                                    const double* __restrict__ x0, const T* __restrict__ u0,
                                                    const T* __restrict__ Hown, const T* __restrict__ Hhalo,
                                                    const int* __restrict__ n_nbr_cell, int64_t ncell,
                                                    const double* __restrict__ mi,
                                                    const uint8_t* __restrict__ flags, int64_t nnode,
                                                    int n_nblk, double* __restrict__ x, double* __restrict__ r,
                                                    double* __restrict__ pbb, double* __restrict__ prr) {
  __shared__ double sh[4];
  const int nb = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  double bb = 0.0, rr = 0.0;
  if (nb < n_nblk) {
    const int64_t ni = (int64_t)nb * MPL_BC + l;
    const uint8_t fl = flags[ni];
    T h[3] = {T(0), T(0), T(0)};
    if (x0) gather_kp(Hown, Hhalo, n_nbr_cell, ncell, nb, l, h);
    const double m = mi[ni];
    for (int a = 0; a < 3; ++a) {
      const int64_t i = a * nnode + ni;
      const bool fa = mpl_free(fl, a);
      const double bv = fa ? b[i] : 0.0;
      double rv = bv;
      if (x0 && fa) rv = bv - ((double)h[a] + m * (double)u0[i]);
      x[i] = (x0 && fa) ? x0[i] : 0.0;
      r[i] = fa ? rv : 0.0;
      bb += bv * bv;
      rr += fa ? rv * rv : 0.0;
    }
  }
  bb = block4_sum(bb, sh);
  rr = block4_sum(rr, sh);
  if (threadIdx.x == 0) {
    pbb[blockIdx.x] = bb;
    prr[blockIdx.x] = rr;
  }
}

// u0 = x0 in the tangent's precision on the free components
template <class T>
__global__ void k_mgpcg_cast(const double* __restrict__ x0, const uint8_t* __restrict__ flags, int64_t nnode,
                             T* __restrict__ u) {
  const int64_t ni = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ni >= nnode) return;
  const uint8_t fl = flags[ni];
  for (int a = 0; a < 3; ++a) u[a * nnode + ni] = mpl_free(fl, a) ? (T)x0[a * nnode + ni] : T(0);
}

// q = K p + M p, x += alpha p, r -= alpha q on the free components; partial r.r
template <class T>
__global__ __launch_bounds__(256) void k_mgpcg_update(const T* __restrict__ p, const T* __restrict__ Hown,
                                                      const T* __restrict__ Hhalo,
                                                      const int* __restrict__ n_nbr_cell, int64_t ncell,
                                                      const double* __restrict__ mi,
                                                      const uint8_t* __restrict__ flags, int64_t nnode,
                                                      int n_nblk, double* __restrict__ x, double* __restrict__ r,
                                                      double* __restrict__ prr,
                                                      const SolverScalars* __restrict__ s) {
  if (done_flag(s)) return;
  __shared__ double sh[4];
  const int nb = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  const double alpha = s->alpha;
  double rr = 0.0;
  if (nb < n_nblk) {
    const int64_t ni = (int64_t)nb * MPL_BC + l;
    const uint8_t fl = flags[ni];
    if (fl & MPL_NODE_FREE_ALL) {
      T h[3];
      gather_kp(Hown, Hhalo, n_nbr_cell, ncell, nb, l, h);
      const T m = (T)mi[ni];
      for (int a = 0; a < 3; ++a) {
        if (!mpl_free(fl, a)) continue;
        const int64_t i = a * nnode + ni;
        const T pv = p[i];
        const double q = (double)(h[a] + m * pv);
        x[i] += alpha * (double)pv;
        const double rv = r[i] - alpha * q;
        r[i] = rv;
        rr += rv * rv;
      }
    }
  }
  rr = block4_sum(rr, sh);
  if (threadIdx.x == 0) prr[blockIdx.x] = rr;
}

// partial r.z (FP64 r, z in the cycle's precision)
template <class T>
__global__ __launch_bounds__(256) void k_mgpcg_dot(const double* __restrict__ r, const T* __restrict__ z,
                                                   int64_t nnode, int n_nblk, double* __restrict__ prz,
                                                   const SolverScalars* __restrict__ s) {
  if (done_flag(s)) return;
  __shared__ double sh[4];
  const int nb = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  double rz = 0.0;
  if (nb < n_nblk) {
    const int64_t ni = (int64_t)nb * MPL_BC + l;
    for (int a = 0; a < 3; ++a) rz += r[a * nnode + ni] * (double)z[a * nnode + ni];
  }
  rz = block4_sum(rz, sh);
  if (threadIdx.x == 0) prz[blockIdx.x] = rz;
}

// p = z + beta p (FIRST: p = z); partial p^T M p
template <class T, bool FIRST>
__global__ __launch_bounds__(256) void k_mgpcg_dir(const T* __restrict__ z, const double* __restrict__ mi,
                                                   const uint8_t* __restrict__ flags, int64_t nnode,
                                                   int n_nblk, T* __restrict__ p, double* __restrict__ pmm,
                                                   const SolverScalars* __restrict__ s) {
  if (done_flag(s)) return;
  __shared__ double sh[4];
  const int nb = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
  const double beta = FIRST ? 0.0 : s->beta;
  double mm = 0.0;
  if (nb < n_nblk) {
    const int64_t ni = (int64_t)nb * MPL_BC + l;
    const uint8_t fl = flags[ni];
    const double m = mi[ni];
    for (int a = 0; a < 3; ++a) {
      const int64_t i = a * nnode + ni;
      const T pv = mpl_free(fl, a) ? (FIRST ? z[i] : (T)((double)z[i] + beta * (double)p[i])) : T(0);
      p[i] = pv;
      mm += m * (double)pv * (double)pv;
    }
  }
  mm = block4_sum(mm, sh);
  if (threadIdx.x == 0) pmm[blockIdx.x] = mm;
}

enum { MG_SETUP = 0, MG_RZ0 = 1, MG_ALPHA = 2, MG_CHECK = 3, MG_BETA = 4 };

// Fixed-order reduction of one or two partial arrays and the PCG scalar logic.
template <int MODE>
__global__ __launch_bounds__(1024) void k_mg_reduce(const double* __restrict__ a, int na,
                                                    const double* __restrict__ b, int nb,
                                                    SolverScalars* __restrict__ s, double rtol2) {
  __shared__ double sh[2][16];
  const int t = threadIdx.x;
  if (MODE != MG_SETUP && done_flag(s)) return;
  double va = 0.0, vb = 0.0;
  for (int i = t; i < na; i += 1024) va += a[i];
  for (int i = t; i < nb; i += 1024) vb += b[i];
  va = wave_sum(va);
  vb = wave_sum(vb);
  if ((t & 63) == 0) {
    sh[0][t >> 6] = va;
    sh[1][t >> 6] = vb;
  }
  __syncthreads();
  if (t != 0) return;
  double A = 0.0, B = 0.0;
  for (int w = 0; w < 16; ++w) {
    A += sh[0][w];
    B += sh[1][w];
  }
  if (MODE == MG_SETUP) {  // A = b.b, B = r.r of the start
    s->bnorm2 = A;
    s->rr = B;
    s->tol2 = rtol2 * A;
    s->iters = 0;
    s->alpha = s->beta = 0.0;
    s->done = (A == 0.0 || B <= s->tol2) ? 1 : (isfinite(B) ? 0 : 2);
  } else if (MODE == MG_RZ0) {  // A = r.z
    if (!(A > 0.0) || !isfinite(A)) s->done = 2;
    else s->rz = A;
  } else if (MODE == MG_ALPHA) {  // A = p^T K p (cells), B = p^T M p (nodes)
    const double pq = A + B;
    s->pq = pq;
    if (!(pq > 0.0) || !isfinite(pq)) s->done = 2;
    else s->alpha = s->rz / pq;
  } else if (MODE == MG_CHECK) {  // A = r.r
    s->rr = A;
    s->iters += 1;
    if (!isfinite(A)) s->done = 2;
    else if (A <= s->tol2) s->done = 1;
  } else {  // MG_BETA: A = r.z
    if (!(A > 0.0) || !isfinite(A)) {
      s->done = 2;
    } else {
      s->beta = A / s->rz;
      s->rz = A;
    }
  }
}

// ---------------------------------------------------------------- exports

template <class T>
__global__ void k_mg_to_f64(const T* __restrict__ a, double* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (double)a[i];
}

__global__ void k_mg_fill(double* __restrict__ a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0;
}

// field 0 mass, 1 fixed components (bits), 3 inverse diagonal (3 values)
__global__ __launch_bounds__(64) void k_mg_export_nodes(const int4* __restrict__ ncoord, int d0, int d1, int d2,
                                                        const double* __restrict__ mi,
                                                        const uint8_t* __restrict__ flags,
                                                        const double* __restrict__ D, int64_t nnode, int field,
                                                        double* __restrict__ out) {
  const int nb = blockIdx.x, l = threadIdx.x;
  const int64_t ni = (int64_t)nb * MPL_BC + l;
  const int4 b = ncoord[nb];
  const int x = b.x * 4 + local_x(l), y = b.y * 4 + local_y(l), z = b.z * 4 + local_z(l);
  if (x > d0 || y > d1 || z > d2) return;
  const int64_t di = ((int64_t)x * (d1 + 1) + y) * (d2 + 1) + z;
  const uint8_t fl = flags[ni];
  if (field == 0) {
    out[di] = mi[ni];
  } else if (field == 1) {
    int bits = 0;
    for (int a = 0; a < 3; ++a)
      if ((fl & MPL_NODE_ACTIVE) && !mpl_free(fl, a)) bits |= 1 << a;
    out[di] = (double)bits;
  } else {
    for (int a = 0; a < 3; ++a) out[di * 3 + a] = D[a * nnode + ni];
  }
}

template <class T>
__global__ __launch_bounds__(64) void k_mg_export_tangent(const T* __restrict__ A, const uint64_t* __restrict__ cmask,
                                                          const int32_t* __restrict__ coff,
                                                          const int4* __restrict__ ccoord, int d1, int d2,
                                                          double* __restrict__ out) {
  const int cb = blockIdx.x, l = threadIdx.x;
  const TanSlot ts = tan_slot(cmask, coff, cb, l, MPL_TAN_DENSE);
  if (!ts.active) return;
  const int4 b = ccoord[cb];
  const int64_t x = b.x * 4 + local_x(l), y = b.y * 4 + local_y(l), z = b.z * 4 + local_z(l);
  const int64_t di = (x * d1 + y) * d2 + z;
  for (int r = 0; r < 9; ++r)
    for (int q = 0; q < 9; ++q) out[di * 81 + r * 9 + q] = (double)A[ts.base + (int64_t)sym9(r, q) * ts.n + ts.rank];
}

}  // namespace

// ====================================================================== host

namespace {

GeoDev geo0(const mpl_ctx* c) {
  GeoDev g{};
  for (int a = 0; a < 3; ++a) {
    g.dims[a] = c->dims[a];
    g.cbd[a] = c->cbd[a];
    g.nbd[a] = c->nbd[a];
  }
  g.cmap = P<int32_t>(c->cmap);
  g.nmap = P<int32_t>(c->nmap);
  g.ccoord = P<int4>(c->ccoord);
  g.ncoord = P<int4>(c->ncoord);
  g.cmask = P<uint64_t>(c->cmask);
  g.mi = P<double>(c->mi);
  g.flags = P<uint8_t>(c->flags);
  return g;
}

GeoDev geo_level(const MGLevel& L) {
  GeoDev g{};
  for (int a = 0; a < 3; ++a) {
    g.dims[a] = L.dims[a];
    g.cbd[a] = L.cbd[a];
    g.nbd[a] = L.nbd[a];
  }
  g.cmap = P<int32_t>(L.cmap);
  g.nmap = P<int32_t>(L.nmap);
  g.ccoord = P<int4>(L.ccoord);
  g.ncoord = P<int4>(L.ncoord);
  g.cmask = P<uint64_t>(L.cmask);
  g.mi = P<double>(L.mi);
  g.flags = P<uint8_t>(L.flags);
  return g;
}

GeoDev geo(const mpl_ctx* c, int l) { return l == 0 ? geo0(c) : geo_level(c->mg->lev[l]); }

template <class T>
LevelArrays arrays(const mpl_ctx* c, int l) {
  if (l == 0) return mpl_level0<T>(c);
  const MGLevel& L = c->mg->lev[l];
  LevelArrays a;
  a.n_cblk = L.n_cblk;
  a.n_nblk = L.n_nblk;
  a.ncell = L.ncell();
  a.nnode = L.nnode();
  a.c_nbr_node = P<int>(L.c_nbr_node);
  a.n_nbr_cell = P<int>(L.n_nbr_cell);
  a.cmask = P<uint64_t>(L.cmask);
  a.coff = P<int32_t>(L.coff);
  a.Abar = L.Abar.p;
  a.mi = P<double>(L.mi);
  a.flags = P<uint8_t>(L.flags);
  a.inv_dx = L.inv_dx;
  return a;
}

// inverse Jacobi diagonal of level l: FP64 and in T
const double* dinv64(const mpl_ctx* c, int l) { return l == 0 ? P<double>(c->D) : P<double>(c->mg->lev[l].D); }
template <class T>
const T* dinv_t(const mpl_ctx* c, int l) { return l == 0 ? P<T>(c->Dt) : P<T>(c->mg->lev[l].Dt); }
const int4* ncoord_of(const mpl_ctx* c, int l) { return l == 0 ? P<int4>(c->ncoord) : P<int4>(c->mg->lev[l].ncoord); }

int vgrid(int n_nblk) { return (n_nblk + 3) / 4; }

// Structure, tangent, masses and diagonal of level l >= 1 from level l - 1.
template <class T>
mpl_status build_level(mpl_ctx* c, int l) {
  MGState& M = *c->mg;
  MGLevel& L = M.lev[l];
  const GeoDev F = geo(c, l - 1);
  const int f_ncblk = l == 1 ? c->n_cblk : M.lev[l - 1].n_cblk;
  for (int a = 0; a < 3; ++a) {
    L.dims[a] = F.dims[a] / 2;
    L.cbd[a] = (L.dims[a] + 3) / 4;
    L.nbd[a] = L.cbd[a] + 1;
  }
  L.dx = (l == 1 ? c->dx : M.lev[l - 1].dx) * 2.0;
  L.inv_dx = 1.0 / L.dx;
  const int ncb = L.cbd[0] * L.cbd[1] * L.cbd[2], nnb = L.nbd[0] * L.nbd[1] * L.nbd[2];
  MPL_TRY(mpl_ensure(c, L.cflag, sizeof(int32_t) * ncb));
  MPL_TRY(mpl_ensure(c, L.cmap, sizeof(int32_t) * (ncb + 1)));
  MPL_TRY(mpl_ensure(c, L.nflag, sizeof(int32_t) * nnb));
  MPL_TRY(mpl_ensure(c, L.nmap, sizeof(int32_t) * (nnb + 1)));
  MPL_TRY(mpl_ensure(c, L.ccoord, sizeof(int4) * ncb));
  MPL_TRY(mpl_ensure(c, L.ncoord, sizeof(int4) * nnb));
  MPL_TRY(mpl_ensure(c, L.c_nbr_node, sizeof(int32_t) * 8 * ncb));
  MPL_TRY(mpl_ensure(c, L.n_nbr_cell, sizeof(int32_t) * 8 * nnb));
  MPL_TRY(mpl_ensure(c, L.scan, sizeof(int32_t) * (ncb + nnb + 2)));
  MPL_TRY(mpl_ensure(c, M.counts, sizeof(int32_t) * 4));
  MPL_HIP(c, hipMemsetAsync(L.cflag.p, 0, sizeof(int32_t) * ncb, c->stream));
  MPL_HIP(c, hipMemsetAsync(L.nflag.p, 0, sizeof(int32_t) * nnb, c->stream));
  MPL_LAUNCH(c, k_mg_mark, (f_ncblk + 255) / 256, 256, F, f_ncblk, L.cbd[1], L.cbd[2], P<int32_t>(L.cflag));
  int32_t* cnt = P<int32_t>(M.counts);
  MPL_TRY(mpl_block_maps(c, L.dims, L.cbd, L.nbd, P<int32_t>(L.cflag), P<int32_t>(L.cmap), P<int4>(L.ccoord),
                         P<int32_t>(L.nflag), P<int32_t>(L.nmap), P<int4>(L.ncoord), P<int32_t>(L.scan), cnt));
  int32_t h[2] = {0, 0};
  MPL_HIP(c, hipMemcpyAsync(h, cnt, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  MPL_HIP(c, hipStreamSynchronize(c->stream));
  L.n_cblk = h[0];
  L.n_nblk = h[1];
  MPL_TRY(mpl_block_neighbours(c, L.dims, L.cbd, L.nbd, P<int4>(L.ccoord), P<int4>(L.ncoord), P<int32_t>(L.cmap),
                               P<int32_t>(L.nmap), P<int32_t>(L.c_nbr_node), P<int32_t>(L.n_nbr_cell), L.n_cblk,
                               L.n_nblk));
  const int64_t ncell = L.ncell(), nnode = L.nnode();
  MPL_TRY(mpl_ensure(c, L.cmask, sizeof(uint64_t) * (L.n_cblk + 1)));
  MPL_TRY(mpl_ensure(c, L.ccnt, sizeof(int32_t) * (L.n_cblk + 1)));
  MPL_TRY(mpl_ensure(c, L.coff, sizeof(int32_t) * (L.n_cblk + 1)));
  MPL_LAUNCH(c, k_mg_cell_mask, L.n_cblk, 64, F, P<int4>(L.ccoord), P<uint64_t>(L.cmask), P<int32_t>(L.ccnt));
  MPL_TRY(mpl_scan_i32(c, P<int32_t>(L.ccnt), P<int32_t>(L.coff), L.n_cblk, cnt + 2));
  // tangent: dense 45 values per tangent-carrying cell (at most all of them)
  MPL_TRY(mpl_ensure(c, L.Abar, sizeof(T) * MPL_TAN_DENSE * (ncell + 1)));
  const LevelArrays Fa = arrays<T>(c, l - 1);
  const T* Ap = (const T*)Fa.Abar;
  if (Fa.fact)
    MPL_LAUNCH(c, (k_mg_tangent<T, true, false>), L.n_cblk, 64, F, Ap, Fa.coff, Fa.cfmt, P<int4>(L.ccoord),
               P<uint64_t>(L.cmask), P<int32_t>(L.coff), P<T>(L.Abar));
  else if (Fa.mixed)
    MPL_LAUNCH(c, (k_mg_tangent<T, false, true>), L.n_cblk, 64, F, Ap, Fa.coff, Fa.cfmt, P<int4>(L.ccoord),
               P<uint64_t>(L.cmask), P<int32_t>(L.coff), P<T>(L.Abar));
  else
    MPL_LAUNCH(c, (k_mg_tangent<T, false, false>), L.n_cblk, 64, F, Ap, Fa.coff, Fa.cfmt, P<int4>(L.ccoord),
               P<uint64_t>(L.cmask), P<int32_t>(L.coff), P<T>(L.Abar));
  // nodes
  MPL_TRY(mpl_ensure(c, L.mi, sizeof(double) * nnode));
  MPL_TRY(mpl_ensure(c, L.flags, nnode + 64));
  MPL_LAUNCH(c, k_mg_nodes, L.n_nblk, 64, F, P<int4>(L.ncoord), L.dims[0], L.dims[1], L.dims[2], P<double>(L.mi),
             P<uint8_t>(L.flags));
  MPL_TRY(mpl_ensure(c, L.D, sizeof(double) * 3 * nnode));
  MPL_TRY(mpl_ensure(c, L.Dt, sizeof(T) * 3 * nnode));
  MPL_TRY(mpl_ensure(c, L.mt, sizeof(T) * nnode));
  MPL_TRY(mpl_level_diag<T>(c, arrays<T>(c, l), P<double>(L.D), P<T>(L.Dt), P<T>(L.mt)));
  return MPL_OK;
}

// Cycle vectors of level l (x, b, res, pieces, partials).
template <class T>
mpl_status level_vectors(mpl_ctx* c, int l) {
  MGLevel& L = c->mg->lev[l];
  const LevelArrays a = arrays<T>(c, l);
  MPL_TRY(mpl_ensure(c, L.x, sizeof(T) * 3 * a.nnode));
  MPL_TRY(mpl_ensure(c, L.b, sizeof(T) * 3 * a.nnode));
  MPL_TRY(mpl_ensure(c, L.res, sizeof(T) * 3 * a.nnode));
  MPL_TRY(mpl_ensure(c, L.pieces, sizeof(T) * 6 * a.ncell + 64));
  MPL_TRY(mpl_ensure(c, L.part, sizeof(double) * 3 * (vgrid(a.n_nblk) + 8)));
  return MPL_OK;
}

// lambda_l by power iterations (every level at once, one synchronisation).
template <class T>
mpl_status estimate_lambdas(mpl_ctx* c, int iters) {
  MGState& M = *c->mg;
  MPL_TRY(mpl_ensure(c, M.pw, sizeof(double) * 4 * MPL_MG_MAX_LEVELS));
  double* pw = P<double>(M.pw);
  for (int l = 0; l < M.nlev; ++l) {
    MGLevel& L = M.lev[l];
    const LevelArrays a = arrays<T>(c, l);
    const int d1 = l == 0 ? c->dims[1] : L.dims[1], d2 = l == 0 ? c->dims[2] : L.dims[2];
    const int ng = vgrid(a.n_nblk);
    double* pa = P<double>(L.part);
    double* pb = pa + ng + 8;
    double* s = pw + 4 * l;  // s[0] = x.x, s[1] = (x/|x|).y, s[2] = y.y
    T* x = P<T>(L.x);
    T* u = P<T>(L.res);
    MPL_LAUNCH(c, k_mg_pw_start<T>, ng, 256, a.flags, ncoord_of(c, l), d1, d2, a.nnode, a.n_nblk, x, pa);
    MPL_LAUNCH(c, k_mg_sum, 1, 1024, pa, (const double*)nullptr, ng, s);
    for (int k = 0; k < iters; ++k) {
      if (k > 0)
        MPL_HIP(c, hipMemcpyAsync(s, s + 2, sizeof(double), hipMemcpyDeviceToDevice, c->stream));
      MPL_LAUNCH(c, k_mg_pw_scale<T>, ng, 256, x, dinv64(c, l), s, a.nnode, a.n_nblk, u);
      MPL_TRY(mpl_level_hv_pieces<T>(c, a, u, P<T>(L.pieces), nullptr));
      const T* Hown = P<T>(L.pieces);
      MPL_LAUNCH(c, k_mg_pw_apply<T>, ng, 256, u, Hown, Hown + 3 * a.ncell, a.n_nbr_cell, a.ncell, a.mi, a.flags,
                 dinv64(c, l), s, a.nnode, a.n_nblk, x, pa, pb);
      MPL_LAUNCH(c, k_mg_sum, 1, 1024, pa, pb, ng, s + 1);
    }
  }
  double h[4 * MPL_MG_MAX_LEVELS];
  MPL_HIP(c, hipMemcpyAsync(h, pw, sizeof(double) * 4 * M.nlev, hipMemcpyDeviceToHost, c->stream));
  MPL_HIP(c, hipStreamSynchronize(c->stream));
  for (int l = 0; l < M.nlev; ++l) {
    const double lam = h[4 * l + 1];
    // exactly 0: the level has no free DOF (its start vector is 0), so its
    // sweeps have nothing to do; otherwise A is positive definite on it
    if (lam == 0.0) {
      M.lev[l].lambda = M.lev[l].omega = 0.0;
      continue;
    }
    if (!(lam > 0.0) || !std::isfinite(lam))
      return mpl_fail(c, MPL_ERR_NONFINITE, "multigrid: power iteration gave no positive eigenvalue");
    M.lev[l].lambda = lam;
    M.lev[l].omega = c->opts.mg_omega / lam;
  }
  return MPL_OK;
}

// Level count: halve while every axis stays even and its half >= 4 cells.
int level_count(const mpl_ctx* c) {
  int d[3] = {c->dims[0], c->dims[1], c->dims[2]};
  int n = 1;
  while (n < c->opts.mg_levels) {
    bool ok = true;
    for (int a = 0; a < 3; ++a) ok = ok && d[a] % 2 == 0 && d[a] / 2 >= 4;
    if (!ok) break;
    for (int a = 0; a < 3; ++a) d[a] /= 2;
    ++n;
  }
  return n;
}

template <class T>
mpl_status mg_ensure(mpl_ctx* c) {
  if (!c->tangent_built) return mpl_fail(c, MPL_ERR_STATE, "multigrid needs a tangent");
  if (c->tangent_precision != (sizeof(T) == 4 ? MPL_F32 : MPL_F64))
    return mpl_fail(c, MPL_ERR_STATE, "multigrid: tangent precision mismatch");
  if (!c->mg) c->mg = new MGState();
  MGState& M = *c->mg;
  if (M.serial == c->tangent_serial && M.precision == c->tangent_precision && M.levels_opt == c->opts.mg_levels &&
      M.omega_opt == c->opts.mg_omega)
    return MPL_OK;
  M.serial = -1;
  M.nlev = level_count(c);
  for (int l = 1; l < M.nlev; ++l) MPL_TRY(build_level<T>(c, l));
  for (int l = 0; l < M.nlev; ++l) MPL_TRY(level_vectors<T>(c, l));
  MPL_TRY(estimate_lambdas<T>(c, 20));
  M.serial = c->tangent_serial;
  M.precision = c->tangent_precision;
  M.levels_opt = c->opts.mg_levels;
  M.omega_opt = c->opts.mg_omega;
  return MPL_OK;
}

// One V-cycle from level l: x_l = B_l b.  BT: the right-hand side's type
// (FP64 on level 0 inside PCG, T elsewhere).
template <class T, class BT>
mpl_status vcycle(mpl_ctx* c, int l, const BT* b, const SolverScalars* s) {
  MGState& M = *c->mg;
  MGLevel& L = M.lev[l];
  const LevelArrays a = arrays<T>(c, l);
  const int ng = vgrid(a.n_nblk);
  T* x = P<T>(L.x);
  T* pieces = P<T>(L.pieces);
  const T* Hown = pieces;
  const T* Hhalo = pieces + 3 * a.ncell;
  const T* Dinv = dinv_t<T>(c, l);
  const double w = L.omega;
  const bool coarsest = l == M.nlev - 1;
  const int pre = coarsest ? c->opts.mg_coarse_sweeps : c->opts.mg_smooth;
  auto sweep = [&](bool first) -> mpl_status {
    if (first) {
      MPL_LAUNCH(c, (k_mg_jacobi<T, BT, true>), ng, 256, b, Dinv, Hown, Hhalo, a.n_nbr_cell, a.ncell, a.mi, a.flags,
                 a.nnode, a.n_nblk, w, x, s);
    } else {
      MPL_TRY(mpl_level_hv_pieces<T>(c, a, x, pieces, s));
      MPL_LAUNCH(c, (k_mg_jacobi<T, BT, false>), ng, 256, b, Dinv, Hown, Hhalo, a.n_nbr_cell, a.ncell, a.mi, a.flags,
                 a.nnode, a.n_nblk, w, x, s);
    }
    return MPL_OK;
  };
  for (int k = 0; k < pre; ++k) MPL_TRY(sweep(k == 0));
  if (coarsest) return MPL_OK;
  // residual, restriction, coarse cycle, prolongation
  T* res = P<T>(L.res);
  MPL_TRY(mpl_level_hv_pieces<T>(c, a, x, pieces, s));
  MPL_LAUNCH(c, (k_mg_residual<T, BT>), ng, 256, b, Hown, Hhalo, a.n_nbr_cell, a.ncell, a.mi, a.flags, a.nnode,
             a.n_nblk, x, res, s);
  MGLevel& C = M.lev[l + 1];
  const LevelArrays ca = arrays<T>(c, l + 1);
  T* bc = P<T>(C.b);
  MPL_LAUNCH(c, k_mg_restrict<T>, vgrid(ca.n_nblk), 256, geo(c, l), (const T*)res, a.nnode, P<int4>(C.ncoord),
             ca.flags, ca.nnode, ca.n_nblk, bc, s);
  MPL_TRY((vcycle<T, T>(c, l + 1, bc, s)));
  MPL_LAUNCH(c, k_mg_prolong<T>, ng, 256, geo(c, l + 1), (const T*)P<T>(C.x), ca.nnode, ncoord_of(c, l), a.flags,
             a.nnode, a.n_nblk, x, s);
  for (int k = 0; k < c->opts.mg_smooth; ++k) MPL_TRY(sweep(false));
  return MPL_OK;
}

template <class T>
mpl_status pcg_mg(mpl_ctx* c, const double* b, double* x, int* iters, double* rel, const double* x0) {
  MPL_TRY(mg_ensure<T>(c));
  MGState& M = *c->mg;
  const LevelArrays a = arrays<T>(c, 0);
  const int ng = vgrid(a.n_nblk), ngc = (a.n_cblk + 3) / 4;
  MPL_TRY(mpl_ensure(c, c->r, 8 * 3 * a.nnode));
  MPL_TRY(mpl_ensure(c, M.p, sizeof(T) * 3 * a.nnode));
  MPL_TRY(mpl_ensure(c, M.partials, sizeof(double) * 4 * (std::max(ng, ngc) + 8)));
  const int stride = std::max(ng, ngc) + 8;
  double* pk = P<double>(M.partials);
  double* pm = pk + stride;
  double* pa = pm + stride;
  double* pb = pa + stride;
  double* r = P<double>(c->r);
  T* p = P<T>(M.p);
  MGLevel& L0 = M.lev[0];
  T* pieces = P<T>(L0.pieces);
  SolverScalars* s = c->dscal();
  const T* z = P<T>(L0.x);
  // start
  if (x0) {
    T* u0 = P<T>(L0.res);
    MPL_LAUNCH(c, k_mgpcg_cast<T>, (int)((a.nnode + 255) / 256), 256, x0, a.flags, a.nnode, u0);
    MPL_TRY(mpl_level_hv_pieces<T>(c, a, u0, pieces, nullptr));
    MPL_LAUNCH(c, k_mgpcg_init<T>, ng, 256, b, x0, (const T*)u0, (const T*)pieces,
               (const T*)pieces + 3 * a.ncell, a.n_nbr_cell, a.ncell, a.mi, a.flags, a.nnode, a.n_nblk, x, r,
               pa, pb);
  } else {
    MPL_LAUNCH(c, k_mgpcg_init<T>, ng, 256, b, (const double*)nullptr, (const T*)nullptr, (const T*)nullptr,
               (const T*)nullptr, a.n_nbr_cell, a.ncell, a.mi, a.flags, a.nnode, a.n_nblk, x, r, pa, pb);
  }
  const double rtol2 = c->opts.pcg_rtol * c->opts.pcg_rtol;
  MPL_LAUNCH(c, k_mg_reduce<MG_SETUP>, 1, 1024, pa, ng, pb, ng, s, rtol2);
  MPL_TRY((vcycle<T, double>(c, 0, r, s)));
  MPL_LAUNCH(c, k_mgpcg_dot<T>, ng, 256, r, z, a.nnode, a.n_nblk, pa, s);
  MPL_LAUNCH(c, k_mg_reduce<MG_RZ0>, 1, 1024, pa, ng, pa, 0, s, 0.0);
  MPL_LAUNCH(c, (k_mgpcg_dir<T, true>), ng, 256, z, a.mi, a.flags, a.nnode, a.n_nblk, p, pm, s);
  const int check = std::max(1, c->opts.pcg_check_every);
  int launched = 0;
  for (;;) {
    MPL_TRY(mpl_sync_scalars(c));
    if (c->hscal.done != 0 || launched >= c->opts.max_pcg) break;
    const int n = std::min(check, c->opts.max_pcg - launched);
    for (int k = 0; k < n; ++k) {
      MPL_TRY(mpl_level_hv_pieces<T>(c, a, p, pieces, s, pk));
      MPL_LAUNCH(c, k_mg_reduce<MG_ALPHA>, 1, 1024, pk, ngc, pm, ng, s, 0.0);
      MPL_LAUNCH(c, k_mgpcg_update<T>, ng, 256, p, (const T*)pieces, (const T*)pieces + 3 * a.ncell, a.n_nbr_cell,
                 a.ncell, a.mi, a.flags, a.nnode, a.n_nblk, x, r, pb, s);
      MPL_LAUNCH(c, k_mg_reduce<MG_CHECK>, 1, 1024, pb, ng, pb, 0, s, 0.0);
      MPL_TRY((vcycle<T, double>(c, 0, r, s)));
      MPL_LAUNCH(c, k_mgpcg_dot<T>, ng, 256, r, z, a.nnode, a.n_nblk, pa, s);
      MPL_LAUNCH(c, k_mg_reduce<MG_BETA>, 1, 1024, pa, ng, pa, 0, s, 0.0);
      MPL_LAUNCH(c, (k_mgpcg_dir<T, false>), ng, 256, z, a.mi, a.flags, a.nnode, a.n_nblk, p, pm, s);
    }
    launched += n;
  }
  if (iters) *iters = c->hscal.iters;
  if (rel) *rel = c->hscal.bnorm2 > 0.0 ? std::sqrt(c->hscal.rr / c->hscal.bnorm2) : 0.0;
  if (c->hscal.done == 2 && c->hscal.iters == 0 && c->hscal.bnorm2 > 0.0)
    return mpl_fail(c, MPL_ERR_NONFINITE, "multigrid PCG breakdown (r.z or p.Hp <= 0 or not finite)");
  return MPL_OK;
}

}  // namespace

mpl_status mpl_stage_pcg_mg(mpl_ctx* c, const double* b, double* x, int* iters, double* rel, const double* x0) {
  if (!c->tangent_built) return mpl_fail(c, MPL_ERR_STATE, "PCG before tangent");
  if (c->tangent_precision == MPL_F32) return pcg_mg<float>(c, b, x, iters, rel, x0);
  return pcg_mg<double>(c, b, x, iters, rel, x0);
}

void mpl_mg_destroy(mpl_ctx* c) {
  if (!c->mg) return;
  MGState& M = *c->mg;
  for (MGLevel& L : M.lev) {
    DevBuf* all[] = {&L.cflag, &L.cmap, &L.nflag, &L.nmap, &L.ccoord, &L.ncoord, &L.c_nbr_node, &L.n_nbr_cell,
                     &L.scan, &L.cmask, &L.ccnt, &L.coff, &L.Abar, &L.mi, &L.flags, &L.D, &L.Dt, &L.mt,
                     &L.x, &L.b, &L.res, &L.pieces, &L.part};
    for (DevBuf* b : all)
      if (b->p) mpl_dev_free(c, b->p, b->bytes);
  }
  DevBuf* rest[] = {&M.counts, &M.pw, &M.rblk, &M.p, &M.partials};
  for (DevBuf* b : rest)
    if (b->p) mpl_dev_free(c, b->p, b->bytes);
  delete c->mg;
  c->mg = nullptr;
}

extern "C" {

mpl_status mpl_mg_apply(mpl_ctx* c, const double* r, double* z, int32_t* n_levels, double* omega) {
  if (!c || !r || !z) return MPL_ERR_INVALID_ARG;
  if (!c->tangent_built) return mpl_fail(c, MPL_ERR_STATE, "mpl_mg_apply needs a tangent");
  const bool f32 = c->tangent_precision == MPL_F32;
  MPL_TRY(f32 ? mg_ensure<float>(c) : mg_ensure<double>(c));
  MGState& M = *c->mg;
  const int64_t nnode = (int64_t)c->nnode_alloc();
  MPL_TRY(mpl_ensure(c, M.rblk, 8 * 3 * nnode));
  MPL_TRY(mpl_dense_to_block_nodes(c, r, M.rblk.p, 3, 0));
  if (f32) MPL_TRY((vcycle<float, double>(c, 0, P<double>(M.rblk), nullptr)));
  else MPL_TRY((vcycle<double, double>(c, 0, P<double>(M.rblk), nullptr)));
  // the cycle's output in FP64 block layout (rblk is free again), then dense
  const int64_t n3 = 3 * nnode;
  if (f32) MPL_LAUNCH(c, k_mg_to_f64<float>, (int)((n3 + 255) / 256), 256, P<float>(M.lev[0].x), P<double>(M.rblk), n3);
  else MPL_LAUNCH(c, k_mg_to_f64<double>, (int)((n3 + 255) / 256), 256, P<double>(M.lev[0].x), P<double>(M.rblk), n3);
  MPL_TRY(mpl_block_to_dense_nodes(c, M.rblk.p, z, 3, 0));
  if (n_levels) *n_levels = M.nlev;
  if (omega)
    for (int l = 0; l < M.nlev; ++l) omega[l] = M.lev[l].omega;
  MPL_HIP(c, hipStreamSynchronize(c->stream));
  return MPL_OK;
}

mpl_status mpl_mg_export(mpl_ctx* c, int32_t level, int32_t field, double* out) {
  if (!c || !out) return MPL_ERR_INVALID_ARG;
  if (!c->tangent_built) return mpl_fail(c, MPL_ERR_STATE, "mpl_mg_export needs a tangent");
  if (field < 0 || field > 3) return mpl_fail(c, MPL_ERR_INVALID_ARG, "mpl_mg_export: field 0..3");
  const bool f32 = c->tangent_precision == MPL_F32;
  MPL_TRY(f32 ? mg_ensure<float>(c) : mg_ensure<double>(c));
  MGState& M = *c->mg;
  if (level < 1 || level >= M.nlev) return mpl_fail(c, MPL_ERR_INVALID_ARG, "mpl_mg_export: level out of range");
  MGLevel& L = M.lev[level];
  const int d0 = L.dims[0], d1 = L.dims[1], d2 = L.dims[2];
  const int64_t rows = field == 2 ? (int64_t)d0 * d1 * d2 : (int64_t)(d0 + 1) * (d1 + 1) * (d2 + 1);
  const int64_t n = rows * (field == 2 ? 81 : field == 3 ? 3 : 1);
  MPL_LAUNCH(c, k_mg_fill, (int)((n + 255) / 256), 256, out, n);
  if (field == 2) {
    if (f32)
      MPL_LAUNCH(c, k_mg_export_tangent<float>, L.n_cblk, 64, P<float>(L.Abar), P<uint64_t>(L.cmask),
                 P<int32_t>(L.coff), P<int4>(L.ccoord), d1, d2, out);
    else
      MPL_LAUNCH(c, k_mg_export_tangent<double>, L.n_cblk, 64, P<double>(L.Abar), P<uint64_t>(L.cmask),
                 P<int32_t>(L.coff), P<int4>(L.ccoord), d1, d2, out);
  } else {
    MPL_LAUNCH(c, k_mg_export_nodes, L.n_nblk, 64, P<int4>(L.ncoord), d0, d1, d2, P<double>(L.mi), P<uint8_t>(L.flags),
               P<double>(L.D), L.nnode(), field, out);
  }
  MPL_HIP(c, hipStreamSynchronize(c->stream));
  return MPL_OK;
}

}  // extern "C"
