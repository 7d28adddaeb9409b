// Block geometry shared by the kernels (device side).
#pragma once
#include <hip/hip_runtime.h>

#include "mpl_internal.h"

namespace mpl {

struct GridDev {
  int dims[3], cbd[3], nbd[3];
  double dx, inv_dx, origin[3];
};

inline GridDev grid_dev(const mpl_ctx* c) {
  GridDev g;
  for (int a = 0; a < 3; ++a) {
    g.dims[a] = c->dims[a];
    g.cbd[a] = c->cbd[a];
    g.nbd[a] = c->nbd[a];
    g.origin[a] = c->origin[a];
  }
  g.dx = c->dx;
  g.inv_dx = c->inv_dx;
  return g;
}

__device__ __forceinline__ int local_x(int l) { return l >> 4; }
__device__ __forceinline__ int local_y(int l) { return (l >> 2) & 3; }
__device__ __forceinline__ int local_z(int l) { return l & 3; }
__device__ __forceinline__ int local_index(int x, int y, int z) { return (x * 4 + y) * 4 + z; }

// Corner d of a cell: offsets ((d>>2)&1, (d>>1)&1, d&1); Q1 centre->node
// gradient grad w = (2 delta - 1)/(4 dx) per component (Sec. 3.3, 3-D).
__device__ __forceinline__ void corner_grad(int d, double inv4dx, double* gw) {
  gw[0] = (((d >> 2) & 1) ? 1.0 : -1.0) * inv4dx;
  gw[1] = (((d >> 1) & 1) ? 1.0 : -1.0) * inv4dx;
  gw[2] = ((d & 1) ? 1.0 : -1.0) * inv4dx;
}

// Compact node index of corner d of local cell l in cell block cb.
__device__ __forceinline__ int corner_node(const int* c_nbr_node, int cb, int l, int d) {
  int x = local_x(l) + ((d >> 2) & 1), y = local_y(l) + ((d >> 1) & 1), z = local_z(l) + (d & 1);
  int o = ((x >> 2) * 2 + (y >> 2)) * 2 + (z >> 2);
  return c_nbr_node[cb * 8 + o] * MPL_BC + local_index(x & 3, y & 3, z & 3);
}

// XCD-major workgroup mapping.  The dispatcher deals consecutive workgroups
// round-robin to the 8 XCDs, each with its own L2; mapping workgroup wg to
// block (wg mod 8) * ceil(n/8) + wg / 8 gives every XCD a contiguous range of
// blocks, so neighbouring blocks (which read the same halo lines) share one
// L2.  A bijection on [0, 8 ceil(n/8)): launch that many workgroups and let
// those with a result >= n exit.
__device__ __forceinline__ int xcd_block(int wg, int n) {
  const int per = (n + 7) >> 3;
  return (wg & 7) * per + (wg >> 3);
}
__host__ __device__ inline int xcd_grid(int n) { return ((n + 7) / 8) * 8; }

// Compact cell index of the cell c = node - delta_d around local node l of
// node block nb, or -1 when that cell block is not active.
__device__ __forceinline__ int node_cell(const int* n_nbr_cell, int nb, int l, int d) {
  int x = local_x(l) - ((d >> 2) & 1), y = local_y(l) - ((d >> 1) & 1), z = local_z(l) - (d & 1);
  int o = ((x < 0) * 2 + (y < 0)) * 2 + (z < 0);
  int blk = n_nbr_cell[nb * 8 + o];
  return blk < 0 ? -1 : blk * MPL_BC + local_index(x & 3, y & 3, z & 3);
}

// Slot of local cell l of cell block cb in the compact block-major tangent
// storage of `stride` entries per cell: entry e lives at base + e*n + rank.
struct TanSlot {
  int64_t base;
  int n, rank;
  bool active;
};
__device__ __forceinline__ TanSlot tan_slot(const uint64_t* __restrict__ cmask,
                                            const int32_t* __restrict__ coff, int cb, int l,
                                            int stride) {
  const uint64_t m = cmask[cb];
  TanSlot t;
  t.active = (m >> l) & 1ull;
  t.n = __popcll(m);
  t.rank = __popcll(m & ((1ull << l) - 1ull));
  t.base = (int64_t)stride * coff[cb];
  return t;
}

// Factored single-material FP32 tangent (37 entries per cell):
//   0-3   unit quaternion (w, x, y, z) of U, the left singular vectors of
//         F = (I + dt G) S (a proper rotation)
//   4-12  M = S V (row-major)
//   13-18 A3, the projected scaling block (00 01 02 11 12 22)
//   19-24 (a_p, b_p) of the twist/flip pairs p = (0,1), (1,2), (0,2)
//   25-36 Q_e(s): the cell's contribution to diagonal entry e = (xx, yy, zz)
//         of the 3x3 node block of H for corner sign pattern s (see
//         k_tangent), the Jacobi diagonal; with block-Jacobi the off-diagonal
//         entries (xy, yz, xz) go to a separate array of MPL_TAN_OFF entries
//         per cell in the same compact layout, so the product's reads keep
//         this layout
// so that Abar vec(g) = vec(U yhat M^T) with Ghat = U^T g M,
// diag(yhat) = A3 diag(Ghat) and, for pair (i,j), yhat_ij = a Ghat_ij + b Ghat_ji,
// yhat_ji = b Ghat_ij + a Ghat_ji.  A product reads entries 0-24.
#define MPL_TAN_DENSE 45
#define MPL_TAN_FACT 37
#define MPL_TAN_OFF 12
#define MPL_TAN_FACT_READ 25

// Rotation matrix (row-major) of a unit quaternion (w, x, y, z).
template <class T>
__host__ __device__ __forceinline__ void quat_to_rot(T w, T x, T y, T z, T* U) {
  U[0] = T(1) - T(2) * (y * y + z * z);
  U[1] = T(2) * (x * y - w * z);
  U[2] = T(2) * (x * z + w * y);
  U[3] = T(2) * (x * y + w * z);
  U[4] = T(1) - T(2) * (x * x + z * z);
  U[5] = T(2) * (y * z - w * x);
  U[6] = T(2) * (x * z - w * y);
  U[7] = T(2) * (y * z + w * x);
  U[8] = T(1) - T(2) * (x * x + y * y);
}

// Unit quaternion of a proper rotation matrix (Shepperd's method: divide by
// the largest of the four candidate squared components).
__host__ __device__ __forceinline__ void rot_to_quat(const double* U, double* q) {
  const double tr = U[0] + U[4] + U[8];
  if (tr > 0.0) {
    const double S = 2.0 * sqrt(tr + 1.0);
    q[0] = 0.25 * S; q[1] = (U[7] - U[5]) / S; q[2] = (U[2] - U[6]) / S; q[3] = (U[3] - U[1]) / S;
  } else if (U[0] > U[4] && U[0] > U[8]) {
    const double S = 2.0 * sqrt(1.0 + U[0] - U[4] - U[8]);
    q[0] = (U[7] - U[5]) / S; q[1] = 0.25 * S; q[2] = (U[1] + U[3]) / S; q[3] = (U[2] + U[6]) / S;
  } else if (U[4] > U[8]) {
    const double S = 2.0 * sqrt(1.0 + U[4] - U[0] - U[8]);
    q[0] = (U[2] - U[6]) / S; q[1] = (U[1] + U[3]) / S; q[2] = 0.25 * S; q[3] = (U[5] + U[7]) / S;
  } else {
    const double S = 2.0 * sqrt(1.0 + U[8] - U[0] - U[4]);
    q[0] = (U[3] - U[1]) / S; q[1] = (U[2] + U[6]) / S; q[2] = (U[5] + U[7]) / S; q[3] = 0.25 * S;
  }
  const double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int i = 0; i < 4; ++i) q[i] /= n;
}

// Halo slots of a 5x5x5 tile over a 4x4x4 block: the 61 tile positions with
// some coordinate equal to 4 (they belong to the +x/+y/+z neighbour blocks):
// faces 0-15 (x), 16-31 (y), 32-47 (z), edges 48-51 (xy), 52-55 (xz),
// 56-59 (yz), corner 60.
__device__ __forceinline__ void halo_tile(int l, int& tx, int& ty, int& tz) {
  if (l < 16) { tx = 4; ty = l >> 2; tz = l & 3; }
  else if (l < 32) { int k = l - 16; tx = k >> 2; ty = 4; tz = k & 3; }
  else if (l < 48) { int k = l - 32; tx = k >> 2; ty = k & 3; tz = 4; }
  else if (l < 52) { tx = 4; ty = 4; tz = l - 48; }
  else if (l < 56) { tx = 4; ty = l - 52; tz = 4; }
  else if (l < 60) { tx = l - 56; ty = 4; tz = 4; }
  else { tx = 4; ty = 4; tz = 4; }
}
__device__ __forceinline__ int halo_slot(int tx, int ty, int tz) {
  const bool X = tx == 4, Y = ty == 4, Z = tz == 4;
  if (X && Y && Z) return 60;
  if (Y && Z) return 56 + tx;
  if (X && Z) return 52 + ty;
  if (X && Y) return 48 + tz;
  if (Z) return 32 + tx * 4 + ty;
  if (Y) return 16 + tx * 4 + tz;
  return ty * 4 + tz;  // X
}
// Sources of local position l of block b in the halos of the blocks at
// -x, -y, -z, -xy, -xz, -yz, -xyz (offset index o = (ox*2+oy)*2+oz into the
// node-block neighbour list n_nbr_cell of the block's co-located node block)
// and the halo slot there; need[k] = false where l is not on that face.
__device__ __forceinline__ void halo_sources(int l, int* o, int* slot, bool* need) {
  const int lx = l >> 4, ly = (l >> 2) & 3, lz = l & 3;
  o[0] = 4; need[0] = lx == 0; slot[0] = ly * 4 + lz;
  o[1] = 2; need[1] = ly == 0; slot[1] = 16 + lx * 4 + lz;
  o[2] = 1; need[2] = lz == 0; slot[2] = 32 + lx * 4 + ly;
  o[3] = 6; need[3] = lx == 0 && ly == 0; slot[3] = 48 + lz;
  o[4] = 5; need[4] = lx == 0 && lz == 0; slot[4] = 52 + ly;
  o[5] = 3; need[5] = ly == 0 && lz == 0; slot[5] = 56 + lx;
  o[6] = 7; need[6] = lx == 0 && ly == 0 && lz == 0; slot[6] = 60;
}

// Deterministic wavefront sum (butterfly over 64 lanes).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Device flag of a CG solve: 1 converged, 2 breakdown (kernels of later
// iterations return at once).
__device__ __forceinline__ bool done_flag(const SolverScalars* s) {
  return *(volatile const int32_t*)&s->done != 0;
}

// Assemble (K p)_i for local node l of node block nb: the own partial of the
// cell block with the same coordinates plus the halo pieces of the cell
// blocks at -x, -y, -z (faces, edges, corner), summed in a fixed order.
template <class T>
__device__ __forceinline__ void gather_kp(const T* __restrict__ Hown, const T* __restrict__ Hhalo,
                                          const int* __restrict__ n_nbr_cell, int64_t ncell,
                                          int nb, int l, T* h) {
  // every load is issued unconditionally (absent sources read slot 0 and
  // add zero), so the eight sources cost one memory round trip
  const int* nbr = n_nbr_cell + nb * 8;
  int o[7], slot[7];
  bool need[7];
  halo_sources(l, o, slot, need);
  T v[8][3];
  bool use[8];
  {
    const int src = nbr[0];
    use[0] = src >= 0;
    const int64_t i = use[0] ? (int64_t)src * MPL_BC + l : 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) v[0][a] = Hown[a * ncell + i];
  }
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    const int src = nbr[o[k]];
    use[k + 1] = need[k] && src >= 0;
    const int64_t i = use[k + 1] ? (int64_t)src * MPL_BC + slot[k] : 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) v[k + 1][a] = Hhalo[a * ncell + i];
  }
  h[0] = h[1] = h[2] = T(0);
#pragma unroll
  for (int k = 0; k < 8; ++k)
#pragma unroll
    for (int a = 0; a < 3; ++a)
      if (use[k]) h[a] += v[k][a];
}

}  // namespace mpl

// node flag bits: ACTIVE (the node has mass), FIXED (a boundary condition
// prescribes at least one velocity component), and MPL_NODE_FREE_X << a
// (velocity component a is a degree of freedom of the solve)
#define MPL_NODE_ACTIVE 1
#define MPL_NODE_FIXED 2
#define MPL_NODE_FREE_X 4
#define MPL_NODE_FREE_ALL 28
__host__ __device__ __forceinline__ bool mpl_free(uint8_t fl, int a) { return (fl >> (2 + a)) & 1; }
