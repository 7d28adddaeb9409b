// Unload (Alg. 2; Sec. 3.1-3.3): particle binning, Kirchhoff stress per
// particle, particle -> cell-centre scatter and centre -> node gather.
//
// Scatter design (no atomics on floating point, deterministic):
//   * particles are counting-sorted by their base dual cell b = floor(x/dx - 1/2)
//     (integer atomics only; each bin is then ordered by particle index);
//   * one wavefront owns one active 4x4x4 cell block, one lane per cell: at
//     step i every lane takes the i-th particle of its cell and adds its
//     weighted values to the 8 target centres b + delta in a 5x5x5 centre
//     tile in LDS, corner by corner (for one corner the 64 cells reach 64
//     distinct centres, so the adds of one instruction never collide);
//   * tiles overlap their +x/+y/+z neighbours by one layer: every block
//     stores its own 64 centres directly and the 61 centres of its halo into
//     a per-block staging slot; a second pass (one wave per block) adds to
//     each centre the halo slots of the up to 7 blocks at -x/-y/-z in a fixed
//     order and normalises (no read-modify-write, one launch each).
#include <algorithm>
#include <cmath>

#include "mpl_grid.h"

using namespace mpl;

namespace {

struct ParticlesDev {
  const double *x, *v, *F, *G, *m, *V;
  const int32_t* mat;
  int64_t n;
};


__global__ void k_mark(ParticlesDev P, GridDev g, int32_t* __restrict__ pcell,
                       int32_t* __restrict__ cflag, int32_t* __restrict__ err) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P.n) return;
  int b[3];
  bool ok = true;
  for (int a = 0; a < 3; ++a) {
    double xi = (P.x[3 * p + a] - g.origin[a]) / g.dx - 0.5;
    if (!(xi >= 0.0 && xi < 1e9)) { ok = false; b[a] = 0; continue; }
    double fb = floor(xi);
    b[a] = (int)fb;
    if (b[a] + 1 > g.dims[a] - 1) ok = false;
  }
  if (!ok) {
    atomicOr(err, 1);
    pcell[p] = -1;
    return;
  }
  pcell[p] = (b[0] * g.dims[1] + b[1]) * g.dims[2] + b[2];
  for (int d = 0; d < 8; ++d) {
    int cx = (b[0] + ((d >> 2) & 1)) >> 2, cy = (b[1] + ((d >> 1) & 1)) >> 2, cz = (b[2] + (d & 1)) >> 2;
    cflag[(cx * g.cbd[1] + cy) * g.cbd[2] + cz] = 1;
  }
}

__global__ void k_compact_cells(const int32_t* __restrict__ cflag, const int32_t* __restrict__ scan,
                                int32_t* __restrict__ cmap, int4* __restrict__ ccoord,
                                int32_t* __restrict__ nflag, GridDev g, int ndense) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ndense) return;
  if (!cflag[i]) {
    cmap[i] = -1;
    return;
  }
  int id = scan[i];
  cmap[i] = id;
  int bz = i % g.cbd[2], by = (i / g.cbd[2]) % g.cbd[1], bx = i / (g.cbd[1] * g.cbd[2]);
  ccoord[id] = make_int4(bx, by, bz, 0);
  for (int d = 0; d < 8; ++d) {
    int nx = bx + ((d >> 2) & 1), ny = by + ((d >> 1) & 1), nz = bz + (d & 1);
    nflag[(nx * g.nbd[1] + ny) * g.nbd[2] + nz] = 1;
  }
}

__global__ void k_compact_nodes(const int32_t* __restrict__ nflag, const int32_t* __restrict__ scan,
                                int32_t* __restrict__ nmap, int4* __restrict__ ncoord, GridDev g,
                                int ndense) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ndense) return;
  if (!nflag[i]) {
    nmap[i] = -1;
    return;
  }
  int id = scan[i];
  nmap[i] = id;
  int bz = i % g.nbd[2], by = (i / g.nbd[2]) % g.nbd[1], bx = i / (g.nbd[1] * g.nbd[2]);
  ncoord[id] = make_int4(bx, by, bz, 0);
}

__global__ void k_neighbours(const int4* __restrict__ ccoord, const int4* __restrict__ ncoord,
                             const int32_t* __restrict__ cmap, const int32_t* __restrict__ nmap,
                             int32_t* __restrict__ c_nbr_node, int32_t* __restrict__ n_nbr_cell,
                             GridDev g, int n_cblk, int n_nblk) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_cblk) {
    int4 b = ccoord[i];
    for (int o = 0; o < 8; ++o) {
      int nx = b.x + ((o >> 2) & 1), ny = b.y + ((o >> 1) & 1), nz = b.z + (o & 1);
      c_nbr_node[i * 8 + o] = nmap[(nx * g.nbd[1] + ny) * g.nbd[2] + nz];
    }
  }
  if (i < n_nblk) {
    int4 b = ncoord[i];
    for (int o = 0; o < 8; ++o) {
      int cx = b.x - ((o >> 2) & 1), cy = b.y - ((o >> 1) & 1), cz = b.z - (o & 1);
      int id = -1;
      if (cx >= 0 && cy >= 0 && cz >= 0 && cx < g.cbd[0] && cy < g.cbd[1] && cz < g.cbd[2])
        id = cmap[(cx * g.cbd[1] + cy) * g.cbd[2] + cz];
      n_nbr_cell[i * 8 + o] = id;
    }
  }
}

// Column sums of a block-major [n][ncols] int32 array (ncols <= 2) by one
// workgroup in a fixed order, written to out[0..ncols).
__global__ __launch_bounds__(1024) void k_sum_counts(const int32_t* __restrict__ part, int n, int ncols,
                                                     int32_t* __restrict__ out) {
  __shared__ int32_t sh[2][16];
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  for (int col = 0; col < ncols; ++col) {
    int32_t acc = 0;
    for (int i = t; i < n; i += 1024) acc += part[(int64_t)i * ncols + col];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (l == 0) sh[col][w] = acc;
  }
  __syncthreads();
  if (t < ncols) {
    int32_t s = 0;
    for (int k = 0; k < 16; ++k) s += sh[t][k];
    out[t] = s;
  }
}

__global__ void k_keys(const int32_t* __restrict__ pcell, const int32_t* __restrict__ cmap, GridDev g,
                       int64_t n, int32_t* __restrict__ pkey, int32_t* __restrict__ bin_count) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int c = pcell[p];
  int bz = c % g.dims[2], by = (c / g.dims[2]) % g.dims[1], bx = c / (g.dims[1] * g.dims[2]);
  int blk = cmap[((bx >> 2) * g.cbd[1] + (by >> 2)) * g.cbd[2] + (bz >> 2)];
  int key = blk * MPL_BC + local_index(bx & 3, by & 3, bz & 3);
  pkey[p] = key;
  atomicAdd(&bin_count[key], 1);
}

__global__ void k_scatter(const int32_t* __restrict__ pkey, const int32_t* __restrict__ bin_start,
                          int32_t* __restrict__ bin_fill, int32_t* __restrict__ sorted, int64_t n) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int key = pkey[p];
  int pos = bin_start[key] + atomicAdd(&bin_fill[key], 1);
  sorted[pos] = (int32_t)p;
}

// Order each bin by particle index so that every later sum is reproducible.
__global__ void k_sort_bins(const int32_t* __restrict__ bin_start, int32_t* __restrict__ sorted,
                            int nbins) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbins) return;
  int s = bin_start[b], e = bin_start[b + 1];
  for (int i = s + 1; i < e; ++i) {
    int v = sorted[i];
    int j = i - 1;
    while (j >= s && sorted[j] > v) {
      sorted[j + 1] = sorted[j];
      --j;
    }
    sorted[j + 1] = v;
  }
}

// Accumulator slots per centre: 0 mass, 1-3 momentum, 4-12 mass-weighted G,
// then per material k: 13+7k volume, 14+7k..19+7k V*tau (xx,yy,zz,xy,yz,xz).
//
// One lane per cell of the block: at step i every lane takes the i-th
// particle of its own cell (bins are sorted by particle index) and adds its
// weighted values to the 8 centres of the cell in a 5x5x5 LDS tile, corner
// by corner.  For one corner offset the 64 cells of a block reach 64
// distinct tile slots, so the read-modify-write of one instruction never
// collides between lanes; LDS operations of a wave complete in issue order,
// and a compiler barrier between corners keeps that order in the code.  A
// lane with no particle at step i adds zeros.  Each slot thus sums its
// contributions in a fixed order (step, then corner), independent of timing.
template <int K>
__global__ __launch_bounds__(64) void k_p2c(ParticlesDev P, GridDev g,
                                            const int32_t* __restrict__ sorted,
                                            const int32_t* __restrict__ bin_start,
                                            const int4* __restrict__ ccoord,
                                            const int32_t* __restrict__ cmap,
                                            double* __restrict__ mc, double* __restrict__ qc,
                                            double* __restrict__ Gc, double* __restrict__ Vk,
                                            double* __restrict__ Tk, int64_t ncell,
                                            double* __restrict__ halo, int32_t* __restrict__ err,
    const MatParams* __restrict__ mats) {
  constexpr int NV = 13 + 7 * K;
  __shared__ double tile[NV][128];
  const int lane = threadIdx.x;
  const int cb = blockIdx.x;
  const int4 bc = ccoord[cb];
  for (int v = 0; v < NV; ++v) {
    tile[v][lane] = 0.0;
    tile[v][lane + 64] = 0.0;
  }
  const int s = bin_start[cb * MPL_BC + lane], e = bin_start[cb * MPL_BC + lane + 1];
  int nmax = e - s;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) nmax = max(nmax, __shfl_xor(nmax, off, 64));
  const int lx = lane >> 4, ly = (lane >> 2) & 3, lz = lane & 3;
  const int t0 = (lx * 5 + ly) * 5 + lz;
  __syncthreads();
  for (int i = 0; i < nmax; ++i) {
    const bool valid = s + i < e;
    double f[3], xp[3], vp[3], Gp[9], tau[6] = {0, 0, 0, 0, 0, 0}, mp = 0.0, Vp = 0.0;
    int k = 0;
    if (valid) {
      const int p = sorted[s + i];
      for (int a = 0; a < 3; ++a) {
        xp[a] = P.x[3 * p + a];
        vp[a] = P.v[3 * p + a];
        double xi = (xp[a] - g.origin[a]) / g.dx - 0.5;
        f[a] = xi - floor(xi);
      }
      for (int j = 0; j < 9; ++j) Gp[j] = P.G ? P.G[9 * p + j] : 0.0;
      mp = P.m[p];
      Vp = P.V[p];
      k = P.mat[p];
      double F[9];
      for (int j = 0; j < 9; ++j) F[j] = P.F[9 * p + j];
      if (k < 0 || k >= K || !kirchhoff(mats[k], F, tau)) {
        atomicOr(err, 2);
        for (int j = 0; j < 6; ++j) tau[j] = 0.0;
        if (k < 0 || k >= K) k = 0;
      }
    } else {
      for (int a = 0; a < 3; ++a) f[a] = xp[a] = vp[a] = 0.0;
      for (int j = 0; j < 9; ++j) Gp[j] = 0.0;
    }
    double* const mat_slot = &tile[13 + 7 * k][0];
#pragma unroll
    for (int d = 0; d < 8; ++d) {
      const int dx = (d >> 2) & 1, dy = (d >> 1) & 1, dz = d & 1;
      const double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) * (dz ? f[2] : 1.0 - f[2]);
      const int t = t0 + (dx * 5 + dy) * 5 + dz;
      double rc[3];
      rc[0] = g.origin[0] + ((bc.x * 4 + lx + dx) + 0.5) * g.dx - xp[0];
      rc[1] = g.origin[1] + ((bc.y * 4 + ly + dy) + 0.5) * g.dx - xp[1];
      rc[2] = g.origin[2] + ((bc.z * 4 + lz + dz) + 0.5) * g.dx - xp[2];
      const double wm = valid ? w * mp : 0.0;
      const double wV = valid ? w * Vp : 0.0;
      double val[20];
      val[0] = wm;
#pragma unroll
      for (int a = 0; a < 3; ++a)
        val[1 + a] = wm * (vp[a] + (Gp[a * 3] * rc[0] + Gp[a * 3 + 1] * rc[1] + Gp[a * 3 + 2] * rc[2]));
#pragma unroll
      for (int j = 0; j < 9; ++j) val[4 + j] = wm * Gp[j];
      val[13] = wV;
#pragma unroll
      for (int j = 0; j < 6; ++j) val[14 + j] = wV * tau[j];
#pragma unroll
      for (int v = 0; v < 13; ++v) tile[v][t] += val[v];
#pragma unroll
      for (int j = 0; j < 7; ++j) mat_slot[j * 128 + t] += val[13 + j];
      __asm__ __volatile__("" ::: "memory");
    }
  }
  __syncthreads();
  // own centres: plain stores (this block is their only writer in this pass)
  {
    const int t = ((lane >> 4) * 5 + ((lane >> 2) & 3)) * 5 + (lane & 3);
    const int64_t ci = (int64_t)cb * MPL_BC + lane;
    mc[ci] = tile[0][t];
    for (int a = 0; a < 3; ++a) qc[a * ncell + ci] = tile[1 + a][t];
    for (int e2 = 0; e2 < 9; ++e2) Gc[e2 * ncell + ci] = tile[4 + e2][t];
    for (int kk = 0; kk < K; ++kk) {
      Vk[kk * ncell + ci] = tile[13 + 7 * kk][t];
      for (int j = 0; j < 6; ++j) Tk[(kk * 6 + j) * ncell + ci] = tile[14 + 7 * kk + j][t];
    }
  }
  // halo centres: staged per block ([value][block][64 slots]); a nonzero
  // contribution to a centre outside the grid is a stencil leaving it
  if (lane < 61) {
    int tx, ty, tz;
    halo_tile(lane, tx, ty, tz);
    const int t = (tx * 5 + ty) * 5 + tz;
    const int gx = bc.x * 4 + tx, gy = bc.y * 4 + ty, gz = bc.z * 4 + tz;
    const bool inside = gx < g.dims[0] && gy < g.dims[1] && gz < g.dims[2];
    bool any = false;
    for (int v = 0; v < NV; ++v) {
      const double val = tile[v][t];
      any = any || (val != 0.0);
      halo[((int64_t)v * gridDim.x + cb) * MPL_BC + lane] = val;
    }
    if (any) {
      // the receiving block must exist (else a stencil left the grid or the
      // active-block marking missed it)
      if (!inside) atomicOr(err, 4);
      else if (cmap[((gx >> 2) * g.cbd[1] + (gy >> 2)) * g.cbd[2] + (gz >> 2)] < 0) atomicOr(err, 4);
    }
  }
}

// Second pass of the scatter: own value + halo slots of the blocks at
// -x/-y/-z (fixed order), then Alg. 2 normalisation
//   v_c = (mv)_c / m_c, G_c = (mG)_c / m_c, tau_{c,k} = (V tau)_{c,k} / V_{c,k}.
template <int K>
__global__ __launch_bounds__(64) void k_p2c_combine(const int* __restrict__ c_nbr_node,
                                                    const int* __restrict__ n_nbr_cell, int n_cblk,
                                                    const double* __restrict__ halo,
                                                    double* __restrict__ mc, double* __restrict__ qc,
                                                    double* __restrict__ Gc, double* __restrict__ Vk,
                                                    double* __restrict__ Tk, int64_t ncell,
                                                    int32_t* __restrict__ count, int32_t* __restrict__ err) {
  constexpr int NV = 13 + 7 * K;
  const int cb = blockIdx.x, l = threadIdx.x;
  const int64_t ci = (int64_t)cb * MPL_BC + l;
  double acc[NV];
  acc[0] = mc[ci];
#pragma unroll
  for (int a = 0; a < 3; ++a) acc[1 + a] = qc[a * ncell + ci];
#pragma unroll
  for (int e2 = 0; e2 < 9; ++e2) acc[4 + e2] = Gc[e2 * ncell + ci];
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    acc[13 + 7 * kk] = Vk[kk * ncell + ci];
#pragma unroll
    for (int j = 0; j < 6; ++j) acc[14 + 7 * kk + j] = Tk[(kk * 6 + j) * ncell + ci];
  }
  // the co-located node block lists the cell blocks at -{0,1}^3
  const int nb = c_nbr_node[cb * 8];
  int o[7], slot[7];
  bool need[7];
  halo_sources(l, o, slot, need);
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    if (!need[k]) continue;
    const int src = n_nbr_cell[nb * 8 + o[k]];
    if (src < 0) continue;
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += halo[((int64_t)v * n_cblk + src) * MPL_BC + slot[k]];
  }
  const double m = acc[0];
  if (m != 0.0) {
#pragma unroll
    for (int v = 1; v < 13; ++v) acc[v] /= m;
  }
  {
    // occupied-cell count of the block (one wave), summed by k_sum_counts
    const uint64_t bm = __ballot(m != 0.0);
    if (l == 0) count[cb] = (int32_t)__popcll(bm);
  }
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const double V = acc[13 + 7 * kk];
    if (V != 0.0)
#pragma unroll
      for (int j = 0; j < 6; ++j) acc[14 + 7 * kk + j] /= V;
  }
  mc[ci] = acc[0];
#pragma unroll
  for (int a = 0; a < 3; ++a) qc[a * ncell + ci] = acc[1 + a];
#pragma unroll
  for (int e2 = 0; e2 < 9; ++e2) Gc[e2 * ncell + ci] = acc[4 + e2];
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    Vk[kk * ncell + ci] = acc[13 + 7 * kk];
#pragma unroll
    for (int j = 0; j < 6; ++j) Tk[(kk * 6 + j) * ncell + ci] = acc[14 + 7 * kk + j];
  }
  (void)err;
}

// Tangent-carrying cells (some V_{c,k} != 0) per cell block: 64-bit mask
// and count, for the compact tangent storage.
__global__ __launch_bounds__(64) void k_cell_mask(const double* __restrict__ Vk, int64_t ncell, int K,
                                                  uint64_t* __restrict__ cmask,
                                                  int32_t* __restrict__ ccnt) {
  const int cb = blockIdx.x, l = threadIdx.x;
  const int64_t ci = (int64_t)cb * MPL_BC + l;
  bool act = false;
  for (int k = 0; k < K; ++k) act = act || (Vk[k * ncell + ci] != 0.0);
  const uint64_t m = __ballot(act);
  if (l == 0) {
    cmask[cb] = m;
    ccnt[cb] = __popcll(m);
  }
}

// Sec. 3.3 centre -> node gather with w_ic = 1/8 (race-free: every node
// gathers from its own 8 cells), then Dirichlet sets and vhat.  One wave per
// node block (XCD-major); the block's 5x5x5 centre tile goes through LDS so
// that every centre value is read from memory once per block, not once per
// corner.
__global__ __launch_bounds__(64) void k_c2n(GridDev g, const int32_t* __restrict__ n_nbr_cell,
                                            const int4* __restrict__ ncoord,
                                            const double* __restrict__ mc,
                                            const double* __restrict__ vc,
                                            const double* __restrict__ Gc, int64_t ncell,
                                            int64_t nnode, int n_nblk, const BCDev* __restrict__ bcp,
                                            double time, double dt,
                                            double gx, double gy, double gz,
                                            double* __restrict__ mi, double* __restrict__ vn,
                                            double* __restrict__ vhat, double* __restrict__ v,
                                            uint8_t* __restrict__ flags,
                                            int32_t* __restrict__ counts) {
  const int nb = xcd_block(blockIdx.x, n_nblk), l = threadIdx.x;
  if (nb >= n_nblk) return;
  const int64_t ni = (int64_t)nb * MPL_BC + l;
  // the 5x5x5 tile of centres around the block's nodes (cells -1..3 along
  // each axis, from the block and its -x/-y/-z neighbours) is staged in LDS
  // once: m, v (3) and G (9) per centre, zeros for absent blocks
  __shared__ double tile[13][128];
  for (int t = l; t < 125; t += 64) {
    const int cx = t / 25 - 1, cy = (t / 5) % 5 - 1, cz = t % 5 - 1;
    const int o = ((cx < 0) * 2 + (cy < 0)) * 2 + (cz < 0);
    const int blk = n_nbr_cell[nb * 8 + o];
    const int64_t ci = (int64_t)(blk < 0 ? 0 : blk) * MPL_BC + local_index(cx & 3, cy & 3, cz & 3);
    double val[13];
    val[0] = mc[ci];
#pragma unroll
    for (int a = 0; a < 3; ++a) val[1 + a] = vc[a * ncell + ci];
#pragma unroll
    for (int e = 0; e < 9; ++e) val[4 + e] = Gc[e * ncell + ci];
#pragma unroll
    for (int v2 = 0; v2 < 13; ++v2) tile[v2][t] = blk < 0 ? 0.0 : val[v2];
  }
  __syncthreads();
  double m = 0.0, q[3] = {0.0, 0.0, 0.0};
  // corner by corner in a fixed order; an absent or empty centre has m = 0,
  // enters with weight 0 and adds exact zeros
  const int lx = local_x(l), ly = local_y(l), lz = local_z(l);
#pragma unroll
  for (int d = 0; d < 8; ++d) {
    const int dx = (d >> 2) & 1, dy = (d >> 1) & 1, dz = d & 1;
    const int t = ((lx - dx + 1) * 5 + (ly - dy + 1)) * 5 + (lz - dz + 1);
    const double wm = tile[0][t] / 8.0;
    const double r[3] = {(dx - 0.5) * g.dx, (dy - 0.5) * g.dx, (dz - 0.5) * g.dx};
    m += wm;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double aff = tile[4 + a * 3][t] * r[0] + tile[5 + a * 3][t] * r[1] + tile[6 + a * 3][t] * r[2];
      q[a] += wm * (tile[1 + a][t] + aff);
    }
  }
  double vv[3] = {0.0, 0.0, 0.0};
  if (m != 0.0)
    for (int a = 0; a < 3; ++a) vv[a] = q[a] / m;
  uint8_t fl = 0;
  double vf[3] = {0.0, 0.0, 0.0};
  int fixmask = 0;  // the prescribed components, one bit each
  if (m != 0.0) {
    fl |= MPL_NODE_ACTIVE;
    int4 bcrd = ncoord[nb];
    int idx[3] = {bcrd.x * 4 + local_x(l), bcrd.y * 4 + local_y(l), bcrd.z * 4 + local_z(l)};
    double xn[3];
    for (int a = 0; a < 3; ++a) xn[a] = g.origin[a] + idx[a] * g.dx;
    const double eps = 1e-6 * g.dx;
    const BCDev& bcs = *bcp;
    for (int b = 0; b < bcs.n; ++b) {
      bool in = true;
      for (int a = 0; a < 3; ++a) {
        double sh = (bcs.kind[b] == MPL_BC_MOVING_BOX) ? bcs.vel[b][a] * time : 0.0;
        if (xn[a] < bcs.lo[b][a] + sh - eps || xn[a] > bcs.hi[b][a] + sh + eps) in = false;
      }
      if (!in) continue;
      if (bcs.kind[b] == MPL_BC_SLIP_PLANE) {
        // a frictionless wall fixes the normal component only, to 0
        fixmask |= 1 << bcs.axis[b];
        vf[bcs.axis[b]] = 0.0;
        continue;
      }
      fixmask = 7;
      for (int a = 0; a < 3; ++a) vf[a] = (bcs.kind[b] == MPL_BC_MOVING_BOX) ? bcs.vel[b][a] : 0.0;
    }
    if (fixmask) fl |= MPL_NODE_FIXED;
    fl |= (uint8_t)(((~fixmask) & 7) << 2);
  }
  {
    // active node and free component counts of the block (one wave),
    // summed later by k_sum_counts: device-scope atomics on one address
    // from every wave serialise at the memory side
    const uint64_t ba = __ballot((fl & MPL_NODE_ACTIVE) != 0);
    int nfree = 0;
    for (int a = 0; a < 3; ++a) nfree += __popcll(__ballot(mpl_free(fl, a)));
    if (l == 0) {
      counts[2 * nb] = (int32_t)__popcll(ba);
      counts[2 * nb + 1] = nfree;
    }
  }
  const double grav[3] = {gx, gy, gz};
  mi[ni] = m;
  flags[ni] = fl;
  for (int a = 0; a < 3; ++a) {
    double vh = mpl_free(fl, a) ? vv[a] + dt * grav[a] : (((fixmask >> a) & 1) ? vf[a] : 0.0);
    vn[a * nnode + ni] = vv[a];
    vhat[a * nnode + ni] = vh;
    v[a * nnode + ni] = vh;
  }
}

}  // namespace

static GridDev level_grid(const int dims[3], const int cbd[3], const int nbd[3]) {
  GridDev g{};
  for (int a = 0; a < 3; ++a) {
    g.dims[a] = dims[a];
    g.cbd[a] = cbd[a];
    g.nbd[a] = nbd[a];
  }
  return g;
}

mpl_status mpl_block_maps(mpl_ctx* c, const int dims[3], const int cbd[3], const int nbd[3],
                          int32_t* cflag, int32_t* cmap, int4* ccoord, int32_t* nflag,
                          int32_t* nmap, int4* ncoord, int32_t* scan, int32_t* totals_dev) {
  const GridDev g = level_grid(dims, cbd, nbd);
  const int ncb = cbd[0] * cbd[1] * cbd[2], nnb = nbd[0] * nbd[1] * nbd[2];
  const int TPB = 256;
  int32_t* scan_c = scan;
  int32_t* scan_n = scan + ncb + 1;
  MPL_TRY(mpl_scan_i32(c, cflag, scan_c, ncb, totals_dev));
  MPL_LAUNCH(c, k_compact_cells, (ncb + TPB - 1) / TPB, TPB, cflag, scan_c, cmap, ccoord, nflag, g, ncb);
  MPL_TRY(mpl_scan_i32(c, nflag, scan_n, nnb, totals_dev + 1));
  MPL_LAUNCH(c, k_compact_nodes, (nnb + TPB - 1) / TPB, TPB, nflag, scan_n, nmap, ncoord, g, nnb);
  return MPL_OK;
}

mpl_status mpl_block_neighbours(mpl_ctx* c, const int dims[3], const int cbd[3], const int nbd[3],
                                const int4* ccoord, const int4* ncoord, const int32_t* cmap,
                                const int32_t* nmap, int32_t* c_nbr_node, int32_t* n_nbr_cell,
                                int n_cblk, int n_nblk) {
  const GridDev g = level_grid(dims, cbd, nbd);
  const int mx = std::max(n_cblk, n_nblk), TPB = 256;
  MPL_LAUNCH(c, k_neighbours, (mx + TPB - 1) / TPB, TPB, ccoord, ncoord, cmap, nmap, c_nbr_node,
             n_nbr_cell, g, n_cblk, n_nblk);
  return MPL_OK;
}

mpl_status mpl_stage_unload(mpl_ctx* c, const Parts64* in, double dt, const double* gravity,
                            const mpl_bc* bcs, int n_bcs, double time) {
  if (!in || in->n < 0 ||
      (in->n > 0 && (!in->x || !in->v || !in->F || !in->G || !in->m || !in->V0 || !in->mat)))
    return mpl_fail(c, MPL_ERR_INVALID_ARG, "particle arrays missing");
  if (n_bcs < 0 || n_bcs > 16 || (n_bcs > 0 && !bcs))
    return mpl_fail(c, MPL_ERR_INVALID_ARG, "at most 16 boundary boxes");
  if (!(dt > 0.0)) return mpl_fail(c, MPL_ERR_INVALID_ARG, "dt must be positive");
  for (int b = 0; b < n_bcs; ++b) {
    const int k = bcs[b].kind;
    if (k != MPL_BC_STICKY_BOX && k != MPL_BC_MOVING_BOX && k != MPL_BC_SLIP_PLANE)
      return mpl_fail(c, MPL_ERR_INVALID_ARG, "unknown boundary condition kind");
    if (k == MPL_BC_SLIP_PLANE) {
      int nz = 0;
      for (int a = 0; a < 3; ++a) nz += bcs[b].velocity[a] != 0.0;
      if (nz != 1) return mpl_fail(c, MPL_ERR_INVALID_ARG, "a slip plane's normal must name one axis");
    }
  }
  c->unloaded = c->reconstructed = c->tangent_built = c->solved = false;
  c->dt = dt;
  c->np = in->n;
  const GridDev g = grid_dev(c);
  const int ncb_dense = c->cbd[0] * c->cbd[1] * c->cbd[2];
  const int nnb_dense = c->nbd[0] * c->nbd[1] * c->nbd[2];
  const int64_t np = in->n;
  // FLIP/PIC transfer: the particles' G does not enter the grid (a null G
  // reads as zero), so G_c = 0 and the centre->node affine term vanishes
  const double* Gin = c->opts.transfer == MPL_TRANSFER_FLIP_PIC ? nullptr : in->G;
  ParticlesDev parts{in->x, in->v, in->F, Gin, in->m, in->V0, in->mat, np};

  MPL_TRY(mpl_ensure(c, c->cflag, sizeof(int32_t) * ncb_dense));
  MPL_TRY(mpl_ensure(c, c->cmap, sizeof(int32_t) * (ncb_dense + 1)));
  MPL_TRY(mpl_ensure(c, c->nflag, sizeof(int32_t) * nnb_dense));
  MPL_TRY(mpl_ensure(c, c->nmap, sizeof(int32_t) * (nnb_dense + 1)));
  MPL_TRY(mpl_ensure(c, c->ccoord, sizeof(int4) * ncb_dense));
  MPL_TRY(mpl_ensure(c, c->ncoord, sizeof(int4) * nnb_dense));
  MPL_TRY(mpl_ensure(c, c->c_nbr_node, sizeof(int32_t) * 8 * ncb_dense));
  MPL_TRY(mpl_ensure(c, c->n_nbr_cell, sizeof(int32_t) * 8 * nnb_dense));
  MPL_TRY(mpl_ensure(c, c->pcell, sizeof(int32_t) * (np + 1)));
  MPL_TRY(mpl_ensure(c, c->pkey, sizeof(int32_t) * (np + 1)));
  MPL_TRY(mpl_ensure(c, c->sorted, sizeof(int32_t) * (np + 1)));
  SolverScalars* ds = c->dscal();
  MPL_HIP(c, hipMemsetAsync(ds, 0, sizeof(SolverScalars), c->stream));
  MPL_HIP(c, hipMemsetAsync(c->cflag.p, 0, sizeof(int32_t) * ncb_dense, c->stream));
  MPL_HIP(c, hipMemsetAsync(c->nflag.p, 0, sizeof(int32_t) * nnb_dense, c->stream));

  const int TPB = 256;
  MPL_LAUNCH(c, k_mark, (int)((np + TPB - 1) / TPB), TPB, parts, g, P<int32_t>(c->pcell),
             P<int32_t>(c->cflag), &ds->err);
  // compact cell blocks (cmap doubles as scan output before it is rewritten)
  MPL_TRY(mpl_ensure(c, c->bin_count, sizeof(int32_t) * (ncb_dense + nnb_dense + 2)));
  int32_t* scan_c = P<int32_t>(c->bin_count);
  int32_t* scan_n = scan_c + ncb_dense + 1;
  MPL_TRY(mpl_scan_i32(c, P<int32_t>(c->cflag), scan_c, ncb_dense, &ds->n_cblk));
  MPL_LAUNCH(c, k_compact_cells, (ncb_dense + TPB - 1) / TPB, TPB, P<int32_t>(c->cflag), scan_c,
             P<int32_t>(c->cmap), P<int4>(c->ccoord), P<int32_t>(c->nflag), g, ncb_dense);
  MPL_TRY(mpl_scan_i32(c, P<int32_t>(c->nflag), scan_n, nnb_dense, &ds->n_nblk));
  MPL_LAUNCH(c, k_compact_nodes, (nnb_dense + TPB - 1) / TPB, TPB, P<int32_t>(c->nflag), scan_n,
             P<int32_t>(c->nmap), P<int4>(c->ncoord), g, nnb_dense);
  MPL_TRY(mpl_sync_scalars(c));
  if (c->hscal.err & 1)
    return mpl_fail(c, MPL_ERR_DOMAIN, "a particle stencil leaves the grid (or x is not finite)");
  c->n_cblk = c->hscal.n_cblk;
  c->n_nblk = c->hscal.n_nblk;
  const int mx = std::max(c->n_cblk, c->n_nblk);
  MPL_LAUNCH(c, k_neighbours, (mx + TPB - 1) / TPB, TPB, P<int4>(c->ccoord), P<int4>(c->ncoord),
             P<int32_t>(c->cmap), P<int32_t>(c->nmap), P<int32_t>(c->c_nbr_node),
             P<int32_t>(c->n_nbr_cell), g, c->n_cblk, c->n_nblk);

  // per-cell and per-node storage
  const int64_t ncell = (int64_t)c->ncell_alloc(), nnode = (int64_t)c->nnode_alloc();
  const int K = c->nmat;
  MPL_TRY(mpl_ensure(c, c->mc, 8 * ncell));
  MPL_TRY(mpl_ensure(c, c->qc, 8 * 3 * ncell));
  MPL_TRY(mpl_ensure(c, c->Gc, 8 * 9 * ncell));
  MPL_TRY(mpl_ensure(c, c->Vk, 8 * K * ncell));
  MPL_TRY(mpl_ensure(c, c->Tk, 8 * 6 * K * ncell));
  MPL_TRY(mpl_ensure(c, c->Sk, 8 * 6 * K * ncell));
  MPL_TRY(mpl_ensure(c, c->mi, 8 * nnode));
  MPL_TRY(mpl_ensure(c, c->vn, 8 * 3 * nnode));
  MPL_TRY(mpl_ensure(c, c->vhat, 8 * 3 * nnode));
  MPL_TRY(mpl_ensure(c, c->v, 8 * 3 * nnode));
  MPL_TRY(mpl_ensure(c, c->flags, nnode + 64));
  const int nbins = c->n_cblk * MPL_BC;
  MPL_TRY(mpl_ensure(c, c->bin_count, sizeof(int32_t) * (nbins + 1)));
  MPL_TRY(mpl_ensure(c, c->bin_start, sizeof(int32_t) * (nbins + 1)));
  MPL_TRY(mpl_ensure(c, c->bin_fill, sizeof(int32_t) * (nbins + 1)));
  MPL_HIP(c, hipMemsetAsync(c->bin_count.p, 0, sizeof(int32_t) * (nbins + 1), c->stream));
  MPL_HIP(c, hipMemsetAsync(c->bin_fill.p, 0, sizeof(int32_t) * (nbins + 1), c->stream));
  MPL_LAUNCH(c, k_keys, (int)((np + TPB - 1) / TPB), TPB, P<int32_t>(c->pcell), P<int32_t>(c->cmap), g,
             np, P<int32_t>(c->pkey), P<int32_t>(c->bin_count));
  int32_t* bstart = P<int32_t>(c->bin_start);
  MPL_TRY(mpl_scan_i32(c, P<int32_t>(c->bin_count), bstart, nbins, bstart + nbins));
  MPL_LAUNCH(c, k_scatter, (int)((np + TPB - 1) / TPB), TPB, P<int32_t>(c->pkey), bstart,
             P<int32_t>(c->bin_fill), P<int32_t>(c->sorted), np);
  MPL_LAUNCH(c, k_sort_bins, (nbins + TPB - 1) / TPB, TPB, bstart, P<int32_t>(c->sorted), nbins);

  // P2C: one pass over all active blocks (own centres + staged halos), then
  // the combine / normalise pass
  MPL_TRY(mpl_ensure(c, c->p2c_halo, sizeof(double) * (13 + 7 * K) * (size_t)c->n_cblk * MPL_BC + 64));
  // per-block counts: n_cblk for the combine pass, then 2 n_nblk for the gather
  MPL_TRY(mpl_ensure(c, c->cntbuf, sizeof(int32_t) * (2 * (size_t)std::max(c->n_cblk, c->n_nblk) + 64)));
#define MPL_P2C(KK)                                                                                     \
  MPL_LAUNCH(c, k_p2c<KK>, c->n_cblk, 64, parts, g, P<int32_t>(c->sorted), bstart, \
             P<int4>(c->ccoord), P<int32_t>(c->cmap), P<double>(c->mc), P<double>(c->qc), P<double>(c->Gc), \
             P<double>(c->Vk), P<double>(c->Tk), ncell, P<double>(c->p2c_halo), &ds->err, P<MatParams>(c->matbuf));             \
  MPL_LAUNCH(c, k_p2c_combine<KK>, c->n_cblk, 64, P<int>(c->c_nbr_node), P<int>(c->n_nbr_cell),         \
             c->n_cblk, P<double>(c->p2c_halo), P<double>(c->mc), P<double>(c->qc), P<double>(c->Gc),   \
             P<double>(c->Vk), P<double>(c->Tk), ncell, P<int32_t>(c->cntbuf), &ds->err);            \
  MPL_LAUNCH(c, k_sum_counts, 1, 1024, P<int32_t>(c->cntbuf), c->n_cblk, 1, &ds->n_active_cells)
  switch (K) {
    case 1: MPL_P2C(1); break;
    case 2: MPL_P2C(2); break;
    case 3: MPL_P2C(3); break;
    default: MPL_P2C(4); break;
  }
#undef MPL_P2C
  MPL_TRY(mpl_ensure(c, c->cmask, sizeof(uint64_t) * (c->n_cblk + 1)));
  MPL_TRY(mpl_ensure(c, c->ccnt, sizeof(int32_t) * (c->n_cblk + 1)));
  MPL_TRY(mpl_ensure(c, c->coff, sizeof(int32_t) * (c->n_cblk + 1)));
  MPL_LAUNCH(c, k_cell_mask, c->n_cblk, 64, P<double>(c->Vk), ncell, K, P<uint64_t>(c->cmask),
             P<int32_t>(c->ccnt));
  MPL_TRY(mpl_scan_i32(c, P<int32_t>(c->ccnt), P<int32_t>(c->coff), c->n_cblk, &ds->n_tan_cells));

  BCDev& bd = c->bc_host;
  bd = BCDev{};
  bd.n = n_bcs;
  for (int b = 0; b < n_bcs; ++b) {
    bd.kind[b] = bcs[b].kind;
    bd.axis[b] = 0;
    for (int a = 0; a < 3; ++a)
      if (bcs[b].kind == MPL_BC_SLIP_PLANE && bcs[b].velocity[a] != 0.0) bd.axis[b] = a;
    for (int a = 0; a < 3; ++a) {
      bd.lo[b][a] = bcs[b].lo[a];
      bd.hi[b][a] = bcs[b].hi[a];
      bd.vel[b][a] = bcs[b].velocity[a];
    }
  }
  MPL_TRY(mpl_ensure(c, c->bcbuf, sizeof(BCDev)));
  MPL_HIP(c, hipMemcpyAsync(c->bcbuf.p, &bd, sizeof(BCDev), hipMemcpyHostToDevice, c->stream));
  const double gz[3] = {0.0, 0.0, 0.0};
  const double* gr = gravity ? gravity : gz;
  MPL_LAUNCH(c, k_c2n, xcd_grid(c->n_nblk), 64, g, P<int32_t>(c->n_nbr_cell), P<int4>(c->ncoord),
             P<double>(c->mc), P<double>(c->qc), P<double>(c->Gc), ncell, nnode, c->n_nblk, P<BCDev>(c->bcbuf), time, dt, gr[0],
             gr[1], gr[2], P<double>(c->mi), P<double>(c->vn), P<double>(c->vhat), P<double>(c->v),
             P<uint8_t>(c->flags), P<int32_t>(c->cntbuf));
  // n_active_nodes and n_free_dofs are adjacent in SolverScalars
  MPL_LAUNCH(c, k_sum_counts, 1, 1024, P<int32_t>(c->cntbuf), c->n_nblk, 2, &ds->n_active_nodes);
  MPL_TRY(mpl_sync_scalars(c));
  if (c->hscal.err & 2) return mpl_fail(c, MPL_ERR_DOMAIN, "particle F outside the model domain (det F <= 0) or bad material id");
  if (c->hscal.err & 4) return mpl_fail(c, MPL_ERR_HIP, "internal: scatter reached an inactive block");
  c->unloaded = true;
  return MPL_OK;
}

extern "C" mpl_status mpl_unload(mpl_ctx* c, const mpl_particles* in, double dt,
                                 const double gravity[3], const mpl_bc* bcs, int32_t n_bcs,
                                 double time) {
  if (!c || !in) return MPL_ERR_INVALID_ARG;
  Parts64 pin;
  MPL_TRY(mpl_particles_in(c, in, &pin));
  return mpl_stage_unload(c, &pin, dt, gravity, bcs, n_bcs, time);
}
