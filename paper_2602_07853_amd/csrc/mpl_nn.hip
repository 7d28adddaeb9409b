// Learned preconditioner: a 4-level 3-D U-Net (channels 16/32/64/128, two
// 3x3x3 convolutions per level and side, 2x2x2 stride-2 down/up sampling,
// skip concatenation, ReLU) on a dense box over the grid nodes, with BF16
// activations and weights and FP32 accumulation on MFMA
// (v_mfma_f32_16x16x32_bf16), FP32 master weights and Adam.
//
// Tensors are channels-last views (ptr, ldc): channel c of voxel v is at
// ptr[v*ldc + c], voxel v = (i*Y + j)*Z + k.  Skip concatenation is a
// layout choice: the encoder writes its output into the upper channel half
// of the decoder's input tensor and the up-sampling layer into the lower
// half, so no copy is made.
//
// GEMM orientation (all convolutions): D[m = out channel][n = voxel] +=
// A[m][k] B[k][n] with k enumerating (tap, in channel), in channel fastest.
// A is the weight, pre-swizzled so that every lane loads its 8 bf16 with one
// 16-byte load; B is 8 consecutive channels of one voxel (16 bytes); each
// lane of D holds 4 consecutive output channels of one voxel.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "mpl_grid.h"
#include "mpl_nn.h"

using namespace mpl;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

struct Dims3 {
  int x, y, z;
};

// ---------------------------------------------------------------- gather conv
// y[v, o] = act(b[o] + sum_{t, i} x[s v + t - p, i] W[t, i, o]) (+ y if accum)
// One wavefront computes VT tiles of 16 consecutive output voxels x all CT*16
// output channels.  Wsw: [kstep][CT][64 lanes][8] bf16.
template <int CT, int VT>
__global__ __launch_bounds__(256) void k_conv(const uint16_t* __restrict__ x, int ldx, Dims3 din,
                                              const uint16_t* __restrict__ Wsw, int nk, int Ci,
                                              int ktaps, int ks, int stride, int pad,
                                              const float* __restrict__ bias,
                                              uint16_t* __restrict__ y, int ldy, Dims3 dout,
                                              int relu, int accum, const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t nvox = (int64_t)dout.x * dout.y * dout.z;
  const int64_t vbase = ((int64_t)blockIdx.x * 4 + wave) * (VT * 16);
  if (vbase >= nvox) return;
  int vi[VT][3];
  bool vok[VT];
#pragma unroll
  for (int t = 0; t < VT; ++t) {
    const int64_t v = vbase + t * 16 + (lane & 15);
    vok[t] = v < nvox;
    const int64_t vv = vok[t] ? v : 0;
    vi[t][2] = (int)(vv % dout.z);
    vi[t][1] = (int)((vv / dout.z) % dout.y);
    vi[t][0] = (int)(vv / ((int64_t)dout.z * dout.y));
  }
  f32x4 acc[VT][CT];
#pragma unroll
  for (int t = 0; t < VT; ++t)
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[t][c] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int ksub = (lane >> 4) * 8;
  for (int kstep = 0; kstep < nk; ++kstep) {
    const int kk = kstep * 32 + ksub;
    const int tap = kk / Ci, c0 = kk - tap * Ci;
    const int tx = tap / (ks * ks), ty = (tap / ks) % ks, tz = tap % ks;
    bf16x8 bop[VT];
#pragma unroll
    for (int t = 0; t < VT; ++t) {
      const int ix = vi[t][0] * stride + tx - pad, iy = vi[t][1] * stride + ty - pad,
                iz = vi[t][2] * stride + tz - pad;
      uint4 raw = make_uint4(0, 0, 0, 0);
      if (tap < ktaps && vok[t] && ix >= 0 && iy >= 0 && iz >= 0 && ix < din.x && iy < din.y &&
          iz < din.z) {
        const int64_t src = (((int64_t)ix * din.y + iy) * din.z + iz) * ldx + c0;
        raw = *reinterpret_cast<const uint4*>(x + src);
      }
      bop[t] = __builtin_bit_cast(bf16x8, raw);
    }
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      const uint4 wr = *reinterpret_cast<const uint4*>(Wsw + (((int64_t)kstep * CT + c) * 64 + lane) * 8);
      const bf16x8 aop = __builtin_bit_cast(bf16x8, wr);
#pragma unroll
      for (int t = 0; t < VT; ++t)
        acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, bop[t], acc[t][c], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < VT; ++t) {
    if (!vok[t]) continue;
    const int64_t v = vbase + t * 16 + (lane & 15);
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      const int o0 = c * 16 + (lane >> 4) * 4;
      uint16_t* dst = y + v * ldy + o0;
      float r[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        float val = acc[t][c][e] + (bias ? bias[o0 + e] : 0.f);
        if (accum) val += bf2f(dst[e]);
        if (relu) val = fmaxf(val, 0.f);
        r[e] = val;
      }
      const uint2 packed = make_uint2((uint32_t)f2bf(r[0]) | ((uint32_t)f2bf(r[1]) << 16),
                                      (uint32_t)f2bf(r[2]) | ((uint32_t)f2bf(r[3]) << 16));
      *reinterpret_cast<uint2*>(dst) = packed;
    }
  }
}

// ---------------------------------------------------------------- LDS-tiled 3x3x3 conv
// 3x3x3 stride-1 pad-1 convolution (forward, and the data gradient with the
// flipped-tap weights).  An output tile is 4 (x) x 4 (y) x 16 (z) voxels for
// CT*16 of the output channels (blockIdx.y selects which); wavefront w owns
// x = x0 + w and the four 16-voxel z-strips y0..y0+3.  The input tile with
// its one-voxel halo (6 x 6 x 18 voxels) is staged in LDS 16 channels at a
// time, so every input value is read from memory once per workgroup and
// chunk instead of once per tap; an MFMA K step covers two taps x the 16
// channels of the chunk (14 steps per chunk, the last one half empty), and
// each B operand read from LDS feeds the CT output-channel tiles.  The
// workgroups stride over the (tile, chunk) items, and the global loads of the
// next item are issued before the MFMAs of the current one.  On small grids
// the input-channel chunks are split over blockIdx.z: split z sums chunks
// [z nchunk / nsplit, (z + 1) nchunk / nsplit) and stores its FP32 partial
// sums to part[z][voxel][channel]; k_conv3_split_reduce then adds the splits
// in order and applies bias, accumulation and ReLU.
// Wsw: [chunk][kstep 0..13][CT][64 lanes][8] (swizzle modes 3 and 4).
namespace lds3 {
constexpr int HX = 6, HY = 6, HZ = 18, NV = HX * HY * HZ;
constexpr int PER = (NV * 2 + 255) / 256;
}  // namespace lds3

template <int CT>
__global__ __launch_bounds__(256) void k_conv3_lds(const uint16_t* __restrict__ x, int ldx, Dims3 d,
                                                   int Ci, const uint16_t* __restrict__ Wsw, int CTT,
                                                   const float* __restrict__ bias,
                                                   uint16_t* __restrict__ y, int ldy, int relu,
                                                   int accum, const int32_t* __restrict__ skip,
                                                   float* __restrict__ part) {
  // blockIdx.y selects output channels [16 CT y, 16 CT (y + 1)) of the CTT*16
  using namespace lds3;
  if (skip && *skip) return;
  __shared__ uint4 tile[2 * NV];  // [channel half][voxel]
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nbx = (d.x + 3) >> 2, nby = (d.y + 3) >> 2, nbz = (d.z + 15) >> 4;
  const int ntiles = nbx * nby * nbz;
  const int j = lane & 15, g = lane >> 4;
  const int nchunk_all = Ci >> 4, nsplit = (int)gridDim.z, zs = (int)blockIdx.z;
  const int qbeg = zs * nchunk_all / nsplit, qend = (zs + 1) * nchunk_all / nsplit;
  const int ct0 = blockIdx.y * CT;
  uint4 pre[PER];
  auto fetch = [&](int t, int q) {
    const int bz = t / (nbx * nby), rem = t - bz * nbx * nby;
    const int by = rem / nbx, bx = rem - by * nbx;
    const int x0 = bx * 4, y0 = by * 4, z0 = bz * 16;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int idx = threadIdx.x + 256 * k;
      const int h = idx & 1, vv = idx >> 1;
      const int hz = vv % HZ, hy = (vv / HZ) % HY, hx = vv / (HZ * HY);
      const int gx = x0 - 1 + hx, gy = y0 - 1 + hy, gz = z0 - 1 + hz;
      pre[k] = make_uint4(0, 0, 0, 0);
      if (idx < NV * 2 && gx >= 0 && gy >= 0 && gz >= 0 && gx < d.x && gy < d.y && gz < d.z)
        pre[k] = *reinterpret_cast<const uint4*>(x + (((int64_t)gx * d.y + gy) * d.z + gz) * ldx + q * 16 + h * 8);
    }
  };
  f32x4 acc[4][CT];
#pragma unroll
  for (int st = 0; st < 4; ++st)
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[st][c] = f32x4{0.f, 0.f, 0.f, 0.f};
  int t = blockIdx.x, q = qbeg;
  if (t >= ntiles || qbeg >= qend) return;
  fetch(t, qbeg);
  while (true) {
    __syncthreads();  // every wavefront is done reading the previous item's tile
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int idx = threadIdx.x + 256 * k;
      if (idx < NV * 2) tile[(idx & 1) * NV + (idx >> 1)] = pre[k];
    }
    __syncthreads();
    int tn = t, qn = q + 1;
    if (qn == qend) {
      qn = qbeg;
      tn = t + (int)gridDim.x;
    }
    if (tn < ntiles) fetch(tn, qn);
    const uint16_t* Wq = Wsw + (int64_t)q * 14 * CTT * 512;
    for (int m = 0; m < 14; ++m) {
      const int tap = 2 * m + (g >> 1);
      bf16x8 aop[CT];
#pragma unroll
      for (int c = 0; c < CT; ++c)
        aop[c] = __builtin_bit_cast(
            bf16x8, *reinterpret_cast<const uint4*>(Wq + ((m * CTT + ct0 + c) * 64 + lane) * 8));
      const bool tv = tap < 27;
      const int tx = tv ? tap / 9 : 0, ty = tv ? (tap / 3) % 3 : 0, tz = tv ? tap % 3 : 0;
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int hv = ((w + tx) * HY + (st + ty)) * HZ + (j + tz);
        const uint4 raw = tv ? tile[(g & 1) * NV + hv] : make_uint4(0, 0, 0, 0);
        const bf16x8 bop = __builtin_bit_cast(bf16x8, raw);
#pragma unroll
        for (int c = 0; c < CT; ++c)
          acc[st][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop[c], bop, acc[st][c], 0, 0, 0);
      }
    }
    if (q == qend - 1) {
      const int bz = t / (nbx * nby), rem = t - bz * nbx * nby;
      const int by = rem / nbx, bx = rem - by * nbx;
      const int ox = bx * 4 + w, oz = bz * 16 + j;
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int oy = by * 4 + st;
        const bool ok = ox < d.x && oy < d.y && oz < d.z;
        const int64_t v = ((int64_t)ox * d.y + oy) * d.z + oz;
#pragma unroll
        for (int c = 0; c < CT; ++c) {
          if (ok && part) {
            const int o0 = (ct0 + c) * 16 + g * 4;
            const int64_t nv = (int64_t)d.x * d.y * d.z;
            *reinterpret_cast<float4*>(part + ((int64_t)zs * nv + v) * (16 * CTT) + o0) =
                make_float4(acc[st][c][0], acc[st][c][1], acc[st][c][2], acc[st][c][3]);
          } else if (ok) {
            const int o0 = (ct0 + c) * 16 + g * 4;
            uint16_t* dst = y + v * ldy + o0;
            float r[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              float val = acc[st][c][e] + (bias ? bias[o0 + e] : 0.f);
              if (accum) val += bf2f(dst[e]);
              if (relu) val = fmaxf(val, 0.f);
              r[e] = val;
            }
            const uint2 packed = make_uint2((uint32_t)f2bf(r[0]) | ((uint32_t)f2bf(r[1]) << 16),
                                            (uint32_t)f2bf(r[2]) | ((uint32_t)f2bf(r[3]) << 16));
            *reinterpret_cast<uint2*>(dst) = packed;
          }
          acc[st][c] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
      }
    }
    if (tn >= ntiles) break;
    t = tn;
    q = qn;
  }
}

// Sum of the nsplit FP32 partials of a split 3x3x3 layer in split order, then
// bias, accumulation onto y and ReLU; 4 channels per thread.
__global__ __launch_bounds__(256) void k_conv3_split_reduce(const float* __restrict__ part, int nsplit,
                                                            int64_t nv, int co,
                                                            const float* __restrict__ bias,
                                                            uint16_t* __restrict__ y, int ldy, int relu,
                                                            int accum, const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = co >> 2;
  if (i >= nv * q) return;
  const int64_t v = i / q;
  const int o0 = (int)(i - v * q) * 4;
  float4 s = *reinterpret_cast<const float4*>(part + v * co + o0);
  for (int z = 1; z < nsplit; ++z) {
    const float4 a = *reinterpret_cast<const float4*>(part + ((int64_t)z * nv + v) * co + o0);
    s.x += a.x;
    s.y += a.y;
    s.z += a.z;
    s.w += a.w;
  }
  uint16_t* dst = y + v * ldy + o0;
  float r[4] = {s.x, s.y, s.z, s.w};
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    float val = r[e] + (bias ? bias[o0 + e] : 0.f);
    if (accum) val += bf2f(dst[e]);
    if (relu) val = fmaxf(val, 0.f);
    r[e] = val;
  }
  *reinterpret_cast<uint2*>(dst) = make_uint2((uint32_t)f2bf(r[0]) | ((uint32_t)f2bf(r[1]) << 16),
                                              (uint32_t)f2bf(r[2]) | ((uint32_t)f2bf(r[3]) << 16));
}

// ---------------------------------------------------------------- register-blocked 3x3x3 conv
// 3x3x3 stride-1 pad-1 convolution with 16 output channels (the finest level
// of the network, forward, and the data gradient of its 16-channel layers).
// With one output-channel tile k_conv3_lds feeds one MFMA per LDS read; here
// a B operand is reused across the output rows it reaches.  An output tile
// is 8 (x) x 4 (y) x 16 (z) voxels; wavefront w of the workgroup owns
// x = x0 + 2w, x0 + 2w + 1 and y = y0 .. y0 + 3, eight 16-voxel z strips.
// The input tile with its one-voxel halo (10 x 6 x 18 voxels, 16 channels)
// is staged in LDS per 16-channel chunk.  One MFMA K step covers the z taps
// 0 and 1 x 16 channels (step 0) or the z tap 2 x 16 channels with 16 zero
// channels (step 1), so a B operand is one input row (x, y) at two z shifts,
// and it serves every strip (x - tx, y - ty) of the wavefront: up to six
// MFMAs per LDS read.  The weights of all nine (tx, ty) pairs and both steps
// stay in registers for the chunk (for the whole launch when Ci = 16).
// The workgroups stride over the (tile, chunk) items, and the global loads
// of the next item are issued before the MFMAs of the current one, so their
// latency hides behind the arithmetic instead of stalling the workgroup.
// Wrr: [chunk][tx*3 + ty][step][64 lanes][8] bf16 (swizzle modes 3 and 4).
namespace rr {
constexpr int HX = 10, HY = 6, HZ = 18, NV = HX * HY * HZ;
constexpr int PER = (NV * 2 + 255) / 256;  // staged 16-byte pieces per thread
}  // namespace rr

__global__ __launch_bounds__(256) void k_conv3_rr(const uint16_t* __restrict__ x, int ldx, Dims3 d,
                                                  int Ci, const uint16_t* __restrict__ Wrr,
                                                  const float* __restrict__ bias,
                                                  uint16_t* __restrict__ y, int ldy, int relu,
                                                  int accum, const int32_t* __restrict__ skip) {
  using namespace rr;
  if (skip && *skip) return;
  // [channel half][voxel]: the 16 lanes of an MFMA column group read 16
  // consecutive voxels of one half, 256 contiguous bytes
  __shared__ uint4 tile[2 * NV];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nbx = (d.x + 7) >> 3, nby = (d.y + 3) >> 2, nbz = (d.z + 15) >> 4;
  const int ntiles = nbx * nby * nbz;
  const int j = lane & 15, g = lane >> 4;
  const int nchunk = Ci >> 4;
  // this lane's LDS position in its wavefront's rows: x row 2w, z = j, the
  // channel half g & 1; step 0 reads z shift g >> 1, step 1 shift 2 (lanes
  // g >= 2 of step 1 carry the zero channels)
  const int lbase = (g & 1) * NV + (2 * w) * HY * HZ + j;
  const int sh0 = g >> 1;
  const bool has1 = g < 2;
  uint4 pre[PER];
  auto fetch = [&](int t, int q) {
    const int bz = t / (nbx * nby), rem = t - bz * nbx * nby;
    const int by = rem / nbx, bx = rem - by * nbx;
    const int x0 = bx * 8, y0 = by * 4, z0 = bz * 16;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int idx = threadIdx.x + 256 * k;
      const int h = idx & 1, vv = idx >> 1;
      const int hz = vv % HZ, hy = (vv / HZ) % HY, hx = vv / (HZ * HY);
      const int gx = x0 - 1 + hx, gy = y0 - 1 + hy, gz = z0 - 1 + hz;
      pre[k] = make_uint4(0, 0, 0, 0);
      if (idx < NV * 2 && gx >= 0 && gy >= 0 && gz >= 0 && gx < d.x && gy < d.y && gz < d.z)
        pre[k] = *reinterpret_cast<const uint4*>(x + (((int64_t)gx * d.y + gy) * d.z + gz) * ldx + q * 16 + h * 8);
    }
  };
  f32x4 acc[2][4];
#pragma unroll
  for (int sx = 0; sx < 2; ++sx)
#pragma unroll
    for (int sy = 0; sy < 4; ++sy) acc[sx][sy] = f32x4{0.f, 0.f, 0.f, 0.f};
  // the weights of the chunk (loaded once when there is only one)
  bf16x8 A[9][2];
  auto loadA = [&](int q) {
    const uint16_t* Wq = Wrr + (int64_t)q * 18 * 512;
#pragma unroll
    for (int tt = 0; tt < 9; ++tt)
#pragma unroll
      for (int st = 0; st < 2; ++st)
        A[tt][st] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(Wq + ((tt * 2 + st) * 64 + lane) * 8));
  };
  int t = blockIdx.x, q = 0;
  if (t >= ntiles) return;
  fetch(t, 0);
  if (nchunk == 1) loadA(0);
  while (true) {
    __syncthreads();  // every wavefront is done reading the previous item's tile
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int idx = threadIdx.x + 256 * k;
      if (idx < NV * 2) tile[(idx & 1) * NV + (idx >> 1)] = pre[k];
    }
    if (nchunk > 1) loadA(q);
    __syncthreads();
    int tn = t, qn = q + 1;
    if (qn == nchunk) {
      qn = 0;
      tn = t + (int)gridDim.x;
    }
    if (tn < ntiles) fetch(tn, qn);
#pragma unroll
    for (int hx = 0; hx < 4; ++hx)
#pragma unroll
      for (int hy = 0; hy < HY; ++hy) {
        const int row = lbase + (hx * HY + hy) * HZ;
        const bf16x8 bs[2] = {__builtin_bit_cast(bf16x8, tile[row + sh0]),
                              __builtin_bit_cast(bf16x8, has1 ? tile[row + 2] : make_uint4(0, 0, 0, 0))};
        // the two steps in separate passes, so that consecutive MFMAs update
        // different accumulators
#pragma unroll
        for (int st = 0; st < 2; ++st)
#pragma unroll
          for (int tx = 0; tx < 3; ++tx)
#pragma unroll
            for (int ty = 0; ty < 3; ++ty) {
              const int sx = hx - tx, sy = hy - ty;
              if (sx < 0 || sx > 1 || sy < 0 || sy > 3) continue;
              acc[sx][sy] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[tx * 3 + ty][st], bs[st], acc[sx][sy], 0, 0, 0);
            }
      }
    if (q == nchunk - 1) {
      const int bz = t / (nbx * nby), rem = t - bz * nbx * nby;
      const int by = rem / nbx, bx = rem - by * nbx;
      const int x0 = bx * 8, y0 = by * 4, oz = bz * 16 + j;
#pragma unroll
      for (int sx = 0; sx < 2; ++sx)
#pragma unroll
        for (int sy = 0; sy < 4; ++sy) {
          const int ox = x0 + 2 * w + sx, oy = y0 + sy;
          if (ox < d.x && oy < d.y && oz < d.z) {
            const int64_t v = ((int64_t)ox * d.y + oy) * d.z + oz;
            const int o0 = g * 4;
            uint16_t* dst = y + v * ldy + o0;
            float r[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              float val = acc[sx][sy][e] + (bias ? bias[o0 + e] : 0.f);
              if (accum) val += bf2f(dst[e]);
              if (relu) val = fmaxf(val, 0.f);
              r[e] = val;
            }
            const uint2 packed = make_uint2((uint32_t)f2bf(r[0]) | ((uint32_t)f2bf(r[1]) << 16),
                                            (uint32_t)f2bf(r[2]) | ((uint32_t)f2bf(r[3]) << 16));
            *reinterpret_cast<uint2*>(dst) = packed;
          }
          acc[sx][sy] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
    }
    if (tn >= ntiles) break;
    t = tn;
    q = qn;
  }
}

// Weights of k_conv3_rr: out[((q*9 + tx*3 + ty)*2 + st)*64 + lane][e], output
// channel lane & 15, group gg = lane >> 4; step 0: z tap gg >> 1, step 1: z
// tap 2 for gg < 2 and zero for gg >= 2; input channel 16q + (gg & 1)*8 + e;
//   mode 3 (forward): W[tap][in][out];  mode 4 (data gradient): W[26 - tap][out][in],
// tap = (tx*3 + ty)*3 + tz.
__global__ void k_swizzle3rr(const float* __restrict__ W, int Ci, int Co, int mode, int nchunk,
                             uint16_t* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)nchunk * 18 * 512;
  if (idx >= total) return;
  int64_t r = idx;
  const int e = (int)(r % 8);
  r /= 8;
  const int lane = (int)(r % 64);
  r /= 64;
  const int st = (int)(r % 2);
  r /= 2;
  const int txy = (int)(r % 9);
  const int q = (int)(r / 9);
  const int gg = lane >> 4;
  const int tz = st == 0 ? (gg >> 1) : (gg < 2 ? 2 : -1);
  const int cin = 16 * q + (gg & 1) * 8 + e, cout = lane & 15;
  float val = 0.f;
  if (tz >= 0) {
    const int tap = txy * 3 + tz;
    if (mode == 3) val = W[((int64_t)tap * Ci + cin) * Co + cout];
    else val = W[((int64_t)(26 - tap) * Ci + cout) * Co + cin];
  }
  out[idx] = f2bf(val);
}

// Weights of k_conv3_lds: out[((q*14 + m)*CT + ct)*64 + lane][e] with
// tap = 2m + (lane>>4 >> 1), input channel 16q + ((lane>>4) & 1)*8 + e and
// output channel 16ct + (lane & 15);
//   mode 3 (forward): W[tap][in][out];  mode 4 (data gradient): the input is
//   the forward output: W[26 - tap][out][in].
__global__ void k_swizzle3(const float* __restrict__ W, int Ci, int Co, int mode, int CT, int nchunk,
                           uint16_t* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)nchunk * 14 * CT * 512;
  if (idx >= total) return;
  int64_t r = idx;
  const int e = (int)(r % 8);
  r /= 8;
  const int lane = (int)(r % 64);
  r /= 64;
  const int ct = (int)(r % CT);
  r /= CT;
  const int m = (int)(r % 14);
  const int q = (int)(r / 14);
  const int gg = lane >> 4;
  const int tap = 2 * m + (gg >> 1);
  const int cin = 16 * q + (gg & 1) * 8 + e, cout = 16 * ct + (lane & 15);
  float val = 0.f;
  if (tap < 27) {
    if (mode == 3) val = W[((int64_t)tap * Ci + cin) * Co + cout];
    else val = W[((int64_t)(26 - tap) * Ci + cout) * Co + cin];
  }
  out[idx] = f2bf(val);
}

// ---------------------------------------------------------------- up conv
// y[2 v + t, o] = act(b[o] + sum_i x[v, i] W[t, i, o]) (+ y if accum); the
// tap t is blockIdx.y so that all 16 voxels of an MFMA share the weight.
// Wsw: [t][kstep][CT][64][8].
template <int CT, int VT>
__global__ __launch_bounds__(256) void k_up(const uint16_t* __restrict__ x, int ldx, Dims3 din,
                                            const uint16_t* __restrict__ Wsw, int nk,
                                            const float* __restrict__ bias,
                                            uint16_t* __restrict__ y, int ldy, int relu,
                                            int accum, const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tap = blockIdx.y;
  const int tx = tap >> 2, ty = (tap >> 1) & 1, tz = tap & 1;
  const int64_t nvox = (int64_t)din.x * din.y * din.z;
  const int64_t vbase = ((int64_t)blockIdx.x * 4 + wave) * (VT * 16);
  if (vbase >= nvox) return;
  f32x4 acc[VT][CT];
#pragma unroll
  for (int t = 0; t < VT; ++t)
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[t][c] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int ksub = (lane >> 4) * 8;
  for (int kstep = 0; kstep < nk; ++kstep) {
    bf16x8 bop[VT];
#pragma unroll
    for (int t = 0; t < VT; ++t) {
      const int64_t v = vbase + t * 16 + (lane & 15);
      uint4 raw = make_uint4(0, 0, 0, 0);
      if (v < nvox) raw = *reinterpret_cast<const uint4*>(x + v * ldx + kstep * 32 + ksub);
      bop[t] = __builtin_bit_cast(bf16x8, raw);
    }
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      const uint4 wr = *reinterpret_cast<const uint4*>(
          Wsw + ((((int64_t)tap * nk + kstep) * CT + c) * 64 + lane) * 8);
      const bf16x8 aop = __builtin_bit_cast(bf16x8, wr);
#pragma unroll
      for (int t = 0; t < VT; ++t)
        acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, bop[t], acc[t][c], 0, 0, 0);
    }
  }
  const Dims3 dout{2 * din.x, 2 * din.y, 2 * din.z};
#pragma unroll
  for (int t = 0; t < VT; ++t) {
    const int64_t v = vbase + t * 16 + (lane & 15);
    if (v >= nvox) continue;
    const int k = (int)(v % din.z), j = (int)((v / din.z) % din.y), i = (int)(v / ((int64_t)din.z * din.y));
    const int64_t u = (((int64_t)(2 * i + tx) * dout.y + (2 * j + ty)) * dout.z + (2 * k + tz));
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      const int o0 = c * 16 + (lane >> 4) * 4;
      uint16_t* dst = y + u * ldy + o0;
      float r[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        float val = acc[t][c][e] + (bias ? bias[o0 + e] : 0.f);
        if (accum) val += bf2f(dst[e]);
        if (relu) val = fmaxf(val, 0.f);
        r[e] = val;
      }
      const uint2 packed = make_uint2((uint32_t)f2bf(r[0]) | ((uint32_t)f2bf(r[1]) << 16),
                                      (uint32_t)f2bf(r[2]) | ((uint32_t)f2bf(r[3]) << 16));
      *reinterpret_cast<uint2*>(dst) = packed;
    }
  }
}

// ---------------------------------------------------------------- wgrad
// Partial weight gradient of one (tap, in-channel tile, out-channel tile)
// over a chunk of output voxels:
//   gather conv: dW[t, i, o] += sum_u x[s u + t - p, i] dy[u, o]
//   up conv:     dW[t, i, o] += sum_v x[v, i] dy[2 v + t, o]
// D[m = i][n = o] with the voxel sum as the MFMA K dimension.
__global__ __launch_bounds__(64) void k_wgrad(const uint16_t* __restrict__ x, int ldx, Dims3 din,
                                              const uint16_t* __restrict__ dy, int ldy,
                                              Dims3 dout, int Ci, int Co, int ks, int stride,
                                              int pad, int is_up, int chunk,
                                              float* __restrict__ part) {
  const int lane = threadIdx.x;
  const int CiT = Ci / 16, CoT = Co / 16;
  const int job = blockIdx.y;
  const int ot = job % CoT, it = (job / CoT) % CiT, tap = job / (CoT * CiT);
  const int tx = tap / (ks * ks), ty = (tap / ks) % ks, tz = tap % ks;
  // the voxels summed over: output voxels u (gather) or input voxels v (up)
  const Dims3 vd = is_up ? din : dout;
  const int64_t nv = (int64_t)vd.x * vd.y * vd.z;
  const int64_t v0 = (int64_t)blockIdx.x * chunk;
  const int64_t v1 = (v0 + chunk < nv) ? v0 + chunk : nv;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  const int ci = it * 16 + (lane & 15), co = ot * 16 + (lane & 15);
  for (int64_t vb = v0; vb < v1; vb += 32) {
    bf16x8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t v = vb + (lane >> 4) * 8 + e;
      float xa = 0.f, gb = 0.f;
      if (v < v1) {
        const int k = (int)(v % vd.z), j = (int)((v / vd.z) % vd.y), i = (int)(v / ((int64_t)vd.z * vd.y));
        if (is_up) {
          xa = bf2f(x[v * ldx + ci]);
          const int64_t u = (((int64_t)(2 * i + tx) * dout.y + (2 * j + ty)) * dout.z + (2 * k + tz));
          gb = bf2f(dy[u * ldy + co]);
        } else {
          const int ix = i * stride + tx - pad, iy = j * stride + ty - pad, iz = k * stride + tz - pad;
          if (ix >= 0 && iy >= 0 && iz >= 0 && ix < din.x && iy < din.y && iz < din.z)
            xa = bf2f(x[(((int64_t)ix * din.y + iy) * din.z + iz) * ldx + ci]);
          gb = bf2f(dy[v * ldy + co]);
        }
      }
      a[e] = (__bf16)xa;
      b[e] = (__bf16)gb;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
  }
  // lane holds D[i = (lane>>4)*4 + e][o = lane & 15]
  float* dst = part + ((int64_t)blockIdx.x * gridDim.y + job) * 256;
#pragma unroll
  for (int e = 0; e < 4; ++e) dst[((lane >> 4) * 4 + e) * 16 + (lane & 15)] = acc[e];
}

// dW[t][i][o] (flat, added to grad) = sum over chunks of the partial tiles.
__global__ void k_wgrad_reduce(const float* __restrict__ part, int nchunks, int njobs, int Ci,
                               int Co, float* __restrict__ gW) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)njobs * 256;
  if (idx >= total) return;
  const int job = (int)(idx / 256), e = (int)(idx % 256);
  const int CiT = Ci / 16, CoT = Co / 16;
  const int ot = job % CoT, it = (job / CoT) % CiT, tap = job / (CoT * CiT);
  const int i = it * 16 + e / 16, o = ot * 16 + e % 16;
  float s = 0.f;
  for (int c = 0; c < nchunks; ++c) s += part[((int64_t)c * njobs + job) * 256 + e];
  gW[((int64_t)tap * Ci + i) * Co + o] += s;
}

// db[o] += sum_u dy[u, o] (one workgroup per output channel, fixed order).
// Bias gradient sum_v dy[v, o] in two passes: per chunk of voxels one
// partial per channel (threads of a workgroup read consecutive channels of
// the same voxels), then a fixed-order sum over the chunks.
__global__ __launch_bounds__(256) void k_bias_partial(const uint16_t* __restrict__ dy, int ldy,
                                                      int64_t nvox, int co, int64_t chunk,
                                                      float* __restrict__ part) {
  __shared__ float sh[256];
  const int t = threadIdx.x, c = t % co, v0 = t / co, step = 256 / co;
  const int64_t beg = (int64_t)blockIdx.x * chunk, end = beg + chunk < nvox ? beg + chunk : nvox;
  float s = 0.f;
  for (int64_t v = beg + v0; v < end; v += step) s += bf2f(dy[v * ldy + c]);
  sh[t] = s;
  __syncthreads();
  if (t < co) {
    float acc = 0.f;
    for (int k = 0; k < step; ++k) acc += sh[t + k * co];
    part[(int64_t)blockIdx.x * co + t] = acc;
  }
}
__global__ void k_bias_reduce(const float* __restrict__ part, int nch, int co, float* __restrict__ gb) {
  const int c = threadIdx.x;
  if (c >= co) return;
  float acc = 0.f;
  for (int k = 0; k < nch; ++k) acc += part[(int64_t)k * co + c];
  gb[c] += acc;
}

// g <- g * (y > 0) over C channels of strided views.
__global__ void k_relu_bwd(uint16_t* __restrict__ g, int ldg, const uint16_t* __restrict__ y, int ldy,
                           int C, int64_t nvox) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nvox * C) return;
  const int64_t v = idx / C;
  const int c = (int)(idx % C);
  if (!(bf2f(y[v * ldy + c]) > 0.f)) g[v * ldg + c] = 0;
}

// Swizzle FP32 weights into the MFMA A-operand layout.
//   mode 0 (forward):      A[m = o][k = (t, i)] = W[t][i][o]
//   mode 1 (conv dgrad):   A[m = i][k = (t', o)] = W[T-1-t'][i][o]   (flipped taps)
//   mode 2 (transposed):   A[m = i][k = (t, o)]  = W[t][i][o]
// per_tap: the K dimension restarts at every tap (up-type layers).
__global__ void k_swizzle(const float* __restrict__ W, int T, int Ci, int Co, int mode, int per_tap,
                          int nk, int CT, uint16_t* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)nk * CT * 64 * 8;
  const int64_t total = per * (per_tap ? T : 1);
  if (idx >= total) return;
  const int tap_blk = per_tap ? (int)(idx / per) : 0;
  int64_t r = idx % per;
  const int e = (int)(r % 8);
  r /= 8;
  const int lane = (int)(r % 64);
  r /= 64;
  const int ct = (int)(r % CT);
  const int kstep = (int)(r / CT);
  const int m = ct * 16 + (lane & 15);
  const int k = kstep * 32 + (lane >> 4) * 8 + e;
  const int Kin = (mode == 0) ? Ci : Co;  // channels along K
  const int M = (mode == 0) ? Co : Ci;
  float val = 0.f;
  const int tap = per_tap ? tap_blk : k / Kin;
  const int kc = per_tap ? k : k % Kin;
  if (m < M && tap < T && kc < Kin) {
    if (mode == 0) val = W[((int64_t)tap * Ci + kc) * Co + m];
    else if (mode == 1) val = W[((int64_t)(T - 1 - tap) * Ci + m) * Co + kc];
    else val = W[((int64_t)tap * Ci + m) * Co + kc];
  }
  out[idx] = f2bf(val);
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  if (!isfinite(gi)) return;
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_f32_to_bf16(const float* __restrict__ a, uint16_t* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = f2bf(a[i]);
}
__global__ void k_bf16_to_f32(const uint16_t* __restrict__ a, float* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = bf2f(a[i]);
}

// Masked relative L2 loss on channels 0..2 and its gradient w.r.t. y:
//   L = |m (y - t)|^2 / |m t|^2,   dL/dy = 2 m^2 (y - t) / |m t|^2.
// Pass 1: partial sums of numerator and denominator per workgroup.
__global__ __launch_bounds__(256) void k_loss_partial(const uint16_t* __restrict__ y, int ldy,
                                                      const float* __restrict__ t,
                                                      const float* __restrict__ mask, int64_t nvox,
                                                      double* __restrict__ part) {
  __shared__ double sn[256], sd[256];
  double num = 0.0, den = 0.0;
  for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < nvox; v += (int64_t)gridDim.x * 256) {
    const float mv = mask[v];
    for (int c = 0; c < 3; ++c) {
      const double d = (double)(bf2f(y[v * ldy + c]) - t[v * 3 + c]) * mv;
      const double tt = (double)t[v * 3 + c] * mv;
      num += d * d;
      den += tt * tt;
    }
  }
  sn[threadIdx.x] = num;
  sd[threadIdx.x] = den;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      sn[threadIdx.x] += sn[threadIdx.x + off];
      sd[threadIdx.x] += sd[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sn[0];
    part[2 * blockIdx.x + 1] = sd[0];
  }
}
__global__ void k_loss_final(const double* __restrict__ part, int n, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double a = 0.0, b = 0.0;
  for (int i = 0; i < n; ++i) {
    a += part[2 * i];
    b += part[2 * i + 1];
  }
  out[0] = a;
  out[1] = b;
  out[2] = b > 0.0 ? a / b : 0.0;
}
__global__ void k_loss_grad(const uint16_t* __restrict__ y, int ldy, const float* __restrict__ t,
                            const float* __restrict__ mask, int64_t nvox,
                            const double* __restrict__ sums, uint16_t* __restrict__ g, int ldg) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvox) return;
  const double den = sums[1];
  const float mv = mask[v];
  for (int c = 0; c < ldg; ++c) {
    float val = 0.f;
    if (c < 3 && den > 0.0) val = (float)(2.0 * mv * mv * (bf2f(y[v * ldy + c]) - t[v * 3 + c]) / den);
    g[v * ldg + c] = f2bf(val);
  }
}

}  // namespace

// ======================================================================
// Layer table (shared with the parameter layout documented in mpl_nn.h).
namespace {
struct Spec {
  const char* name;
  int up;       // 1: 2x2x2 stride-2 transposed convolution
  int k, s, p;  // gather conv kernel size, stride, padding
  int ci, co, relu, level_in, level_out;
};
const Spec kSpec[NN_LAYERS] = {
    {"enc0a", 0, 3, 1, 1, 16, 16, 1, 0, 0},   {"enc0b", 0, 3, 1, 1, 16, 16, 1, 0, 0},
    {"down0", 0, 2, 2, 0, 16, 32, 1, 0, 1},   {"enc1a", 0, 3, 1, 1, 32, 32, 1, 1, 1},
    {"enc1b", 0, 3, 1, 1, 32, 32, 1, 1, 1},   {"down1", 0, 2, 2, 0, 32, 64, 1, 1, 2},
    {"enc2a", 0, 3, 1, 1, 64, 64, 1, 2, 2},   {"enc2b", 0, 3, 1, 1, 64, 64, 1, 2, 2},
    {"down2", 0, 2, 2, 0, 64, 128, 1, 2, 3},  {"bota", 0, 3, 1, 1, 128, 128, 1, 3, 3},
    {"botb", 0, 3, 1, 1, 128, 128, 1, 3, 3},  {"up2", 1, 2, 2, 0, 128, 64, 1, 3, 2},
    {"dec2a", 0, 3, 1, 1, 128, 64, 1, 2, 2},  {"dec2b", 0, 3, 1, 1, 64, 64, 1, 2, 2},
    {"up1", 1, 2, 2, 0, 64, 32, 1, 2, 1},     {"dec1a", 0, 3, 1, 1, 64, 32, 1, 1, 1},
    {"dec1b", 0, 3, 1, 1, 32, 32, 1, 1, 1},   {"up0", 1, 2, 2, 0, 32, 16, 1, 1, 0},
    {"dec0a", 0, 3, 1, 1, 32, 16, 1, 0, 0},   {"dec0b", 0, 3, 1, 1, 16, 16, 1, 0, 0},
    {"out", 0, 1, 1, 0, 16, 16, 0, 0, 0}};

int taps_of(const Spec& s) { return s.k * s.k * s.k; }
}  // namespace

int64_t nn_param_count() {
  int64_t n = 0;
  for (int l = 0; l < NN_LAYERS; ++l) n += (int64_t)taps_of(kSpec[l]) * kSpec[l].ci * kSpec[l].co + kSpec[l].co;
  return n;
}

static int64_t w_offset(int layer) {
  int64_t n = 0;
  for (int l = 0; l < layer; ++l) n += (int64_t)taps_of(kSpec[l]) * kSpec[l].ci * kSpec[l].co + kSpec[l].co;
  return n;
}

static mpl_status nn_alloc(mpl_ctx* c, NNState& nn) {
  const int64_t np = nn_param_count();
  MPL_TRY(mpl_ensure(c, nn.params, 4 * np));
  MPL_TRY(mpl_ensure(c, nn.grad, 4 * np));
  MPL_TRY(mpl_ensure(c, nn.adam_m, 4 * np));
  MPL_TRY(mpl_ensure(c, nn.adam_v, 4 * np));
  // swizzled weights: forward and backward copies per layer
  size_t sw = 0;
  for (int l = 0; l < NN_LAYERS; ++l) {
    const Spec& s = kSpec[l];
    const int T = taps_of(s);
    const size_t kf = s.up ? (size_t)T * ((s.ci + 31) / 32) * (s.co / 16) : ((size_t)(T * s.ci + 31) / 32) * (s.co / 16);
    const size_t kb = s.up ? ((size_t)(T * s.co + 31) / 32) * (s.ci / 16) : (size_t)(T + 1) * ((s.co + 31) / 32) * (s.ci / 16);
    nn.sw_fwd_off[l] = sw;
    sw += kf * 64 * 8;
    nn.sw_bwd_off[l] = sw;
    sw += kb * 64 * 8;
    if (s.k == 3 && !s.up) {
      const size_t k3 = (size_t)(s.ci / 16) * 14 * (s.co / 16) * 512;
      nn.sw3_fwd_off[l] = sw;
      sw += k3;
      nn.sw3_bwd_off[l] = sw;
      sw += k3;
      if (s.co == 16) {
        nn.sw3rr_fwd_off[l] = sw;
        sw += (size_t)(s.ci / 16) * 18 * 512;
      }
      if (s.ci == 16) {
        nn.sw3rr_bwd_off[l] = sw;
        sw += (size_t)(s.co / 16) * 18 * 512;
      }
    }
  }
  MPL_TRY(mpl_ensure(c, nn.wsw, 2 * sw + 256));
  return MPL_OK;
}

// Upload FP32 parameters, build the swizzled BF16 copies.
static mpl_status nn_refresh(mpl_ctx* c, NNState& nn) {
  const float* P = (const float*)nn.params.p;
  uint16_t* sw = (uint16_t*)nn.wsw.p;
  for (int l = 0; l < NN_LAYERS; ++l) {
    const Spec& s = kSpec[l];
    const int T = taps_of(s);
    const float* W = P + w_offset(l);
    if (s.up) {
      const int nk = (s.ci + 31) / 32, CT = s.co / 16;
      const int64_t tot = (int64_t)T * nk * CT * 512;
      MPL_LAUNCH(c, k_swizzle, (int)((tot + 255) / 256), 256, W, T, s.ci, s.co, 0, 1, nk, CT,
                 sw + nn.sw_fwd_off[l]);
      // dgrad of an up layer is a 2x2x2 stride-2 gather conv with A[m=i][k=(t,o)]
      const int nkb = (T * s.co + 31) / 32, CTb = s.ci / 16;
      const int64_t totb = (int64_t)nkb * CTb * 512;
      MPL_LAUNCH(c, k_swizzle, (int)((totb + 255) / 256), 256, W, T, s.ci, s.co, 2, 0, nkb, CTb,
                 sw + nn.sw_bwd_off[l]);
    } else {
      const int nk = (T * s.ci + 31) / 32, CT = s.co / 16;
      const int64_t tot = (int64_t)nk * CT * 512;
      MPL_LAUNCH(c, k_swizzle, (int)((tot + 255) / 256), 256, W, T, s.ci, s.co, 0, 0, nk, CT,
                 sw + nn.sw_fwd_off[l]);
      if (s.k == 3) {
        const int64_t n3 = (int64_t)(s.ci / 16) * 14 * (s.co / 16) * 512;
        MPL_LAUNCH(c, k_swizzle3, (int)((n3 + 255) / 256), 256, W, s.ci, s.co, 3, s.co / 16, s.ci / 16,
                   sw + nn.sw3_fwd_off[l]);
        MPL_LAUNCH(c, k_swizzle3, (int)((n3 + 255) / 256), 256, W, s.ci, s.co, 4, s.ci / 16, s.co / 16,
                   sw + nn.sw3_bwd_off[l]);
        if (s.co == 16) {
          const int64_t nr = (int64_t)(s.ci / 16) * 18 * 512;
          MPL_LAUNCH(c, k_swizzle3rr, (int)((nr + 255) / 256), 256, W, s.ci, s.co, 3, s.ci / 16,
                     sw + nn.sw3rr_fwd_off[l]);
        }
        if (s.ci == 16) {
          const int64_t nr = (int64_t)(s.co / 16) * 18 * 512;
          MPL_LAUNCH(c, k_swizzle3rr, (int)((nr + 255) / 256), 256, W, s.ci, s.co, 4, s.co / 16,
                     sw + nn.sw3rr_bwd_off[l]);
        }
      }
      if (s.k == 2) {
        // dgrad of a stride-2 down conv is an up-type layer with A[m=i][k=(t,o)], K per tap
        const int nkb = (s.co + 31) / 32, CTb = s.ci / 16;
        const int64_t totb = (int64_t)T * nkb * CTb * 512;
        MPL_LAUNCH(c, k_swizzle, (int)((totb + 255) / 256), 256, W, T, s.ci, s.co, 2, 1, nkb, CTb,
                   sw + nn.sw_bwd_off[l]);
      } else {
        const int nkb = (T * s.co + 31) / 32, CTb = s.ci / 16;
        const int64_t totb = (int64_t)nkb * CTb * 512;
        MPL_LAUNCH(c, k_swizzle, (int)((totb + 255) / 256), 256, W, T, s.ci, s.co, 1, 0, nkb, CTb,
                   sw + nn.sw_bwd_off[l]);
      }
    }
  }
  nn.ready = true;
  return MPL_OK;
}

// Activation buffers for a box of dims (multiples of 8).
static mpl_status nn_buffers(mpl_ctx* c, NNState& nn, const int* dims, bool train) {
  for (int a = 0; a < 3; ++a)
    if (dims[a] <= 0 || dims[a] % 8 != 0) return mpl_fail(c, MPL_ERR_INVALID_ARG, "network box dims must be multiples of 8");
  for (int a = 0; a < 3; ++a) nn.box[a] = dims[a];
  int64_t V[4];
  for (int L = 0; L < 4; ++L) V[L] = (int64_t)(dims[0] >> L) * (dims[1] >> L) * (dims[2] >> L);
  // one tensor per layer output, except the skip outputs (upper half of the
  // level's concatenation tensor) and the up-sampling outputs (lower half)
  const int C[4] = {16, 32, 64, 128};
  size_t off = 0;
  auto place = [&](size_t& o, int64_t n) {
    o = off;
    off += (size_t)((n + 63) / 64) * 64;
  };
  place(nn.t_in, V[0] * 16);
  for (int L = 0; L < 3; ++L) place(nn.t_cat[L], V[L] * 2 * C[L]);
  for (int l = 0; l < NN_LAYERS; ++l) {
    const Spec& s = kSpec[l];
    const std::string n = s.name;
    if (n == "enc0b" || n == "enc1b" || n == "enc2b" || s.up) continue;
    place(nn.t_lay[l], V[s.level_out] * s.co);
  }
  nn.t_out = nn.t_lay[NN_LAYERS - 1];
  nn.act_elems = off;
  MPL_TRY(mpl_ensure(c, nn.act, 2 * off + 256));
  if (train) {
    MPL_TRY(mpl_ensure(c, nn.gact, 2 * off + 256));
    // wgrad partials: worst layer
    size_t worst = 0;
    for (int l = 0; l < NN_LAYERS; ++l) {
      const Spec& s = kSpec[l];
      const int64_t nv = s.up ? V[s.level_in] : V[s.level_out];
      const int64_t chunks = (nv + NN_WGRAD_CHUNK - 1) / NN_WGRAD_CHUNK;
      const size_t jobs = (size_t)taps_of(s) * (s.ci / 16) * (s.co / 16);
      const size_t bias = (size_t)((V[s.level_out] + 4095) / 4096) * s.co;
      worst = std::max(worst, (size_t)chunks * jobs * 256 + bias);
    }
    MPL_TRY(mpl_ensure(c, nn.wpart, 4 * worst + 256));
    MPL_TRY(mpl_ensure(c, nn.lpart, 8 * 2 * 1024 + 64));
  }
  return MPL_OK;
}

struct View {
  uint16_t* p;
  int ld;
};

// Input and output views of layer l in the activation arena A (the same
// offsets address the gradient arena).
static View out_view(const NNState& nn, uint16_t* A, int l) {
  const int C[4] = {16, 32, 64, 128};
  const Spec& s = kSpec[l];
  const std::string n = s.name;
  if (n == "enc0b") return View{A + nn.t_cat[0] + C[0], 2 * C[0]};
  if (n == "enc1b") return View{A + nn.t_cat[1] + C[1], 2 * C[1]};
  if (n == "enc2b") return View{A + nn.t_cat[2] + C[2], 2 * C[2]};
  if (s.up) return View{A + nn.t_cat[s.level_out], 2 * C[s.level_out]};
  return View{A + nn.t_lay[l], s.co};
}
static void layer_views(const NNState& nn, uint16_t* A, int l, View& in, View& out) {
  const int C[4] = {16, 32, 64, 128};
  const Spec& s = kSpec[l];
  const std::string n = s.name;
  out = out_view(nn, A, l);
  if (l == 0) in = View{A + nn.t_in, 16};
  else if (n == "down0") in = out_view(nn, A, 1);
  else if (n == "down1") in = out_view(nn, A, 4);
  else if (n == "down2") in = out_view(nn, A, 7);
  else if (n == "dec2a") in = View{A + nn.t_cat[2], 2 * C[2]};
  else if (n == "dec1a") in = View{A + nn.t_cat[1], 2 * C[1]};
  else if (n == "dec0a") in = View{A + nn.t_cat[0], 2 * C[0]};
  else in = out_view(nn, A, l - 1);
}

static Dims3 level_dims(const NNState& nn, int L) {
  return Dims3{nn.box[0] >> L, nn.box[1] >> L, nn.box[2] >> L};
}

template <int CT>
static mpl_status launch_conv_ct(mpl_ctx* c, View in, Dims3 din, const uint16_t* wsw, int nk, int Ci,
                                 int T, int ks, int s, int p, const float* bias, View out,
                                 Dims3 dout, int relu, int accum, const int32_t* skip) {
  constexpr int VT = (CT <= 1) ? 4 : (CT <= 2 ? 2 : 1);
  const int64_t nv = (int64_t)dout.x * dout.y * dout.z;
  const int64_t per_wg = 4 * VT * 16;
  MPL_LAUNCH(c, (k_conv<CT, VT>), (int)((nv + per_wg - 1) / per_wg), 256, in.p, in.ld, din, wsw, nk,
             Ci, T, ks, s, p, bias, out.p, out.ld, dout, relu, accum, skip);
  return MPL_OK;
}
static mpl_status launch_conv(mpl_ctx* c, View in, Dims3 din, const uint16_t* wsw, int nk, int Ci,
                              int Co, int T, int ks, int s, int p, const float* bias, View out,
                              Dims3 dout, int relu, int accum, const int32_t* skip = nullptr) {
  switch (Co / 16) {
    case 1: return launch_conv_ct<1>(c, in, din, wsw, nk, Ci, T, ks, s, p, bias, out, dout, relu, accum, skip);
    case 2: return launch_conv_ct<2>(c, in, din, wsw, nk, Ci, T, ks, s, p, bias, out, dout, relu, accum, skip);
    case 4: return launch_conv_ct<4>(c, in, din, wsw, nk, Ci, T, ks, s, p, bias, out, dout, relu, accum, skip);
    case 8: return launch_conv_ct<8>(c, in, din, wsw, nk, Ci, T, ks, s, p, bias, out, dout, relu, accum, skip);
  }
  return mpl_fail(c, MPL_ERR_INVALID_ARG, "unsupported channel count");
}
template <int CT>
static mpl_status launch_conv3_ct(mpl_ctx* c, View in, Dims3 d, const uint16_t* wsw, int Ci, int CTT,
                                  const float* bias, View out, int relu, int accum, const int32_t* skip) {
  // as many workgroups as fit on the device at once (they stride over the
  // tiles), at most one per tile and output-channel group
  NNState& nn = *nn_state(c);
  int& resident = nn.lds_grid[CT == 1 ? 0 : (CT == 2 ? 1 : (CT == 4 ? 2 : 3))];
  if (resident == 0) {
    int cus = 0, per_cu = 0;
    MPL_HIP(c, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
    MPL_HIP(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_conv3_lds<CT>, 256, 0));
    resident = std::max(1, cus) * std::max(1, per_cu);
  }
  const int ny = CTT / CT;
  const int64_t ntiles = (int64_t)((d.x + 3) / 4) * ((d.y + 3) / 4) * ((d.z + 15) / 16);
  // grids with fewer than 256 (tile, channel-group) items (the 17^3 level
  // of the 136^3 box: 200) also split the input-channel chunks, each split
  // into FP32 partials reduced after; at 34^3 (486 items) the reduction's
  // traffic cost more than the added workgroups gained
  const int nchunk = Ci / 16;
  const int64_t items = std::max<int64_t>(1, ntiles * ny);
  const int nsplit = items < 256 ? (int)std::min<int64_t>(nchunk, std::max<int64_t>(1, 2048 / items)) : 1;
  const int nwg = (int)std::min<int64_t>(ntiles, std::max(1, resident / (ny * nsplit)));
  float* part = nullptr;
  const int64_t nv = (int64_t)d.x * d.y * d.z;
  const int co = 16 * CTT;
  if (nsplit > 1) {
    MPL_TRY(mpl_ensure(c, nn.csplit, sizeof(float) * (size_t)nsplit * nv * co));
    part = P<float>(nn.csplit);
  }
  hipLaunchKernelGGL((k_conv3_lds<CT>), dim3((unsigned)nwg, ny, nsplit), dim3(256), 0, c->stream, in.p,
                     in.ld, d, Ci, wsw, CTT, bias, out.p, out.ld, relu, accum, skip, part);
  MPL_HIP(c, hipGetLastError());
  if (nsplit > 1) {
    const int64_t n = nv * (co / 4);
    MPL_LAUNCH(c, k_conv3_split_reduce, (int)((n + 255) / 256), 256, (const float*)part, nsplit, nv, co, bias,
               out.p, out.ld, relu, accum, skip);
  }
  return MPL_OK;
}
// 3x3x3 stride-1 convolution with Ci input and Co output channels (multiples
// of 16).  Small grids split the output channels over workgroups (at most
// two 16-channel tiles each) so that the coarse levels still fill the GPU.
static mpl_status launch_conv3(mpl_ctx* c, View in, Dims3 d, const uint16_t* wsw, int Ci, int Co,
                               const float* bias, View out, int relu, int accum,
                               const int32_t* skip = nullptr) {
  const int CTT = Co / 16;
  const int64_t nwg = (int64_t)((d.x + 3) / 4) * ((d.y + 3) / 4) * ((d.z + 15) / 16);
  int CT = CTT;
  while (CT > 2 && nwg * (CTT / CT) < 4096) CT /= 2;
  switch (CT) {
    case 1: return launch_conv3_ct<1>(c, in, d, wsw, Ci, CTT, bias, out, relu, accum, skip);
    case 2: return launch_conv3_ct<2>(c, in, d, wsw, Ci, CTT, bias, out, relu, accum, skip);
    case 4: return launch_conv3_ct<4>(c, in, d, wsw, Ci, CTT, bias, out, relu, accum, skip);
    case 8: return launch_conv3_ct<8>(c, in, d, wsw, Ci, CTT, bias, out, relu, accum, skip);
  }
  return mpl_fail(c, MPL_ERR_INVALID_ARG, "unsupported channel count");
}
// 3x3x3 stride-1 convolution with Ci input (a multiple of 16) and 16 output
// channels on the register-blocked kernel.
static mpl_status launch_conv3_rr(mpl_ctx* c, View in, Dims3 d, const uint16_t* wrr, int Ci,
                                  const float* bias, View out, int relu, int accum,
                                  const int32_t* skip = nullptr) {
  // as many workgroups as fit on the device at once (they stride over the
  // tiles), at most one per tile
  NNState& nn = *nn_state(c);
  if (nn.rr_grid == 0) {
    int cus = 0, per_cu = 0;
    MPL_HIP(c, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
    MPL_HIP(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_conv3_rr, 256, 0));
    nn.rr_grid = std::max(1, cus) * std::max(1, per_cu);
  }
  const int64_t ntiles = (int64_t)((d.x + 7) / 8) * ((d.y + 3) / 4) * ((d.z + 15) / 16);
  const int nwg = (int)std::min<int64_t>(ntiles, nn.rr_grid);
  hipLaunchKernelGGL(k_conv3_rr, dim3((unsigned)nwg), dim3(256), 0, c->stream, in.p, in.ld, d, Ci, wrr,
                     bias, out.p, out.ld, relu, accum, skip);
  MPL_HIP(c, hipGetLastError());
  return MPL_OK;
}
template <int CT>
static mpl_status launch_up_ct(mpl_ctx* c, View in, Dims3 din, const uint16_t* wsw, int nk,
                               const float* bias, View out, int relu, int accum, const int32_t* skip) {
  constexpr int VT = (CT <= 1) ? 4 : (CT <= 2 ? 2 : 1);
  const int64_t nv = (int64_t)din.x * din.y * din.z;
  const int64_t per_wg = 4 * VT * 16;
  hipLaunchKernelGGL((k_up<CT, VT>), dim3((unsigned)((nv + per_wg - 1) / per_wg), 8), dim3(256), 0,
                     c->stream, in.p, in.ld, din, wsw, nk, bias, out.p, out.ld, relu, accum, skip);
  MPL_HIP(c, hipGetLastError());
  return MPL_OK;
}
static mpl_status launch_up(mpl_ctx* c, View in, Dims3 din, const uint16_t* wsw, int nk, int Co,
                            const float* bias, View out, int relu, int accum,
                            const int32_t* skip = nullptr) {
  switch (Co / 16) {
    case 1: return launch_up_ct<1>(c, in, din, wsw, nk, bias, out, relu, accum, skip);
    case 2: return launch_up_ct<2>(c, in, din, wsw, nk, bias, out, relu, accum, skip);
    case 4: return launch_up_ct<4>(c, in, din, wsw, nk, bias, out, relu, accum, skip);
    case 8: return launch_up_ct<8>(c, in, din, wsw, nk, bias, out, relu, accum, skip);
  }
  return mpl_fail(c, MPL_ERR_INVALID_ARG, "unsupported channel count");
}

// Forward of layer l on the tensors staged in nn.act.
static mpl_status nn_forward_layer(mpl_ctx* c, NNState& nn, int l) {
  uint16_t* A = (uint16_t*)nn.act.p;
  const uint16_t* sw = (const uint16_t*)nn.wsw.p;
  const float* P = (const float*)nn.params.p;
  const Spec& s = kSpec[l];
  const int T = taps_of(s);
  View in, out;
  layer_views(nn, A, l, in, out);
  const float* bias = P + w_offset(l) + (int64_t)T * s.ci * s.co;
  const Dims3 din = level_dims(nn, s.level_in), dout = level_dims(nn, s.level_out);
  if (s.up) {
    MPL_TRY(launch_up(c, in, din, sw + nn.sw_fwd_off[l], (s.ci + 31) / 32, s.co, bias, out, s.relu, 0,
                      nn.skip));
  } else if (s.k == 3 && nn.lds_conv && nn.rr_conv && s.co == 16) {
    MPL_TRY(launch_conv3_rr(c, in, din, sw + nn.sw3rr_fwd_off[l], s.ci, bias, out, s.relu, 0, nn.skip));
  } else if (s.k == 3 && nn.lds_conv) {
    MPL_TRY(launch_conv3(c, in, din, sw + nn.sw3_fwd_off[l], s.ci, s.co, bias, out, s.relu, 0, nn.skip));
  } else {
    MPL_TRY(launch_conv(c, in, din, sw + nn.sw_fwd_off[l], (T * s.ci + 31) / 32, s.ci, s.co, T, s.k,
                        s.s, s.p, bias, out, dout, s.relu, 0, nn.skip));
  }
  return MPL_OK;
}

// Forward pass on the tensors already staged in nn.act (input at t_in).
mpl_status nn_forward(mpl_ctx* c, NNState& nn) {
  for (int l = 0; l < NN_LAYERS; ++l) MPL_TRY(nn_forward_layer(c, nn, l));
  return MPL_OK;
}

// Backward of layer l: ReLU mask on its output gradient (staged in nn.gact),
// parameter gradients ADDED into nn.grad, and (if input_grad and l > 0) the
// gradient w.r.t. its input, accumulated into a down layer's input view
// when accum_down (the skip tensor's decoder share is already there).
static mpl_status nn_backward_layer(mpl_ctx* c, NNState& nn, int l, bool input_grad, bool accum_down) {
  uint16_t* A = (uint16_t*)nn.act.p;
  uint16_t* G = (uint16_t*)nn.gact.p;
  const uint16_t* sw = (const uint16_t*)nn.wsw.p;
  float* grad = (float*)nn.grad.p;
  float* part = (float*)nn.wpart.p;
  const Spec& s = kSpec[l];
  const int T = taps_of(s);
  View in, out, gin, gout;
  layer_views(nn, A, l, in, out);
  layer_views(nn, G, l, gin, gout);
  const Dims3 din = level_dims(nn, s.level_in), dout = level_dims(nn, s.level_out);
  const int64_t nvo = (int64_t)dout.x * dout.y * dout.z;
  if (s.relu)
    MPL_LAUNCH(c, k_relu_bwd, (int)((nvo * s.co + 255) / 256), 256, gout.p, gout.ld, out.p, out.ld,
               s.co, nvo);
  // parameter gradients
  float* gW = grad + w_offset(l);
  float* gb = gW + (int64_t)T * s.ci * s.co;
  {
    const int64_t nv = s.up ? (int64_t)din.x * din.y * din.z : nvo;
    const int chunks = (int)((nv + NN_WGRAD_CHUNK - 1) / NN_WGRAD_CHUNK);
    const int jobs = T * (s.ci / 16) * (s.co / 16);
    hipLaunchKernelGGL(k_wgrad, dim3(chunks, jobs), dim3(64), 0, c->stream, in.p, in.ld, din,
                       gout.p, gout.ld, dout, s.ci, s.co, s.up ? 2 : s.k, s.up ? 2 : s.s,
                       s.up ? 0 : s.p, s.up, NN_WGRAD_CHUNK, part);
    MPL_HIP(c, hipGetLastError());
    MPL_LAUNCH(c, k_wgrad_reduce, (jobs * 256 + 255) / 256, 256, part, chunks, jobs, s.ci, s.co, gW);
    {
      const int64_t chunk = 4096;
      const int nch = (int)((nvo + chunk - 1) / chunk);
      float* bpart = part + (size_t)chunks * jobs * 256;  // after the weight-gradient partials
      MPL_LAUNCH(c, k_bias_partial, nch, 256, gout.p, gout.ld, nvo, s.co, chunk, bpart);
      MPL_LAUNCH(c, k_bias_reduce, 1, 128, bpart, nch, s.co, gb);
    }
  }
  if (l == 0 || !input_grad) return MPL_OK;  // no gradient w.r.t. the network input
  // gradient w.r.t. the layer input; the down layers' input is a skip
  // tensor whose gradient already holds the decoder's share: accumulate.
  const int accum = (accum_down && s.k == 2 && !s.up) ? 1 : 0;
  if (s.up) {
    // dgrad of a transposed conv: 2x2x2 stride-2 gather conv, K = (t, o)
    MPL_TRY(launch_conv(c, gout, dout, sw + nn.sw_bwd_off[l], (T * s.co + 31) / 32, s.co, s.ci, T, 2, 2,
                        0, nullptr, gin, din, 0, accum));
  } else if (s.k == 2) {
    MPL_TRY(launch_up(c, gout, dout, sw + nn.sw_bwd_off[l], (s.co + 31) / 32, s.ci, nullptr, gin, 0,
                      accum));
  } else if (s.k == 3 && nn.lds_conv && nn.rr_conv && s.ci == 16) {
    MPL_TRY(launch_conv3_rr(c, gout, dout, sw + nn.sw3rr_bwd_off[l], s.co, nullptr, gin, 0, accum));
  } else if (s.k == 3 && nn.lds_conv) {
    MPL_TRY(launch_conv3(c, gout, dout, sw + nn.sw3_bwd_off[l], s.co, s.ci, nullptr, gin, 0, accum));
  } else {
    MPL_TRY(launch_conv(c, gout, dout, sw + nn.sw_bwd_off[l], (T * s.co + 31) / 32, s.co, s.ci, T, s.k,
                        1, s.p, nullptr, gin, din, 0, accum));
  }
  return MPL_OK;
}

// Backward pass: the gradient w.r.t. the output must be staged at
// gact[t_out]; parameter gradients are ADDED into nn.grad.
mpl_status nn_backward(mpl_ctx* c, NNState& nn) {
  for (int l = NN_LAYERS - 1; l >= 0; --l) MPL_TRY(nn_backward_layer(c, nn, l, true, true));
  return MPL_OK;
}

// One layer on caller tensors: x [in voxels][Ci] into the layer's input
// view, dy [out voxels][Co] into its output-gradient view (FP32 -> BF16);
// y, dx read back from the output and input-gradient views (BF16 -> FP32).
__global__ void k_view_in(const float* __restrict__ src, int64_t nv, int ch, uint16_t* __restrict__ dst,
                          int ld) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nv * ch) dst[(i / ch) * ld + i % ch] = f2bf(src[i]);
}
__global__ void k_view_out(const uint16_t* __restrict__ src, int ld, int64_t nv, int ch,
                           float* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nv * ch) dst[i] = bf2f(src[(i / ch) * ld + i % ch]);
}

static mpl_status nn_layer_grad(mpl_ctx* c, int l, const float* x, const int32_t dims[3], const float* dy,
                                float* y, float* dx, float* dparams) {
  NNState& nn = *c->nn;
  const int d[3] = {dims[0], dims[1], dims[2]};
  MPL_TRY(nn_buffers(c, nn, d, true));
  const Spec& s = kSpec[l];
  const int T = taps_of(s);
  const int32_t* saved_skip = nn.skip;
  nn.skip = nullptr;
  uint16_t* A = (uint16_t*)nn.act.p;
  uint16_t* G = (uint16_t*)nn.gact.p;
  View in, out, gin, gout;
  layer_views(nn, A, l, in, out);
  layer_views(nn, G, l, gin, gout);
  const Dims3 din = level_dims(nn, s.level_in), dout = level_dims(nn, s.level_out);
  const int64_t nvi = (int64_t)din.x * din.y * din.z, nvo = (int64_t)dout.x * dout.y * dout.z;
  MPL_HIP(c, hipMemsetAsync(nn.gact.p, 0, 2 * nn.act_elems, c->stream));
  MPL_HIP(c, hipMemsetAsync(nn.grad.p, 0, 4 * nn_param_count(), c->stream));
  MPL_LAUNCH(c, k_view_in, (int)((nvi * s.ci + 255) / 256), 256, x, nvi, s.ci, in.p, in.ld);
  MPL_TRY(nn_forward_layer(c, nn, l));
  MPL_LAUNCH(c, k_view_in, (int)((nvo * s.co + 255) / 256), 256, dy, nvo, s.co, gout.p, gout.ld);
  mpl_status st = nn_backward_layer(c, nn, l, true, false);
  nn.skip = saved_skip;
  MPL_TRY(st);
  if (y) MPL_LAUNCH(c, k_view_out, (int)((nvo * s.co + 255) / 256), 256, out.p, out.ld, nvo, s.co, y);
  if (dx && l > 0) MPL_LAUNCH(c, k_view_out, (int)((nvi * s.ci + 255) / 256), 256, gin.p, gin.ld, nvi, s.ci, dx);
  if (dparams)
    MPL_HIP(c, hipMemcpyAsync(dparams, (float*)nn.grad.p + w_offset(l),
                              4 * ((int64_t)T * s.ci * s.co + s.co), hipMemcpyDeviceToDevice, c->stream));
  MPL_HIP(c, hipStreamSynchronize(c->stream));
  return MPL_OK;
}

NNState* nn_state(mpl_ctx* c) {
  if (!c->nn) {
    c->nn = new NNState();
    const char* dc = std::getenv("MPL_NN_DIRECT_CONV");
    c->nn->lds_conv = !(dc && dc[0] == '1');
    const char* rr = std::getenv("MPL_NN_RR_CONV");
    c->nn->rr_conv = !(rr && rr[0] == '0');
  }
  return c->nn;
}

void nn_destroy(mpl_ctx* c) {
  if (!c->nn) return;
  NNState& nn = *c->nn;
  DevBuf* all[] = {&nn.params, &nn.grad, &nn.adam_m, &nn.adam_v, &nn.wsw, &nn.act, &nn.gact,
                   &nn.wpart, &nn.lpart, &nn.tmp, &nn.dref, &nn.csplit};
  for (DevBuf* b : all) mpl_dev_free(c, b->p, b->bytes);
  if (nn.store) {
    DevBuf* st[] = {&nn.store->feat, &nn.store->target, &nn.store->mask};
    for (DevBuf* b : st) mpl_dev_free(c, b->p, b->bytes);
    delete nn.store;
  }
  delete c->nn;
  c->nn = nullptr;
}

mpl_status nn_stage_input_f32(mpl_ctx* c, NNState& nn, const float* x) {
  const int64_t n = (int64_t)nn.box[0] * nn.box[1] * nn.box[2] * 16;
  MPL_LAUNCH(c, k_f32_to_bf16, (int)((n + 255) / 256), 256, x, (uint16_t*)nn.act.p + nn.t_in, n);
  return MPL_OK;
}

// ======================================================================
extern "C" {

mpl_status mpl_precond_param_count(mpl_ctx* c, int64_t* n) {
  if (!c || !n) return MPL_ERR_INVALID_ARG;
  *n = nn_param_count();
  return MPL_OK;
}

mpl_status mpl_precond_set_weights(mpl_ctx* c, const float* params, int64_t n) {
  if (!c || !params || n != nn_param_count()) return MPL_ERR_INVALID_ARG;
  NNState& nn = *nn_state(c);
  MPL_TRY(nn_alloc(c, nn));
  MPL_HIP(c, hipMemcpyAsync(nn.params.p, params, 4 * n, hipMemcpyHostToDevice, c->stream));
  MPL_HIP(c, hipMemsetAsync(nn.adam_m.p, 0, 4 * n, c->stream));
  MPL_HIP(c, hipMemsetAsync(nn.adam_v.p, 0, 4 * n, c->stream));
  nn.adam_t = 0;
  MPL_TRY(nn_refresh(c, nn));
  MPL_HIP(c, hipStreamSynchronize(c->stream));
  return MPL_OK;
}

mpl_status mpl_precond_get_weights(mpl_ctx* c, float* params, int64_t n) {
  if (!c || !params || n != nn_param_count()) return MPL_ERR_INVALID_ARG;
  if (!c->nn || !c->nn->ready) return mpl_fail(c, MPL_ERR_STATE, "no network weights");
  MPL_HIP(c, hipMemcpyAsync(params, c->nn->params.p, 4 * n, hipMemcpyDeviceToHost, c->stream));
  MPL_HIP(c, hipStreamSynchronize(c->stream));
  return MPL_OK;
}

mpl_status mpl_nn_forward(mpl_ctx* c, const float* x, const int32_t dims[3], float* y) {
  if (!c || !x || !y || !dims) return MPL_ERR_INVALID_ARG;
  if (!c->nn || !c->nn->ready) return mpl_fail(c, MPL_ERR_STATE, "no network weights");
  NNState& nn = *c->nn;
  int d[3] = {dims[0], dims[1], dims[2]};
  MPL_TRY(nn_buffers(c, nn, d, false));
  // every layer writes all voxels and channels of its output: no clearing
  MPL_TRY(nn_stage_input_f32(c, nn, x));
  MPL_TRY(nn_forward(c, nn));
  const int64_t n = (int64_t)d[0] * d[1] * d[2] * 16;
  MPL_LAUNCH(c, k_bf16_to_f32, (int)((n + 255) / 256), 256, (const uint16_t*)nn.act.p + nn.t_out, y, n);
  MPL_HIP(c, hipStreamSynchronize(c->stream));
  return MPL_OK;
}

mpl_status mpl_nn_backward(mpl_ctx* c, const float* x, const int32_t dims[3], const float* dy,
                           float* grad) {
  if (!c || !x || !dy || !grad || !dims) return MPL_ERR_INVALID_ARG;
  if (!c->nn || !c->nn->ready) return mpl_fail(c, MPL_ERR_STATE, "no network weights");
  NNState& nn = *c->nn;
  int d[3] = {dims[0], dims[1], dims[2]};
  MPL_TRY(nn_buffers(c, nn, d, true));
  MPL_HIP(c, hipMemsetAsync(nn.act.p, 0, 2 * nn.act_elems, c->stream));
  MPL_HIP(c, hipMemsetAsync(nn.gact.p, 0, 2 * nn.act_elems, c->stream));
  MPL_TRY(nn_stage_input_f32(c, nn, x));
  MPL_TRY(nn_forward(c, nn));
  const int64_t n = (int64_t)d[0] * d[1] * d[2] * 16;
  MPL_LAUNCH(c, k_f32_to_bf16, (int)((n + 255) / 256), 256, dy, (uint16_t*)nn.gact.p + nn.t_out, n);
  MPL_HIP(c, hipMemsetAsync(nn.grad.p, 0, 4 * nn_param_count(), c->stream));
  MPL_TRY(nn_backward(c, nn));
  MPL_HIP(c, hipMemcpyAsync(grad, nn.grad.p, 4 * nn_param_count(), hipMemcpyDeviceToDevice, c->stream));
  MPL_HIP(c, hipStreamSynchronize(c->stream));
  return MPL_OK;
}

// One Adam step on the masked relative L2 loss of one sample (device
// tensors: x [X][Y][Z][16] FP32 features, t [X][Y][Z][3] FP32 targets,
// mask [X][Y][Z] FP32).  loss (host, may be NULL) gets the loss before the
// step, grads_out (device, may be NULL) the parameter gradient it applies.
mpl_status mpl_precond_train_step(mpl_ctx* c, const float* x, const float* t, const float* mask,
                                  const int32_t dims[3], float lr, float* loss, float* grads_out) {
  if (!c || !x || !t || !mask || !dims) return MPL_ERR_INVALID_ARG;
  if (!c->nn || !c->nn->ready) return mpl_fail(c, MPL_ERR_STATE, "no network weights");
  NNState& nn = *c->nn;
  int d[3] = {dims[0], dims[1], dims[2]};
  MPL_TRY(nn_buffers(c, nn, d, true));
  const int64_t nvox = (int64_t)d[0] * d[1] * d[2];
  MPL_HIP(c, hipMemsetAsync(nn.gact.p, 0, 2 * nn.act_elems, c->stream));
  MPL_TRY(nn_stage_input_f32(c, nn, x));
  MPL_TRY(nn_forward(c, nn));
  const uint16_t* y = (const uint16_t*)nn.act.p + nn.t_out;
  double* lp = (double*)nn.lpart.p;
  const int nwg = 1024;
  MPL_LAUNCH(c, k_loss_partial, nwg, 256, y, 16, t, mask, nvox, lp + 8);
  MPL_LAUNCH(c, k_loss_final, 1, 1, lp + 8, nwg, lp);
  MPL_LAUNCH(c, k_loss_grad, (int)((nvox + 255) / 256), 256, y, 16, t, mask, nvox, lp,
             (uint16_t*)nn.gact.p + nn.t_out, 16);
  const int64_t np = nn_param_count();
  MPL_HIP(c, hipMemsetAsync(nn.grad.p, 0, 4 * np, c->stream));
  MPL_TRY(nn_backward(c, nn));
  if (grads_out)
    MPL_HIP(c, hipMemcpyAsync(grads_out, nn.grad.p, 4 * np, hipMemcpyDeviceToDevice, c->stream));
  nn.adam_t += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)nn.adam_t), c2 = 1.f - powf(b2, (float)nn.adam_t);
  MPL_LAUNCH(c, k_adam, (int)((np + 255) / 256), 256, (float*)nn.params.p, (const float*)nn.grad.p,
             (float*)nn.adam_m.p, (float*)nn.adam_v.p, np, lr, b1, b2, 1e-8f, c1, c2);
  MPL_TRY(nn_refresh(c, nn));
  if (loss) {
    double h[3];
    MPL_HIP(c, hipMemcpyAsync(h, lp, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    MPL_HIP(c, hipStreamSynchronize(c->stream));
    *loss = (float)h[2];
  }
  return MPL_OK;
}

}  // extern "C"

// ======================================================================
// The network on the solver grid.
namespace {

__global__ __launch_bounds__(64) void k_dref_partial(const double* __restrict__ Dinv,
                                                     const uint8_t* __restrict__ flags, int64_t nnode,
                                                     double* __restrict__ part) {
  const int nb = blockIdx.x, l = threadIdx.x;
  const int64_t ni = (int64_t)nb * MPL_BC + l;
  // a node with a free component contributes the mean diagonal over its
  // free components
  double s = 0.0, n = 0.0;
  const uint8_t fl = flags[ni];
  if (fl & MPL_NODE_FREE_ALL) {
    int nf = 0;
    for (int a = 0; a < 3; ++a)
      if (mpl_free(fl, a)) {
        s += 1.0 / Dinv[a * nnode + ni];
        ++nf;
      }
    s /= nf;
    n = 1.0;
  }
  s = wave_sum(s);
  n = wave_sum(n);
  if (l == 0) {
    part[2 * nb] = s;
    part[2 * nb + 1] = n;
  }
}
__global__ __launch_bounds__(1024) void k_dref_final(const double* __restrict__ part, int n,
                                                     double* __restrict__ out) {
  __shared__ double sh[2][16];
  const int t = threadIdx.x;
  double s = 0.0, m = 0.0;
  for (int i = t; i < n; i += 1024) {
    s += part[2 * i];
    m += part[2 * i + 1];
  }
  s = wave_sum(s);
  m = wave_sum(m);
  if ((t & 63) == 0) {
    sh[0][t >> 6] = s;
    sh[1][t >> 6] = m;
  }
  __syncthreads();
  if (t != 0) return;
  double S = 0.0, M = 0.0;
  for (int w = 0; w < 16; ++w) {
    S += sh[0][w];
    M += sh[1][w];
  }
  out[0] = M > 0.0 ? S / M : 1.0;
}

struct Box3 {
  int d[3];
};

// Map box voxel (i, j, k) (= grid node) to its compact node index, -1 when
// its node block is inactive.
__device__ __forceinline__ int64_t voxel_node(int i, int j, int k, const int32_t* __restrict__ nmap,
                                              Box3 nbd) {
  const int bx = i >> 2, by = j >> 2, bz = k >> 2;
  if (bx >= nbd.d[0] || by >= nbd.d[1] || bz >= nbd.d[2]) return -1;
  const int id = nmap[((int64_t)bx * nbd.d[1] + by) * nbd.d[2] + bz];
  if (id < 0) return -1;
  return (int64_t)id * MPL_BC + (((i & 3) * 4 + (j & 3)) * 4 + (k & 3));
}

// Network input for node vector r, one thread per box voxel (every voxel
// written, zeros off the free nodes): [voxel][16] bf16.
__global__ __launch_bounds__(256) void k_features(const double* __restrict__ r,
                                                  const double* __restrict__ Dinv,
                                                  const uint8_t* __restrict__ flags,
                                                  const int32_t* __restrict__ nmap, Box3 nbd,
                                                  int64_t nnode, Box3 box,
                                                  const double* __restrict__ s2, double inv_nfree,
                                                  const double* __restrict__ dref,
                                                  uint16_t* __restrict__ feat) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nv = (int64_t)box.d[0] * box.d[1] * box.d[2];
  if (v >= nv) return;
  const int k = (int)(v % box.d[2]), j = (int)((v / box.d[2]) % box.d[1]),
            i = (int)(v / ((int64_t)box.d[2] * box.d[1]));
  const int64_t ni = voxel_node(i, j, k, nmap, nbd);
  float f[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
  const uint8_t fl = ni >= 0 ? flags[ni] : (uint8_t)0;
  if (fl & MPL_NODE_FREE_ALL) {
    // fixed components (Dinv = 0) read as 0; the diagonal channel is the
    // mean over the free ones
    const double sc = sqrt(fmax(s2[0] * inv_nfree, 1e-300));
    double dm = 0.0;
    int nf = 0;
    for (int a = 0; a < 3; ++a) {
      if (!mpl_free(fl, a)) continue;
      const double di = Dinv[a * nnode + ni];
      f[a] = (float)(sqrt(di) * r[a * nnode + ni] / sc);
      dm += 1.0 / di;
      ++nf;
    }
    f[3] = (float)log(dm / nf / dref[0]);
    f[4] = 1.f;
  }
  uint16_t* dst = feat + v * 16;
  uint4 lo, hi = make_uint4(0, 0, 0, 0);
  lo.x = (uint32_t)f2bf(f[0]) | ((uint32_t)f2bf(f[1]) << 16);
  lo.y = (uint32_t)f2bf(f[2]) | ((uint32_t)f2bf(f[3]) << 16);
  lo.z = (uint32_t)f2bf(f[4]);
  lo.w = 0;
  reinterpret_cast<uint4*>(dst)[0] = lo;
  reinterpret_cast<uint4*>(dst)[1] = hi;
}

__global__ __launch_bounds__(256) void k_record(const double* __restrict__ r, const double* __restrict__ x,
                                                const double* __restrict__ xstar,
                                                const double* __restrict__ Dinv,
                                                const uint8_t* __restrict__ flags,
                                                const int32_t* __restrict__ nmap, Box3 nbd,
                                                int64_t nnode, Box3 box, const double* __restrict__ s2,
                                                double inv_nfree, float* __restrict__ target,
                                                float* __restrict__ mask) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nv = (int64_t)box.d[0] * box.d[1] * box.d[2];
  if (v >= nv) return;
  const int k = (int)(v % box.d[2]), j = (int)((v / box.d[2]) % box.d[1]),
            i = (int)(v / ((int64_t)box.d[2] * box.d[1]));
  const int64_t ni = voxel_node(i, j, k, nmap, nbd);
  const uint8_t fl = ni >= 0 ? flags[ni] : (uint8_t)0;
  const bool fr = (fl & MPL_NODE_FREE_ALL) != 0;
  const double sc = sqrt(fmax(s2[0] * inv_nfree, 1e-300));
  for (int a = 0; a < 3; ++a) {
    double t = 0.0;
    if (mpl_free(fl, a)) {
      const int64_t q = a * nnode + ni;
      const double di = Dinv[q];
      const double e = xstar[q] - x[q];
      t = (e - di * r[q]) / (sqrt(di) * sc);
    }
    target[v * 3 + a] = (float)t;
  }
  mask[v] = fr ? 1.f : 0.f;
}

// Output gradient of the network from a node vector g (3 comps, block
// layout): gact[t_out][voxel][a] = g_a at the voxel's node (free nodes), all
// other channels and voxels 0.
__global__ __launch_bounds__(256) void k_out_grad(const double* __restrict__ g,
                                                  const uint8_t* __restrict__ flags,
                                                  const int32_t* __restrict__ nmap, Box3 nbd,
                                                  int64_t nnode, Box3 box, uint16_t* __restrict__ gout) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nv = (int64_t)box.d[0] * box.d[1] * box.d[2];
  if (v >= nv) return;
  const int k = (int)(v % box.d[2]), j = (int)((v / box.d[2]) % box.d[1]),
            i = (int)(v / ((int64_t)box.d[2] * box.d[1]));
  const int64_t ni = voxel_node(i, j, k, nmap, nbd);
  float f[3] = {0.f, 0.f, 0.f};
  const uint8_t fl = ni >= 0 ? flags[ni] : (uint8_t)0;
  for (int a = 0; a < 3; ++a)
    if (mpl_free(fl, a)) f[a] = (float)g[a * nnode + ni];
  uint4 lo, hi = make_uint4(0, 0, 0, 0);
  lo.x = (uint32_t)f2bf(f[0]) | ((uint32_t)f2bf(f[1]) << 16);
  lo.y = (uint32_t)f2bf(f[2]);
  lo.z = 0;
  lo.w = 0;
  reinterpret_cast<uint4*>(gout + v * 16)[0] = lo;
  reinterpret_cast<uint4*>(gout + v * 16)[1] = hi;
}

}  // namespace

NNSampleStore& nn_samples(mpl_ctx* c) {
  NNState& nn = *nn_state(c);
  if (!nn.store) nn.store = new NNSampleStore();
  return *nn.store;
}

mpl_status nn_prepare_box(mpl_ctx* c, bool train) {
  NNState& nn = *nn_state(c);
  if (!nn.ready) return mpl_fail(c, MPL_ERR_STATE, "no network weights");
  int d[3];
  for (int a = 0; a < 3; ++a) d[a] = ((c->dims[a] + 1 + 7) / 8) * 8;
  MPL_TRY(nn_buffers(c, nn, d, train));
  MPL_TRY(mpl_ensure(c, nn.dref, 64));
  return MPL_OK;
}

mpl_status nn_set_dref(mpl_ctx* c, const double* Dinv) {
  NNState& nn = *nn_state(c);
  MPL_TRY(mpl_ensure(c, nn.tmp, sizeof(double) * 2 * (c->n_nblk + 64)));
  MPL_TRY(mpl_ensure(c, nn.dref, 64));
  MPL_LAUNCH(c, k_dref_partial, c->n_nblk, 64, Dinv, P<uint8_t>(c->flags), (int64_t)c->nnode_alloc(),
             P<double>(nn.tmp));
  MPL_LAUNCH(c, k_dref_final, 1, 1024, P<double>(nn.tmp), c->n_nblk, P<double>(nn.dref));
  return MPL_OK;
}

double nn_inv_free_dofs(mpl_ctx* c) {
  const double n = std::max(1, c->hscal.n_free_dofs);
  return 1.0 / n;
}
static double inv_nfree(mpl_ctx* c) { return nn_inv_free_dofs(c); }

mpl_status nn_stage_features(mpl_ctx* c, const double* r, const double* Dinv, const double* s2) {
  NNState& nn = *nn_state(c);
  const int64_t nv = (int64_t)nn.box[0] * nn.box[1] * nn.box[2];
  uint16_t* feat = (uint16_t*)nn.act.p + nn.t_in;
  Box3 b{{nn.box[0], nn.box[1], nn.box[2]}}, nbd{{c->nbd[0], c->nbd[1], c->nbd[2]}};
  MPL_LAUNCH(c, k_features, (int)((nv + 255) / 256), 256, r, Dinv, P<uint8_t>(c->flags),
             P<int32_t>(c->nmap), nbd, (int64_t)c->nnode_alloc(), b, s2, inv_nfree(c),
             P<double>(nn.dref), feat);
  return MPL_OK;
}

mpl_status nn_stage_output_grad(mpl_ctx* c, const double* g) {
  NNState& nn = *nn_state(c);
  const int64_t nv = (int64_t)nn.box[0] * nn.box[1] * nn.box[2];
  Box3 b{{nn.box[0], nn.box[1], nn.box[2]}}, nbd{{c->nbd[0], c->nbd[1], c->nbd[2]}};
  MPL_LAUNCH(c, k_out_grad, (int)((nv + 255) / 256), 256, g, P<uint8_t>(c->flags), P<int32_t>(c->nmap),
             nbd, (int64_t)c->nnode_alloc(), b, (uint16_t*)nn.gact.p + nn.t_out);
  return MPL_OK;
}

mpl_status nn_stage_output_f32(mpl_ctx* c, const float* o_box) {
  NNState& nn = *nn_state(c);
  const int64_t n = (int64_t)nn.box[0] * nn.box[1] * nn.box[2] * 16;
  MPL_LAUNCH(c, k_f32_to_bf16, (int)((n + 255) / 256), 256, o_box, (uint16_t*)nn.act.p + nn.t_out, n);
  return MPL_OK;
}

mpl_status nn_record_sample(mpl_ctx* c, const double* r, const double* x, const double* xstar,
                            const double* Dinv, const double* s2) {
  NNState& nn = *nn_state(c);
  NNSampleStore& st = nn_samples(c);
  const int64_t nv = (int64_t)nn.box[0] * nn.box[1] * nn.box[2];
  if (st.voxels != nv) {
    st.voxels = nv;
    st.count = 0;
  }
  if (st.count >= st.capacity) return mpl_fail(c, MPL_ERR_OOM, "training sample store is full");
  MPL_TRY(nn_stage_features(c, r, Dinv, s2));
  uint16_t* feat = P<uint16_t>(st.feat) + (int64_t)st.count * nv * 16;
  MPL_HIP(c, hipMemcpyAsync(feat, (uint16_t*)nn.act.p + nn.t_in, 2 * nv * 16, hipMemcpyDeviceToDevice,
                            c->stream));
  float* tgt = P<float>(st.target) + (int64_t)st.count * nv * 3;
  float* msk = P<float>(st.mask) + (int64_t)st.count * nv;
  Box3 b{{nn.box[0], nn.box[1], nn.box[2]}}, nbd{{c->nbd[0], c->nbd[1], c->nbd[2]}};
  MPL_LAUNCH(c, k_record, (int)((nv + 255) / 256), 256, r, x, xstar, Dinv, P<uint8_t>(c->flags),
             P<int32_t>(c->nmap), nbd, (int64_t)c->nnode_alloc(), b, s2, inv_nfree(c), tgt, msk);
  st.count += 1;
  return MPL_OK;
}

// Parameter gradient of the loss whose output gradient is staged at
// gact[t_out] (activations of the same input in act), then one Adam step
// and the refresh of the swizzled BF16 weights.
mpl_status nn_backward_update(mpl_ctx* c, NNState& nn, float lr) {
  const int64_t np = nn_param_count();
  MPL_HIP(c, hipMemsetAsync(nn.grad.p, 0, 4 * np, c->stream));
  MPL_TRY(nn_backward(c, nn));
  return nn_adam_update(c, nn, lr);
}

mpl_status nn_adam_update(mpl_ctx* c, NNState& nn, float lr) {
  const int64_t np = nn_param_count();
  nn.adam_t += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)nn.adam_t), c2 = 1.f - powf(b2, (float)nn.adam_t);
  MPL_LAUNCH(c, k_adam, (int)((np + 255) / 256), 256, (float*)nn.params.p, (const float*)nn.grad.p,
             (float*)nn.adam_m.p, (float*)nn.adam_v.p, np, lr, b1, b2, 1e-8f, c1, c2);
  MPL_TRY(nn_refresh(c, nn));
  return MPL_OK;
}

// one Adam step on a staged bf16 sample
static mpl_status nn_train_on(mpl_ctx* c, NNState& nn, const uint16_t* feat, const float* t,
                              const float* mask, float lr, double* loss_dev) {
  const int64_t nvox = (int64_t)nn.box[0] * nn.box[1] * nn.box[2];
  MPL_HIP(c, hipMemcpyAsync((uint16_t*)nn.act.p + nn.t_in, feat, 2 * nvox * 16, hipMemcpyDeviceToDevice,
                            c->stream));
  MPL_TRY(nn_forward(c, nn));
  const uint16_t* y = (const uint16_t*)nn.act.p + nn.t_out;
  double* lp = (double*)nn.lpart.p;
  MPL_LAUNCH(c, k_loss_partial, 1024, 256, y, 16, t, mask, nvox, lp + 8);
  MPL_LAUNCH(c, k_loss_final, 1, 1, lp + 8, 1024, loss_dev);
  MPL_LAUNCH(c, k_loss_grad, (int)((nvox + 255) / 256), 256, y, 16, t, mask, nvox, loss_dev,
             (uint16_t*)nn.gact.p + nn.t_out, 16);
  return nn_backward_update(c, nn, lr);
}

extern "C" {

mpl_status mpl_precond_reserve(mpl_ctx* c, int32_t capacity) {
  if (!c || capacity < 0) return MPL_ERR_INVALID_ARG;
  if (!c->nn || !c->nn->ready) return mpl_fail(c, MPL_ERR_STATE, "set network weights first");
  MPL_TRY(nn_prepare_box(c, true));
  NNSampleStore& st = nn_samples(c);
  NNState& nn = *c->nn;
  const int64_t nv = (int64_t)nn.box[0] * nn.box[1] * nn.box[2];
  MPL_TRY(mpl_ensure(c, st.feat, (size_t)2 * nv * 16 * std::max(capacity, 1)));
  MPL_TRY(mpl_ensure(c, st.target, (size_t)4 * nv * 3 * std::max(capacity, 1)));
  MPL_TRY(mpl_ensure(c, st.mask, (size_t)4 * nv * std::max(capacity, 1)));
  st.capacity = capacity;
  st.count = 0;
  st.voxels = nv;
  return MPL_OK;
}

mpl_status mpl_precond_collect(mpl_ctx* c, int32_t every, double rtol) {
  if (!c || every < 0 || !(rtol > 0.0)) return MPL_ERR_INVALID_ARG;
  c->collect_every = every;
  c->collect_rtol = rtol;
  return MPL_OK;
}

mpl_status mpl_precond_online(mpl_ctx* c, int32_t every, int32_t steps, float lr) {
  if (!c || every < 0 || steps < 0 || !(lr >= 0.f)) return MPL_ERR_INVALID_ARG;
  if (every > 0 && (!c->nn || !c->nn->ready)) return mpl_fail(c, MPL_ERR_STATE, "set network weights first");
  c->online_every = every;
  c->online_steps = steps;
  c->online_lr = lr;
  return MPL_OK;
}

mpl_status mpl_precond_online_stats(mpl_ctx* c, int64_t* steps_done, double* mean_loss,
                                    double* mean_jacobi_loss) {
  if (!c) return MPL_ERR_INVALID_ARG;
  if (steps_done) *steps_done = c->online_done;
  if (mean_loss) *mean_loss = c->online_loss_n ? c->online_loss_sum / (double)c->online_loss_n : 0.0;
  if (mean_jacobi_loss)
    *mean_jacobi_loss = c->online_loss_n ? c->online_ref_sum / (double)c->online_loss_n : 0.0;
  c->online_loss_sum = 0.0;
  c->online_ref_sum = 0.0;
  c->online_loss_n = 0;
  return MPL_OK;
}

mpl_status mpl_nn_layer_grad(mpl_ctx* c, int32_t layer, const float* x, const int32_t dims[3],
                             const float* dy, float* y, float* dx, float* dparams) {
  if (!c || !x || !dims || !dy || layer < 0 || layer >= NN_LAYERS) return MPL_ERR_INVALID_ARG;
  if (!c->nn || !c->nn->ready) return mpl_fail(c, MPL_ERR_STATE, "set network weights first");
  return nn_layer_grad(c, layer, x, dims, dy, y, dx, dparams);
}

mpl_status mpl_precond_adam_step(mpl_ctx* c, const float* grad, float lr) {
  if (!c || !grad) return MPL_ERR_INVALID_ARG;
  if (!c->nn || !c->nn->ready) return mpl_fail(c, MPL_ERR_STATE, "set network weights first");
  NNState& nn = *c->nn;
  MPL_HIP(c, hipMemcpyAsync(nn.grad.p, grad, 4 * nn_param_count(), hipMemcpyDeviceToDevice, c->stream));
  MPL_TRY(nn_adam_update(c, nn, lr));
  MPL_HIP(c, hipStreamSynchronize(c->stream));
  return MPL_OK;
}

mpl_status mpl_precond_get_sample(mpl_ctx* c, int32_t i, float* feat, float* target, float* mask) {
  if (!c) return MPL_ERR_INVALID_ARG;
  if (!c->nn || !c->nn->store) return mpl_fail(c, MPL_ERR_STATE, "no training samples");
  NNSampleStore& st = *c->nn->store;
  if (i < 0 || i >= st.count) return mpl_fail(c, MPL_ERR_INVALID_ARG, "sample index out of range");
  const int64_t nv = st.voxels;
  if (feat)
    MPL_LAUNCH(c, k_bf16_to_f32, (int)((nv * 16 + 255) / 256), 256,
               P<uint16_t>(st.feat) + (int64_t)i * nv * 16, feat, nv * 16);
  if (target)
    MPL_HIP(c, hipMemcpyAsync(target, P<float>(st.target) + (int64_t)i * nv * 3, 4 * nv * 3,
                              hipMemcpyDeviceToDevice, c->stream));
  if (mask)
    MPL_HIP(c, hipMemcpyAsync(mask, P<float>(st.mask) + (int64_t)i * nv, 4 * nv, hipMemcpyDeviceToDevice,
                              c->stream));
  MPL_HIP(c, hipStreamSynchronize(c->stream));
  return MPL_OK;
}

mpl_status mpl_precond_sample_count(mpl_ctx* c, int32_t* n) {
  if (!c || !n) return MPL_ERR_INVALID_ARG;
  *n = (c->nn && c->nn->store) ? c->nn->store->count : 0;
  return MPL_OK;
}

// Train on the stored samples: n_steps Adam steps cycling through the
// samples in a fixed pseudo-random order; losses[i] (host, may be NULL)
// receives the loss of step i before its update.
mpl_status mpl_precond_train(mpl_ctx* c, int32_t n_steps, float lr, uint32_t seed, float* losses) {
  if (!c || n_steps < 0) return MPL_ERR_INVALID_ARG;
  if (!c->nn || !c->nn->ready || !c->nn->store || c->nn->store->count == 0)
    return mpl_fail(c, MPL_ERR_STATE, "no training samples");
  NNState& nn = *c->nn;
  MPL_TRY(nn_prepare_box(c, true));
  NNSampleStore& st = *nn.store;
  const int64_t nv = st.voxels;
  MPL_TRY(mpl_ensure(c, nn.tmp, sizeof(double) * 4 * (n_steps + 64) + 4096));
  double* lossd = P<double>(nn.tmp);
  uint32_t rs = seed * 2654435761u + 12345u;
  for (int it = 0; it < n_steps; ++it) {
    rs = rs * 1664525u + 1013904223u;
    const int k = (int)((rs >> 8) % (uint32_t)st.count);
    MPL_TRY(nn_train_on(c, nn, P<uint16_t>(st.feat) + (int64_t)k * nv * 16,
                        P<float>(st.target) + (int64_t)k * nv * 3, P<float>(st.mask) + (int64_t)k * nv,
                        lr, lossd + 4 * it));
  }
  if (losses && n_steps > 0) {
    std::vector<double> h(4 * n_steps);
    MPL_HIP(c, hipMemcpyAsync(h.data(), lossd, sizeof(double) * 4 * n_steps, hipMemcpyDeviceToHost, c->stream));
    MPL_HIP(c, hipStreamSynchronize(c->stream));
    for (int i = 0; i < n_steps; ++i) losses[i] = (float)h[4 * i + 2];
  }
  return MPL_OK;
}

}  // extern "C"
