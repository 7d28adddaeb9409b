// Context life cycle, error handling, buffers, scans and dense <-> block
// conversions.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "mpl_grid.h"
#include "mpl_nn.h"

using namespace mpl;

mpl_status mpl_fail(mpl_ctx* c, mpl_status st, const std::string& msg) {
  if (c) c->last_error = msg;
  return st;
}

mpl_status mpl_hip_check(mpl_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return MPL_OK;
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return mpl_fail(c, e == hipErrorOutOfMemory ? MPL_ERR_OOM : MPL_ERR_HIP, m);
}

mpl_status mpl_dev_alloc(mpl_ctx* c, void** p, size_t bytes) {
  *p = nullptr;
  if (c->allocator.alloc) {
    *p = c->allocator.alloc(c->allocator.user, bytes, (void*)c->stream);
    if (!*p) return mpl_fail(c, MPL_ERR_OOM, "allocator callback failed for " + std::to_string(bytes) + " bytes");
    if (((uintptr_t)*p & 255) != 0) {
      c->allocator.free(c->allocator.user, *p, bytes, (void*)c->stream);
      *p = nullptr;
      return mpl_fail(c, MPL_ERR_OOM, "allocator callback returned memory not aligned to 256 bytes");
    }
    return MPL_OK;
  }
  if (hipMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return mpl_fail(c, MPL_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  return MPL_OK;
}

void mpl_dev_free(mpl_ctx* c, void* p, size_t bytes) {
  if (!p) return;
  if (c->allocator.free) c->allocator.free(c->allocator.user, p, bytes, (void*)c->stream);
  else (void)hipFree(p);
}

mpl_status mpl_ensure(mpl_ctx* c, DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.bytes >= bytes) return MPL_OK;
  if (b.p) {
    MPL_HIP(c, hipStreamSynchronize(c->stream));
    mpl_dev_free(c, b.p, b.bytes);
    b.p = nullptr;
    b.bytes = 0;
  }
  size_t want = bytes + bytes / 8;  // grow with headroom
  MPL_TRY(mpl_dev_alloc(c, &b.p, want));
  b.bytes = want;
  return MPL_OK;
}

mpl_status mpl_sync_scalars(mpl_ctx* c) {
  MPL_HIP(c, hipMemcpyAsync(&c->hscal, c->scal.p, sizeof(SolverScalars), hipMemcpyDeviceToHost,
                            c->stream));
  MPL_HIP(c, hipStreamSynchronize(c->stream));
  return MPL_OK;
}

// ---------------------------------------------------------------- scan
// Three-phase exclusive scan: per-workgroup scan (1024 items) with block sums,
// recursive scan of the block sums, then add the scanned block offsets.
namespace {
constexpr int kScanBlock = 1024;

__global__ void k_scan_local(const int32_t* __restrict__ in, int32_t* __restrict__ out,
                             int32_t* __restrict__ sums, int64_t n) {
  __shared__ int32_t s[kScanBlock];
  int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
  int32_t v = (i < n) ? in[i] : 0;
  s[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    int32_t t = (threadIdx.x >= (unsigned)off) ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  if (i < n) out[i] = s[threadIdx.x] - v;  // exclusive
  if (threadIdx.x == kScanBlock - 1) sums[blockIdx.x] = s[threadIdx.x];
}

__global__ void k_scan_add(int32_t* __restrict__ out, const int32_t* __restrict__ offs, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
  if (i < n) out[i] += offs[blockIdx.x];
}

__global__ void k_scan_total(const int32_t* in, const int32_t* out, int64_t n, int32_t* total) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *total = (n > 0) ? out[n - 1] + in[n - 1] : 0;
}
}  // namespace

mpl_status mpl_scan_i32(mpl_ctx* c, const int32_t* in, int32_t* out, int64_t n, int32_t* total) {
  if (n <= 0) {
    MPL_LAUNCH(c, k_scan_total, 1, 1, in, out, n, total);
    return MPL_OK;
  }
  // Level L scans an array of level_n[L] entries; level 0 is the input,
  // level L+1 the per-1024 block totals of level L.  The top level fits one
  // workgroup.
  std::vector<int64_t> level_n;
  for (int64_t m = n;;) {
    level_n.push_back(m);
    int64_t nb = (m + kScanBlock - 1) / kScanBlock;
    if (nb == 1) break;
    m = nb;
  }
  const size_t T = level_n.size();
  size_t need = 0;
  for (size_t L = 0; L < T; ++L) need += 2 * (size_t)((level_n[L] + kScanBlock - 1) / kScanBlock);
  MPL_TRY(mpl_ensure(c, c->scan_tmp, need * sizeof(int32_t) + 64));
  int32_t* tmp = P<int32_t>(c->scan_tmp);
  std::vector<int32_t*> sums(T), outs(T);
  std::vector<const int32_t*> ins(T);
  size_t off = 0;
  for (size_t L = 0; L < T; ++L) {
    sums[L] = tmp + off;
    off += (level_n[L] + kScanBlock - 1) / kScanBlock;
  }
  for (size_t L = 0; L < T; ++L) {
    ins[L] = (L == 0) ? in : sums[L - 1];
    if (L == 0) {
      outs[L] = out;
    } else {
      outs[L] = tmp + off;
      off += level_n[L];
    }
  }
  for (size_t L = 0; L < T; ++L) {
    int64_t nb = (level_n[L] + kScanBlock - 1) / kScanBlock;
    MPL_LAUNCH(c, k_scan_local, (int)nb, kScanBlock, ins[L], outs[L], sums[L], level_n[L]);
  }
  for (int L = (int)T - 2; L >= 0; --L) {
    int64_t nb = (level_n[L] + kScanBlock - 1) / kScanBlock;
    MPL_LAUNCH(c, k_scan_add, (int)nb, kScanBlock, outs[L], outs[L + 1], level_n[L]);
  }
  MPL_LAUNCH(c, k_scan_total, 1, 1, in, out, n, total);
  return MPL_OK;
}

// ---------------------------------------------------------------- dense I/O
namespace {
template <class T>
__global__ void k_dense_to_block(const T* __restrict__ dense, T* __restrict__ blk,
                                 const int4* __restrict__ ncoord, int comps, int n_nblk,
                                 int nx1, int ny1, int nz1, int64_t nn_block) {
  int b = blockIdx.x, l = threadIdx.x;
  if (b >= n_nblk) return;
  int4 bc = ncoord[b];
  int i = bc.x * 4 + local_x(l), j = bc.y * 4 + local_y(l), k = bc.z * 4 + local_z(l);
  bool in = i < nx1 && j < ny1 && k < nz1;
  int64_t di = ((int64_t)i * ny1 + j) * nz1 + k;
  for (int a = 0; a < comps; ++a)
    blk[(int64_t)a * nn_block + (int64_t)b * MPL_BC + l] = in ? dense[di * comps + a] : T(0);
}
template <class T>
__global__ void k_block_to_dense(const T* __restrict__ blk, T* __restrict__ dense,
                                 const int4* __restrict__ ncoord, int comps, int n_nblk,
                                 int nx1, int ny1, int nz1, int64_t nn_block) {
  int b = blockIdx.x, l = threadIdx.x;
  if (b >= n_nblk) return;
  int4 bc = ncoord[b];
  int i = bc.x * 4 + local_x(l), j = bc.y * 4 + local_y(l), k = bc.z * 4 + local_z(l);
  if (i >= nx1 || j >= ny1 || k >= nz1) return;
  int64_t di = ((int64_t)i * ny1 + j) * nz1 + k;
  for (int a = 0; a < comps; ++a)
    dense[di * comps + a] = blk[(int64_t)a * nn_block + (int64_t)b * MPL_BC + l];
}
__global__ void k_zero_words(uint32_t* __restrict__ a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0u;
}
}  // namespace

mpl_status mpl_dense_to_block_nodes(mpl_ctx* c, const void* dense, void* block, int comps,
                                    int is_f32) {
  int nx1 = c->dims[0] + 1, ny1 = c->dims[1] + 1, nz1 = c->dims[2] + 1;
  if (is_f32)
    MPL_LAUNCH(c, k_dense_to_block<float>, c->n_nblk, MPL_BC, (const float*)dense, (float*)block,
               P<int4>(c->ncoord), comps, c->n_nblk, nx1, ny1, nz1, (int64_t)c->nnode_alloc());
  else
    MPL_LAUNCH(c, k_dense_to_block<double>, c->n_nblk, MPL_BC, (const double*)dense,
               (double*)block, P<int4>(c->ncoord), comps, c->n_nblk, nx1, ny1, nz1,
               (int64_t)c->nnode_alloc());
  return MPL_OK;
}

mpl_status mpl_block_to_dense_nodes(mpl_ctx* c, const void* block, void* dense, int comps,
                                    int is_f32) {
  int nx1 = c->dims[0] + 1, ny1 = c->dims[1] + 1, nz1 = c->dims[2] + 1;
  // cleared by a fill kernel rather than a memset, so that the call can be
  // captured into a HIP graph
  const int64_t words = (int64_t)nx1 * ny1 * nz1 * comps * (is_f32 ? 1 : 2);
  MPL_LAUNCH(c, k_zero_words, (int)((words + 255) / 256), 256, (uint32_t*)dense, words);
  if (is_f32)
    MPL_LAUNCH(c, k_block_to_dense<float>, c->n_nblk, MPL_BC, (const float*)block, (float*)dense,
               P<int4>(c->ncoord), comps, c->n_nblk, nx1, ny1, nz1, (int64_t)c->nnode_alloc());
  else
    MPL_LAUNCH(c, k_block_to_dense<double>, c->n_nblk, MPL_BC, (const double*)block,
               (double*)dense, P<int4>(c->ncoord), comps, c->n_nblk, nx1, ny1, nz1,
               (int64_t)c->nnode_alloc());
  return MPL_OK;
}

// ---------------------------------------------------------------- particle staging
namespace {
__global__ void k_f32_to_f64(const float* __restrict__ a, double* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (double)a[i];
}
__global__ void k_f64_to_f32(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}
// components per particle of x, v, F, G, m, V0, plastic
constexpr int kComps[7] = {3, 3, 9, 9, 1, 1, 1};
}  // namespace

mpl_status mpl_particles_in(mpl_ctx* c, const mpl_particles* p, Parts64* out) {
  if (!p || p->n < 0) return mpl_fail(c, MPL_ERR_INVALID_ARG, "particles");
  out->n = p->n;
  out->mat = p->mat;
  void* const src[7] = {p->x, p->v, p->F, p->G, p->m, p->V0, p->plastic};
  double** dst[7] = {&out->x, &out->v, &out->F, &out->G, &out->m, &out->V0, &out->plastic};
  if (p->dtype == MPL_F64) {
    for (int f = 0; f < 7; ++f) *dst[f] = (double*)src[f];
    return MPL_OK;
  }
  if (p->dtype != MPL_F32) return mpl_fail(c, MPL_ERR_INVALID_ARG, "particle dtype must be MPL_F64 or MPL_F32");
  const int64_t n = p->n;
  MPL_TRY(mpl_ensure(c, c->pstage, 8 * 27 * (size_t)std::max<int64_t>(n, 1)));
  double* base = P<double>(c->pstage);
  int64_t off = 0;
  for (int f = 0; f < 7; ++f) {
    const int64_t cnt = n * kComps[f];
    *dst[f] = nullptr;
    if (src[f]) {
      *dst[f] = base + off;
      MPL_LAUNCH(c, k_f32_to_f64, (int)((cnt + 255) / 256), 256, (const float*)src[f], base + off, cnt);
    }
    off += cnt;
  }
  return MPL_OK;
}

mpl_status mpl_particles_out(mpl_ctx* c, const Parts64* staged, const mpl_particles* p) {
  const int64_t n = staged->n;
  const double* from[5] = {staged->x, staged->v, staged->F, staged->G, staged->plastic};
  void* const to[5] = {p->x, p->v, p->F, p->G, p->plastic};
  const int comps[5] = {3, 3, 9, 9, 1};
  for (int f = 0; f < 5; ++f) {
    if (!from[f] || !to[f]) continue;
    const int64_t cnt = n * comps[f];
    MPL_LAUNCH(c, k_f64_to_f32, (int)((cnt + 255) / 256), 256, from[f], (float*)to[f], cnt);
  }
  return MPL_OK;
}

// ---------------------------------------------------------------- life cycle
static void free_buf(mpl_ctx* c, DevBuf& b) {
  mpl_dev_free(c, b.p, b.bytes);
  b.p = nullptr;
  b.bytes = 0;
}

static mpl_status derive_materials(mpl_ctx* c, const mpl_material* mats, int n) {
  for (int k = 0; k < n; ++k) {
    const mpl_material& m = mats[k];
    if (m.model < 0 || m.model > 3 || m.plastic < 0 || m.plastic > 2)
      return mpl_fail(c, MPL_ERR_INVALID_ARG, "unknown material model or plasticity kind");
    const bool water = m.model == MPL_WATER;
    if (!(m.E > 0.0) || (!water && !(m.nu > -1.0 && m.nu < 0.5)))
      return mpl_fail(c, MPL_ERR_INVALID_ARG, "material needs E > 0 and -1 < nu < 0.5");
    if (water && m.plastic != MPL_PLASTIC_NONE)
      return mpl_fail(c, MPL_ERR_INVALID_ARG, "water takes no plasticity");
    c->mats_in[k] = m;
    MatParams& p = c->mats[k];
    p.model = m.model;
    p.plastic = m.plastic;
    p.mu = m.E / (2.0 * (1.0 + m.nu));
    p.lambda = m.E * m.nu / ((1.0 + m.nu) * (1.0 - 2.0 * m.nu));
    p.kappa = 2.0 * p.mu / 3.0 + p.lambda;
    if (water) {  // E is the bulk modulus of the J-based fluid
      p.mu = p.lambda = 0.0;
      p.kappa = m.E;
    }
    p.yield_stress = m.yield_stress;
    double sphi = std::sin(m.friction_deg * M_PI / 180.0);
    p.alpha_f = std::sqrt(2.0 / 3.0) * 2.0 * sphi / (3.0 - sphi);
  }
  c->nmat = n;
  return MPL_OK;
}

static mpl_status check_opts(mpl_ctx* c, const mpl_solver_opts* o) {
  if (o->hv_precision != MPL_F32 && o->hv_precision != MPL_F64)
    return mpl_fail(c, MPL_ERR_INVALID_ARG, "hv_precision must be MPL_F32 or MPL_F64");
  if (o->precond != MPL_PRECOND_JACOBI && o->precond != MPL_PRECOND_BLOCK_JACOBI &&
      o->precond != MPL_PRECOND_LEARNED && o->precond != MPL_PRECOND_MULTIGRID)
    return mpl_fail(c, MPL_ERR_INVALID_ARG, "unknown preconditioner");
  if (o->mg_levels < 0 || o->mg_levels == 1 || o->mg_levels > MPL_MG_MAX_LEVELS || o->mg_smooth < 0 ||
      o->mg_smooth > 8 || o->mg_coarse_sweeps < 0 || o->mg_coarse_sweeps > 64 ||
      !(o->mg_omega >= 0.0 && o->mg_omega < 2.0))
    return mpl_fail(c, MPL_ERR_INVALID_ARG, "multigrid options out of range");
  if (o->precond == MPL_PRECOND_BLOCK_JACOBI && !c->cg_single)
    return mpl_fail(c, MPL_ERR_INVALID_ARG, "block-Jacobi runs in the single-reduction CG only");
  if (o->time_kernels < 0 || o->time_kernels > 2)
    return mpl_fail(c, MPL_ERR_INVALID_ARG, "time_kernels must be 0, 1 or 2");
  if (o->warm_start < 0 || o->warm_start > 4)
    return mpl_fail(c, MPL_ERR_INVALID_ARG, "warm_start must be 0, 1, 2, 3 or 4");
  if (o->transfer != MPL_TRANSFER_APIC && o->transfer != MPL_TRANSFER_FLIP_PIC)
    return mpl_fail(c, MPL_ERR_INVALID_ARG, "transfer must be MPL_TRANSFER_APIC or MPL_TRANSFER_FLIP_PIC");
  if (!(o->flip_ratio >= 0.0 && o->flip_ratio <= 1.0))
    return mpl_fail(c, MPL_ERR_INVALID_ARG, "flip_ratio must lie in [0, 1]");
  if (o->plasticity != MPL_PLASTICITY_AFTER_SOLVE && o->plasticity != MPL_PLASTICITY_FIXED_POINT)
    return mpl_fail(c, MPL_ERR_INVALID_ARG, "plasticity must be MPL_PLASTICITY_AFTER_SOLVE or _FIXED_POINT");
  if (o->vbd_sweeps < 0 || (o->vbd_sweeps > 0 && o->plasticity == MPL_PLASTICITY_FIXED_POINT))
    return mpl_fail(c, MPL_ERR_INVALID_ARG, "vbd_sweeps must be >= 0 and is not combined with fixed-point plasticity");
  if (o->plastic_anderson < 0 || o->plastic_anderson > 4)
    return mpl_fail(c, MPL_ERR_INVALID_ARG, "plastic_anderson must lie in 0..4");
  if (!(o->newton_forcing >= 0.0 && o->newton_forcing < 1.0))
    return mpl_fail(c, MPL_ERR_INVALID_ARG, "newton_forcing must lie in [0, 1)");
  if (!(o->newton_rtol > 0.0) || !(o->pcg_rtol > 0.0) || o->max_newton < 0 || o->max_pcg < 1 ||
      o->max_ls < 0 || !(o->armijo_c >= 0.0 && o->armijo_c < 1.0))
    return mpl_fail(c, MPL_ERR_INVALID_ARG, "solver options out of range");
  c->opts = *o;
  if (c->opts.pcg_check_every <= 0) c->opts.pcg_check_every = 16;
  if (c->opts.mg_levels == 0) c->opts.mg_levels = 4;
  if (c->opts.mg_smooth == 0) c->opts.mg_smooth = 2;
  if (c->opts.mg_coarse_sweeps == 0) c->opts.mg_coarse_sweeps = 4;
  if (c->opts.mg_omega == 0.0) c->opts.mg_omega = 1.6;
  return MPL_OK;
}

extern "C" {

const char* mpl_version(void) { return "mpmlite-mi355x 0.23 (gfx950)"; }

mpl_status mpl_create(const mpl_grid* grid, const mpl_material* mats, int32_t n_mats,
                      const mpl_solver_opts* opts, void* hip_stream, mpl_ctx** out) {
  return mpl_create_with_allocator(grid, mats, n_mats, opts, hip_stream, nullptr, out);
}

mpl_status mpl_create_with_allocator(const mpl_grid* grid, const mpl_material* mats, int32_t n_mats,
                                     const mpl_solver_opts* opts, void* hip_stream,
                                     const mpl_allocator* allocator, mpl_ctx** out) {
  if (!out) return MPL_ERR_INVALID_ARG;
  *out = nullptr;
  if (allocator && (!allocator->alloc || !allocator->free)) return MPL_ERR_INVALID_ARG;
  if (!grid || !mats || !opts || n_mats < 1 || n_mats > MPL_MAX_MATERIALS) return MPL_ERR_INVALID_ARG;
  for (int a = 0; a < 3; ++a)
    if (grid->dims[a] < 4 || grid->dims[a] % 4 != 0 || grid->dims[a] > 4096) return MPL_ERR_INVALID_ARG;
  if (!(grid->dx > 0.0)) return MPL_ERR_INVALID_ARG;
  mpl_ctx* c = new (std::nothrow) mpl_ctx();
  if (!c) return MPL_ERR_OOM;
  for (int a = 0; a < 3; ++a) {
    c->dims[a] = grid->dims[a];
    c->cbd[a] = grid->dims[a] / 4;
    c->nbd[a] = grid->dims[a] / 4 + 1;
    c->origin[a] = grid->origin[a];
  }
  c->dx = grid->dx;
  c->inv_dx = 1.0 / grid->dx;
  c->stream = (hipStream_t)hip_stream;
  if (allocator) c->allocator = *allocator;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return MPL_ERR_HIP;
  }
  mpl_noalloc_attach(c);
  const char* gr = std::getenv("MPL_GRAPHS");
  c->graphs_enabled = gr && gr[0] == '1';
  const char* dt = std::getenv("MPL_DENSE_TANGENT");
  c->factored_enabled = !(dt && dt[0] == '1');
  const char* cgc = std::getenv("MPL_CG_CLASSIC");
  c->cg_single = !(cgc && cgc[0] == '1');
  mpl_status st = derive_materials(c, mats, n_mats);
  if (st == MPL_OK) st = check_opts(c, opts);
  if (st == MPL_OK) st = mpl_ensure(c, c->scal, sizeof(SolverScalars));
  // the context's own device copy of its materials (kernels take its address)
  if (st == MPL_OK) st = mpl_ensure(c, c->matbuf, sizeof(MatParams) * MPL_MAX_MATERIALS);
  if (st == MPL_OK && (hipMemcpyAsync(c->matbuf.p, c->mats, sizeof(MatParams) * MPL_MAX_MATERIALS,
                                      hipMemcpyHostToDevice, c->stream) != hipSuccess ||
                       hipStreamSynchronize(c->stream) != hipSuccess))
    st = MPL_ERR_HIP;
  if (st == MPL_OK && hipEventCreate(&c->ev[0]) != hipSuccess) st = MPL_ERR_HIP;
  if (st == MPL_OK && hipEventCreate(&c->ev[1]) != hipSuccess) st = MPL_ERR_HIP;
  if (st != MPL_OK) {
    mpl_destroy(c);
    return st;
  }
  *out = c;
  return MPL_OK;
}

void mpl_destroy(mpl_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  DevBuf* all[] = {&c->cflag, &c->cmap, &c->nflag, &c->nmap, &c->scan_tmp, &c->ccoord, &c->ncoord,
                   &c->c_nbr_node, &c->n_nbr_cell, &c->pcell, &c->pkey,
                   &c->bin_count, &c->bin_start, &c->bin_fill, &c->sorted, &c->mc, &c->qc, &c->Gc,
                   &c->Vk, &c->Tk, &c->Sk, &c->Qc, &c->ecell, &c->Abar32, &c->Abar64, &c->Y32,
                   &c->Y64, &c->vcl, &c->Gcl, &c->dvcl, &c->bcbuf, &c->cntbuf, &c->Seff, &c->matbuf, &c->mi, &c->vn, &c->vhat, &c->flags, &c->v, &c->g,
                   &c->vt, &c->dir, &c->r, &c->x, &c->p32, &c->p64, &c->q32, &c->q64, &c->z,
                   &c->D, &c->Bj, &c->Bjt, &c->Aoff, &c->partials, &c->dense_tmp32, &c->dense_tmp64, &c->scal, &c->xstar, &c->ozt, &c->ohz,
                   &c->ogr, &c->cmask, &c->ccnt, &c->coff, &c->Dt, &c->mt, &c->opieces,
                   &c->cg_u, &c->cg_s, &c->cg_dx, &c->cg_red, &c->p2c_halo, &c->pstage, &c->cfmt, &c->fcnt, &c->aa_tmp, &c->aa_part, &c->wtmp, &c->warm_x0, &c->gal_w,
                   &c->gal_u, &c->gal_y,
                   &c->gal_part};
  for (DevBuf* b : all) free_buf(c, *b);
  nn_destroy(c);
  mpl_mg_destroy(c);
  for (GraphCache& gc : c->pcg_cache) {
    if (gc.exec) (void)hipGraphExecDestroy(gc.exec);
    if (gc.graph) (void)hipGraphDestroy(gc.graph);
  }
  for (int i = 0; i < 2; ++i)
    if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
  for (auto& ring : c->whist)
    for (DevBuf& b : ring) free_buf(c, b);
  for (DevBuf& b : c->aa_v) free_buf(c, b);
  for (DevBuf& b : c->aa_f) free_buf(c, b);
  for (hipEvent_t e : c->hv_events) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->up_events) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->cap_order)
    if (e) (void)hipEventDestroy(e);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
}

const char* mpl_last_error(const mpl_ctx* c) { return c ? c->last_error.c_str() : "null context"; }

mpl_status mpl_set_opts(mpl_ctx* c, const mpl_solver_opts* o) {
  if (!c || !o) return MPL_ERR_INVALID_ARG;
  const int warm_before = c->opts.warm_start;
  MPL_TRY(check_opts(c, o));
  // a change of warm-start mode starts the CG start histories afresh
  if (c->opts.warm_start != warm_before)
    for (int j = 0; j < mpl_ctx::kWarm; ++j) c->wcount[j] = c->whead[j] = 0;
  return MPL_OK;
}

}  // extern "C"
