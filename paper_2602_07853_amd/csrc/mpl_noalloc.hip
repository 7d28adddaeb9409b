// Allocation-free Hessian-vector product (mpl_hv_noalloc).
//
// mpl_hv keeps its block-layout copies of u and Hu and the product's
// per-cell pieces in buffers of the context, grown with hipMalloc on first
// use.  Callers that cannot allocate (code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc) use this variant instead:
// the same kernels, with those three buffers carved from one fixed device
// array per GPU, `scratch`, which lives until the process ends.
//
// `scratch` is a device symbol: in host code its name is not a device
// address.  mpl_create (through mpl_noalloc_attach) asks the runtime for the
// array's address on the context's device once per device and keeps it;
// only that address is passed to kernels.
#include <mutex>

#include "mpl_internal.h"

namespace {

constexpr int64_t kScratchBytes = MPL_HV_NOALLOC_MAX_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
hipError_t g_err[kMaxDevices] = {};
bool g_tried[kMaxDevices] = {};

int64_t align256(int64_t n) { return (n + 255) / 256 * 256; }

}  // namespace

void mpl_noalloc_attach(mpl_ctx* c) {
  const int dev = c->device;
  if (dev < 0 || dev >= kMaxDevices) return;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_tried[dev]) return;
  g_tried[dev] = true;
  void* p = nullptr;
  // the caller's device is current (mpl_create runs on it)
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  g_err[dev] = e;
  if (e == hipSuccess) g_ptr[dev] = p;
  else (void)hipGetLastError();
}

extern "C" mpl_status mpl_hv_noalloc(mpl_ctx* c, const void* u, void* Hu, int32_t precision) {
  if (!c || !u || !Hu) return MPL_ERR_INVALID_ARG;
  if (precision != MPL_F32 && precision != MPL_F64) return mpl_fail(c, MPL_ERR_INVALID_ARG, "precision");
  if (!c->tangent_built || c->tangent_precision != precision)
    return mpl_fail(c, MPL_ERR_STATE, "mpl_hv_noalloc needs a tangent built in the same precision");
  int cur = -1;
  MPL_HIP(c, hipGetDevice(&cur));
  if (cur != c->device) return mpl_fail(c, MPL_ERR_INVALID_ARG, "the context's device is not current");
  void* base = nullptr;
  hipError_t err = hipSuccess;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (c->device >= 0 && c->device < kMaxDevices) {
      base = g_ptr[c->device];
      err = g_err[c->device];
    }
  }
  if (!base)
    return mpl_fail(c, MPL_ERR_HIP, std::string("no scratch address for this device: ") +
                                        (err != hipSuccess ? hipGetErrorString(err) : "not attached"));
  const int64_t es = precision == MPL_F32 ? 4 : 8;
  const int64_t vec = align256(3 * (int64_t)c->nnode_alloc() * es);
  const int64_t pcs = align256(6 * (int64_t)c->ncell_alloc() * es);
  const int64_t need = 2 * vec + pcs;
  if (need > kScratchBytes)
    return mpl_fail(c, MPL_ERR_INVALID_ARG,
                    "mpl_hv_noalloc needs " + std::to_string(need) + " bytes of scratch for this grid; its fixed array holds " +
                        std::to_string(kScratchBytes) + " (use mpl_hv)");
  unsigned char* s = (unsigned char*)base;
  void* ub = s;
  void* hb = s + vec;
  void* pieces = s + 2 * vec;
  const int f32 = precision == MPL_F32;
  // no HIP events: they are created on first use
  const int saved_tk = c->opts.time_kernels;
  c->opts.time_kernels = 0;
  mpl_status st = mpl_dense_to_block_nodes(c, u, ub, 3, f32);
  if (st == MPL_OK) st = mpl_mask_free_nodes(c, ub, f32);
  if (st == MPL_OK) st = mpl_stage_hv_into(c, ub, hb, pieces, precision);
  if (st == MPL_OK) st = mpl_block_to_dense_nodes(c, hb, Hu, 3, f32);
  c->opts.time_kernels = saved_tk;
  return st;
}
