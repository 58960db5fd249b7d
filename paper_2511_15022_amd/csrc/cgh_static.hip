// cgh_create_static: a context whose workspace is a fixed device array of the
// library (one copy per GPU, held while the library is loaded) instead of
// caller memory, for callers that cannot allocate device memory.  Nothing here
// allocates: the array's device address is looked up once per device, the
// host handle is a static slot per device, and one such context may exist per
// device at a time.
#include <mutex>

#include "cgh_internal.h"

namespace {

constexpr size_t kStaticBytes = (size_t)CGH_STATIC_WORKSPACE_BYTES;
constexpr int kMaxDevices = 64;

// the static workspace; host code uses its per-device address from
// hipGetSymbolAddress, never this name
__device__ __align__(256) unsigned char scratch[kStaticBytes];

std::mutex g_mu;
void *g_addr[kMaxDevices];  // device address of scratch on each device (null: not looked up)
bool g_busy[kMaxDevices];   // a static context of that device exists
cgh_ctx g_ctx[kMaxDevices]; // the host handles

}  // namespace

void cgh::release_static(cgh_ctx *ctx) {
  std::lock_guard<std::mutex> lock(g_mu);
  const int dev = ctx->c.static_dev;
  if (dev >= 0 && dev < kMaxDevices && ctx == &g_ctx[dev]) g_busy[dev] = false;
}

extern "C" cgh_status cgh_create_static(const cgh_config *cfg, void *stream, cgh_ctx **out) {
  if (!out) return cgh::report(CGH_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  size_t need = 0;
  cgh_status st = cgh_workspace_size(cfg, &need);
  if (st != CGH_OK) return st;
  if (need > kStaticBytes)
    return cgh::report(CGH_ERR_WORKSPACE,
                       "this configuration needs %zu bytes of workspace; the static workspace "
                       "holds %zu (use cgh_create with a caller workspace)", need, kStaticBytes);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return cgh::report(CGH_ERR_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return cgh::report(CGH_ERR_UNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_busy[dev])
    return cgh::report(CGH_ERR_STATE,
                       "the static workspace of device %d holds another context; cgh_destroy it "
                       "first", dev);
  if (!g_addr[dev]) {
    // once per device, with that device current
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return cgh::report(CGH_ERR_DEVICE, "hipGetSymbolAddress(scratch): %s",
                         hipGetErrorString(e));
    g_addr[dev] = p;
  }
  cgh::Ctx c;
  st = cgh::create_into(cfg, g_addr[dev], kStaticBytes, (hipStream_t)stream, &c);
  if (st != CGH_OK) return st;
  c.static_dev = dev;
  g_ctx[dev].c = c;
  g_busy[dev] = true;
  *out = &g_ctx[dev];
  return CGH_OK;
}
