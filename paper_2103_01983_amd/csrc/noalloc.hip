// Velocity call that allocates nothing, for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).  The pair kernels' partial sums go to a
// file-scope device array instead of the context's grow-only workspace.
//
// Host code never passes the array's name to a kernel: in host code that
// name is a host-side stand-in, not a device address.  ptrom_create looks
// up the array's device address once per device (hipGetSymbolAddress, with
// the device current) and every launch takes that address.  Each device
// holds its own copy of the array until the process ends; all calls on one
// device share it, so calls that overlap on one device race.
#include <cmath>
#include <mutex>

#include "internal.h"

using namespace ptrom;

namespace {

// 36 MiB: the each-pair-once slots of the tuned launch up to 32768 bodies,
// or the chunk partials of the one-sided launch at any size.
constexpr size_t kScratchFloats = size_t(9) << 20;
static __device__ __align__(256) float scratch[kScratchFloats];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
bool g_done[kMaxDevices];
hipError_t g_err[kMaxDevices];
float *g_ptr[kMaxDevices];  // device address of `scratch` on each device

}  // namespace

namespace ptrom {

hipError_t noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_done[device]) {
    void *p = nullptr;
    g_err[device] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_ptr[device] = g_err[device] == hipSuccess ? static_cast<float *>(p) : nullptr;
    g_done[device] = true;
  }
  return g_err[device];
}

}  // namespace ptrom

extern "C" int ptrom_velocity_noalloc(ptrom_ctx *ctx, int64_t n, const float *xy, const float *gamma,
                                      float delta, float *f, ptrom_stream stream) {
  if (!ctx) return PTROM_EINVAL;
  ctx->err.clear();
  if (n < 1 || n > kMaxN) return ctx->fail(PTROM_EINVAL, "n must be in [1, 2^30]");
  if (!(delta >= 0.0f) || !std::isfinite(delta)) return ctx->fail(PTROM_EINVAL, "delta must be finite and >= 0");
  if (!xy || !gamma || !f) return ctx->fail(PTROM_EINVAL, "NULL array");
  if (ctx->device < 0 || ctx->device >= kMaxDevices)
    return ctx->fail(PTROM_EINVAL, "device index beyond the no-allocation table");
  if (hipSetDevice(ctx->device) != hipSuccess) return ctx->fail(PTROM_EHIP, "hipSetDevice failed");
  float *base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    base = g_ptr[ctx->device];
    if (!base)
      return ctx->fail(PTROM_EHIP, std::string("no-allocation scratch address unavailable: ") +
                                       hipGetErrorString(g_done[ctx->device] ? g_err[ctx->device]
                                                                             : hipErrorNotInitialized));
  }
  // the context's own launch when its workspace fits the scratch (the result
  // is then bitwise that of ptrom_velocity); otherwise the one-sided launch
  // with as many source chunks as fit (one chunk needs no scratch at all)
  PairCfg cfg = ctx->tune.get(OP_VEL, n);
  size_t need = pair_ws_floats(OP_VEL, cfg, ctx->num_cus, n);
  if (need > kScratchFloats) {
    cfg = large_n_cfg();
    const int64_t fit = int64_t(kScratchFloats / (2 * size_t(n)));
    cfg.max_splits = int(fit < 1 ? 1 : (fit > (int64_t(1) << 20) ? (int64_t(1) << 20) : fit));
    need = pair_ws_floats(OP_VEL, cfg, ctx->num_cus, n);
  }
  if (need > kScratchFloats)
    return ctx->fail(PTROM_ENOMEM, "velocity launch needs " + std::to_string(need * sizeof(float)) +
                                       " bytes of scratch, beyond the " +
                                       std::to_string(kScratchFloats * sizeof(float)) + " of the no-allocation call");
  hipError_t e = launch_pair(OP_VEL, cfg, ctx->num_cus, n, xy, gamma, nullptr, delta, f, nullptr, base,
                             kScratchFloats, (hipStream_t)stream);
  if (e != hipSuccess) return ctx->hip_fail(e, "velocity launch (no allocation)");
  return PTROM_OK;
}
