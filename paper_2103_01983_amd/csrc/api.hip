// Context management, argument validation and the host drivers of the pair
// sums and the single-system time steppers (RK4 via a captured HIP graph;
// implicit k=1 schemes via Newton-GMRES over the Jacobian-product kernel).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>

#include "internal.h"

using namespace ptrom;

int ptrom_ctx::reserve(size_t bytes) {
  if (bytes <= ws_bytes) return PTROM_OK;
  if (ws) {
    hipError_t e = hipFree(ws);  // waits for work that may still use it
    ws = nullptr;
    ws_bytes = 0;
    if (e != hipSuccess) return hip_fail(e, "hipFree(workspace)");
  }
  // captured graphs hold workspace addresses
  for (auto &g : graphs) hipGraphExecDestroy(g.exec);
  graphs.clear();
  size_t want = std::max(bytes, size_t(1) << 20);
  hipError_t e = hipMalloc(&ws, want);
  if (e != hipSuccess) {
    ws = nullptr;
    return fail(PTROM_ENOMEM, std::string("workspace hipMalloc(") + std::to_string(want) +
                                  "): " + hipGetErrorString(e));
  }
  ws_bytes = want;
  return PTROM_OK;
}

extern "C" int ptrom_version(void) { return 10000; }

extern "C" int ptrom_create(ptrom_ctx **out, int device) {
  if (!out) return PTROM_EINVAL;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return PTROM_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return PTROM_EHIP;
  ptrom_ctx *c = new ptrom_ctx();
  c->device = device;
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, device) == hipSuccess) {
    c->num_cus = p.multiProcessorCount;
    if (p.totalGlobalMem) c->tune.ws_cap_bytes = uint64_t(p.totalGlobalMem) / kWsCapDivisor;
  }
  if (hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return PTROM_EHIP;
  }
  // the allocation-free velocity call's scratch address on this device
  // (kept per device; a failure is reported by that call)
  (void)noalloc_init(device);
  const char *cache = std::getenv("PTROM_TUNE_CACHE");
  if (cache && *cache) ptrom_load_tuning(c, cache);
  c->err.clear();
  *out = c;
  return PTROM_OK;
}

extern "C" void ptrom_destroy(ptrom_ctx *ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->device);
  hipDeviceSynchronize();
  for (auto &g : ctx->graphs) hipGraphExecDestroy(g.exec);
  if (ctx->ws) hipFree(ctx->ws);
  if (ctx->capture_stream) hipStreamDestroy(ctx->capture_stream);
  if (ctx->pinned) hipHostFree(ctx->pinned);
  delete ctx;
}

extern "C" const char *ptrom_last_error(const ptrom_ctx *ctx) { return ctx ? ctx->err.c_str() : ""; }

static int check_common(ptrom_ctx *ctx, int64_t n, double delta) {
  if (!ctx) return PTROM_EINVAL;
  ctx->err.clear();
  if (n < 1 || n > kMaxN) return ctx->fail(PTROM_EINVAL, "n must be in [1, 2^30]");
  if (!(delta >= 0.0) || !std::isfinite(delta)) return ctx->fail(PTROM_EINVAL, "delta must be finite and >= 0");
  if (hipSetDevice(ctx->device) != hipSuccess) return ctx->fail(PTROM_EHIP, "hipSetDevice failed");
  return PTROM_OK;
}

static int run_pair(ptrom_ctx *ctx, int op, int64_t n, const float *xy, const float *gamma,
                    const float *aux, float delta, float *out, float *out2, hipStream_t st) {
  const PairCfg cfg = ctx->tune.get(op, n);
  const size_t wsf = pair_ws_floats(op, cfg, ctx->num_cus, n);
  if (int rc = ctx->reserve(wsf * sizeof(float))) return rc;
  hipError_t e = launch_pair(op, cfg, ctx->num_cus, n, xy, gamma, aux, delta, out, out2,
                             static_cast<float *>(ctx->ws), ctx->ws_bytes / sizeof(float), st);
  if (e != hipSuccess) return ctx->hip_fail(e, "pair kernel launch");
  return PTROM_OK;
}

extern "C" int ptrom_velocity(ptrom_ctx *ctx, int64_t n, const float *xy, const float *gamma,
                              float delta, float *f, ptrom_stream stream) {
  if (int rc = check_common(ctx, n, delta)) return rc;
  if (!xy || !gamma || !f) return ctx->fail(PTROM_EINVAL, "NULL array");
  return run_pair(ctx, OP_VEL, n, xy, gamma, nullptr, delta, f, nullptr, (hipStream_t)stream);
}

extern "C" int ptrom_velocity_f64(ptrom_ctx *ctx, int64_t n, const double *xy, const double *gamma,
                                  double delta, double *f, ptrom_stream stream) {
  if (int rc = check_common(ctx, n, delta)) return rc;
  if (!xy || !gamma || !f) return ctx->fail(PTROM_EINVAL, "NULL array");
  hipError_t e = launch_velocity_f64(n, xy, gamma, delta, f, (hipStream_t)stream);
  if (e != hipSuccess) return ctx->hip_fail(e, "velocity_f64 launch");
  return PTROM_OK;
}

extern "C" int ptrom_jvp(ptrom_ctx *ctx, int64_t n, const float *xy, const float *gamma, float delta,
                         const float *v, float *jv, ptrom_stream stream) {
  if (int rc = check_common(ctx, n, delta)) return rc;
  if (!xy || !gamma || !v || !jv) return ctx->fail(PTROM_EINVAL, "NULL array");
  return run_pair(ctx, OP_JVP, n, xy, gamma, v, delta, jv, nullptr, (hipStream_t)stream);
}

extern "C" int ptrom_block_jacobian(ptrom_ctx *ctx, int64_t n, const float *xy, const float *gamma,
                                    float delta, float *B, ptrom_stream stream) {
  if (int rc = check_common(ctx, n, delta)) return rc;
  if (!xy || !gamma || !B) return ctx->fail(PTROM_EINVAL, "NULL array");
  return run_pair(ctx, OP_BJAC, n, xy, gamma, nullptr, delta, B, nullptr, (hipStream_t)stream);
}

extern "C" int ptrom_velocity_block_jacobian(ptrom_ctx *ctx, int64_t n, const float *xy, const float *gamma,
                                             float delta, float *f, float *B, ptrom_stream stream) {
  if (int rc = check_common(ctx, n, delta)) return rc;
  if (!xy || !gamma || !f || !B) return ctx->fail(PTROM_EINVAL, "NULL array");
  return run_pair(ctx, OP_VBJ, n, xy, gamma, nullptr, delta, f, B, (hipStream_t)stream);
}

extern "C" int ptrom_vjp(ptrom_ctx *ctx, int64_t n, const float *xy, const float *gamma, float delta,
                         const float *w, float *gxy, float *ggamma, ptrom_stream stream) {
  if (int rc = check_common(ctx, n, delta)) return rc;
  if (!xy || !gamma || !w || !gxy || !ggamma) return ctx->fail(PTROM_EINVAL, "NULL array");
  return run_pair(ctx, OP_VJP, n, xy, gamma, w, delta, gxy, ggamma, (hipStream_t)stream);
}

extern "C" int ptrom_stream_function(ptrom_ctx *ctx, int64_t n, const float *xy, const float *gamma,
                                     float delta, float *psi, ptrom_stream stream) {
  if (int rc = check_common(ctx, n, delta)) return rc;
  if (!xy || !gamma || !psi) return ctx->fail(PTROM_EINVAL, "NULL array");
  return run_pair(ctx, OP_PSI, n, xy, gamma, nullptr, delta, psi, nullptr, (hipStream_t)stream);
}

namespace {

// H = 1/2 sum_i Gamma_i psi_i in FP64: each workgroup adds a contiguous
// range in a fixed order (tree over its threads), then one workgroup adds
// the partials in workgroup order, so the result is reproducible.
constexpr int kHamBlock = 256;
constexpr int kHamMaxParts = 1024;

__global__ void __launch_bounds__(kHamBlock)
    ham_partial_kernel(int64_t n, const float *__restrict__ gam, const float *__restrict__ psi, int64_t per,
                       double *__restrict__ part) {
  __shared__ double s[kHamBlock];
  const int64_t b0 = int64_t(blockIdx.x) * per;
  const int64_t b1 = b0 + per < n ? b0 + per : n;
  double acc = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += kHamBlock) acc += double(gam[i]) * double(psi[i]);
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kHamBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ void __launch_bounds__(kHamBlock)
    ham_final_kernel(int parts, const double *__restrict__ part, double *__restrict__ H) {
  __shared__ double s[kHamBlock];
  double acc = 0.0;
  for (int q = threadIdx.x; q < parts; q += kHamBlock) acc += part[q];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kHamBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) H[0] = 0.5 * s[0];
}

}  // namespace

extern "C" int ptrom_hamiltonian(ptrom_ctx *ctx, int64_t n, const float *xy, const float *gamma, float delta,
                                 double *H, ptrom_stream stream) {
  if (int rc = check_common(ctx, n, delta)) return rc;
  if (!xy || !gamma || !H) return ctx->fail(PTROM_EINVAL, "NULL array");
  const PairCfg cfg = ctx->tune.get(OP_PSI, n);
  const size_t pwsf = pair_ws_floats(OP_PSI, cfg, ctx->num_cus, n);
  const int parts = int(std::min<int64_t>(kHamMaxParts, (n + kHamBlock - 1) / kHamBlock));
  const int64_t per = (n + parts - 1) / parts;
  if (int rc = ctx->reserve(align256(size_t(n) * sizeof(float)) + align256(parts * sizeof(double)) +
                            align256(pwsf * sizeof(float)) + 256))
    return rc;
  Carver cv{static_cast<char *>(ctx->ws), ctx->ws_bytes};
  float *psi = cv.take<float>(n);
  double *part = cv.take<double>(parts);
  float *pws = cv.take<float>(pwsf ? pwsf : 1);
  if (!psi || !part || !pws) return ctx->fail(PTROM_ENOMEM, "workspace carve");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = launch_pair(OP_PSI, cfg, ctx->num_cus, n, xy, gamma, nullptr, delta, psi, nullptr, pws, pwsf, st);
  if (e != hipSuccess) return ctx->hip_fail(e, "stream function launch");
  hipLaunchKernelGGL(ham_partial_kernel, dim3(parts), dim3(kHamBlock), 0, st, n, gamma, psi, per, part);
  hipLaunchKernelGGL(ham_final_kernel, dim3(1), dim3(kHamBlock), 0, st, parts, part, H);
  PTROM_CHECK_HIP(ctx, hipGetLastError());
  return PTROM_OK;
}

extern "C" int ptrom_velocity_points(ptrom_ctx *ctx, int64_t nt, const float *p, int64_t n, const float *xy,
                                     const float *gamma, float delta, float *f, ptrom_stream stream) {
  if (int rc = check_common(ctx, n, delta)) return rc;
  if (nt < 1 || nt > kMaxN) return ctx->fail(PTROM_EINVAL, "nt must be in [1, 2^30]");
  if (!p || !xy || !gamma || !f) return ctx->fail(PTROM_EINVAL, "NULL array");
  const size_t wsf = points_ws_floats(ctx->num_cus, nt, n);
  if (wsf)
    if (int rc = ctx->reserve(wsf * sizeof(float))) return rc;
  hipError_t e = launch_velocity_points(nt, p, n, xy, gamma, delta, f, static_cast<float *>(ctx->ws),
                                        ctx->ws_bytes / sizeof(float), ctx->num_cus, (hipStream_t)stream);
  if (e != hipSuccess) return ctx->hip_fail(e, "points velocity launch");
  return PTROM_OK;
}

// ---------------------------------------------------------------- RK4

// Records one RK4 step (4 velocity evaluations + stage updates) on `st`.
static int record_rk4_step(ptrom_ctx *ctx, int64_t n, float *xy, const float *gamma, float delta,
                           float dt, float *k[4], float *s, float *pws, size_t pws_floats,
                           hipStream_t st) {
  const PairCfg cfg = ctx->tune.get(OP_VEL, n);
  const int64_t m = 2 * n;
  hipError_t e;
  const float *in = xy;
  for (int q = 0; q < 4; ++q) {
    e = launch_pair(OP_VEL, cfg, ctx->num_cus, n, in, gamma, nullptr, delta, k[q], nullptr, pws,
                    pws_floats, st);
    if (e != hipSuccess) return ctx->hip_fail(e, "rk4 velocity");
    if (q < 3) {
      e = launch_axpy(m, s, xy, (q < 2 ? 0.5f : 1.0f) * dt, k[q], st);
      if (e != hipSuccess) return ctx->hip_fail(e, "rk4 stage");
      in = s;
    }
  }
  e = launch_rk4_combine(m, xy, k[0], k[1], k[2], k[3], dt, st);
  if (e != hipSuccess) return ctx->hip_fail(e, "rk4 combine");
  return PTROM_OK;
}

extern "C" int ptrom_rk4(ptrom_ctx *ctx, int64_t n, float *xy, const float *gamma, float delta,
                         float dt, int nsteps, ptrom_stream stream) {
  if (int rc = check_common(ctx, n, delta)) return rc;
  if (!xy || !gamma) return ctx->fail(PTROM_EINVAL, "NULL array");
  if (!(dt > 0.0f) || nsteps < 0) return ctx->fail(PTROM_EINVAL, "dt must be > 0 and nsteps >= 0");
  if (nsteps == 0) return PTROM_OK;
  const int64_t m = 2 * n;
  const PairCfg cfg = ctx->tune.get(OP_VEL, n);
  const size_t pwsf = pair_ws_floats(OP_VEL, cfg, ctx->num_cus, n);
  const size_t need = 5 * align256(m * sizeof(float)) + align256(pwsf * sizeof(float)) + 256;
  if (int rc = ctx->reserve(need)) return rc;
  Carver cv{static_cast<char *>(ctx->ws), ctx->ws_bytes};
  float *k[4];
  for (int q = 0; q < 4; ++q) k[q] = cv.take<float>(m);
  float *s = cv.take<float>(m);
  float *pws = cv.take<float>(pwsf ? pwsf : 1);
  if (!k[3] || !s || !pws) return ctx->fail(PTROM_ENOMEM, "workspace carve");
  hipStream_t st = (hipStream_t)stream;
  char keybuf[256];
  std::snprintf(keybuf, sizeof keybuf, "rk4:%p:%p:%lld:%a:%a:%p", (void *)xy, (const void *)gamma,
                (long long)n, (double)delta, (double)dt, ctx->ws);
  hipGraphExec_t ex = nullptr;
  if (int rc = ctx->graph_for(
          keybuf,
          [&](hipStream_t cs) { return record_rk4_step(ctx, n, xy, gamma, delta, dt, k, s, pws, pwsf, cs); },
          &ex))
    return rc;
  for (int t = 0; t < nsteps; ++t) PTROM_CHECK_HIP(ctx, hipGraphLaunch(ex, st));
  return PTROM_OK;
}

extern "C" int ptrom_rk4_f64(ptrom_ctx *ctx, int64_t n, double *xy, const double *gamma,
                             double delta, double dt, int nsteps, ptrom_stream stream) {
  if (int rc = check_common(ctx, n, delta)) return rc;
  if (!xy || !gamma) return ctx->fail(PTROM_EINVAL, "NULL array");
  if (!(dt > 0.0) || nsteps < 0) return ctx->fail(PTROM_EINVAL, "dt must be > 0 and nsteps >= 0");
  const int64_t m = 2 * n;
  if (int rc = ctx->reserve(5 * align256(m * sizeof(double)) + 256)) return rc;
  Carver cv{static_cast<char *>(ctx->ws), ctx->ws_bytes};
  double *k[4];
  for (int q = 0; q < 4; ++q) k[q] = cv.take<double>(m);
  double *s = cv.take<double>(m);
  if (!k[3] || !s) return ctx->fail(PTROM_ENOMEM, "workspace carve");
  hipStream_t st = (hipStream_t)stream;
  for (int t = 0; t < nsteps; ++t) {
    const double *in = xy;
    for (int q = 0; q < 4; ++q) {
      PTROM_CHECK_HIP(ctx, launch_velocity_f64(n, in, gamma, delta, k[q], st));
      if (q < 3) {
        PTROM_CHECK_HIP(ctx, launch_axpy_f64(m, s, xy, (q < 2 ? 0.5 : 1.0) * dt, k[q], st));
        in = s;
      }
    }
    PTROM_CHECK_HIP(ctx, launch_rk4_combine_f64(m, xy, k[0], k[1], k[2], k[3], dt, st));
  }
  return PTROM_OK;
}
