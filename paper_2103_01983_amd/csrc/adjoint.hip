// Discrete adjoint of the classic RK4 map with step checkpointing.
//
// Forward: RK4 steps (the captured single-step graph), storing the state at
// every `every`-th step.  Backward: segments are processed last to first;
// each segment's stage inputs s1..s4 are recomputed from its checkpoint and
// kept in HBM (every x 4 x 2N floats), then its steps are reversed:
//   kap4 = h/6 lam,               a4 = J(s4)^T kap4
//   kap3 = h/3 lam + h a4,        a3 = J(s3)^T kap3
//   kap2 = h/3 lam + h/2 a3,      a2 = J(s2)^T kap2
//   kap1 = h/6 lam + h/2 a2,      a1 = J(s1)^T kap1
//   lam += a1 + a2 + a3 + a4,     gGamma += sum_s d(kap_s . f(s_s))/dGamma
// (chain rule through y = x + h/6 (k1 + 2k2 + 2k3 + k4)).  Each J^T kap and
// its circulation partial is one vector-Jacobian pair kernel; lam and
// gGamma are accumulated with Kahan compensation across the 4*nsteps terms.
#include <algorithm>

#include "internal.h"

using namespace ptrom;

namespace {

inline dim3 g1(int64_t m) { return dim3((unsigned)((m + 255) / 256)); }

__global__ void copy_kernel(int64_t m, float *__restrict__ out, const float *__restrict__ x) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < m) out[q] = x[q];
}

__global__ void fill_kernel(int64_t m, float *__restrict__ out, float v) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < m) out[q] = v;
}

// kap = a * lam + b * y   (y may be null)
__global__ void kappa_kernel(int64_t m, float *__restrict__ kap, float a, const float *__restrict__ lam,
                             float b, const float *__restrict__ y) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < m) kap[q] = y ? fmaf(b, y[q], a * lam[q]) : a * lam[q];
}

// lam += a1 + a2 + a3 + a4, compensated
__global__ void lam_update_kernel(int64_t m, float *__restrict__ lam, float *__restrict__ comp,
                                  const float *__restrict__ a1, const float *__restrict__ a2,
                                  const float *__restrict__ a3, const float *__restrict__ a4) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  const float x = (a1[q] + a2[q]) + (a3[q] + a4[q]);
  const float y = x - comp[q];
  const float t = lam[q] + y;
  comp[q] = (t - lam[q]) - y;
  lam[q] = t;
}

// acc += x, compensated
__global__ void kahan_accum_kernel(int64_t m, float *__restrict__ acc, float *__restrict__ comp,
                                   const float *__restrict__ x) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  const float y = x[q] - comp[q];
  const float t = acc[q] + y;
  comp[q] = (t - acc[q]) - y;
  acc[q] = t;
}

int validate(ptrom_ctx *ctx, int64_t n, float delta, float dt, int nsteps, int every) {
  if (!ctx) return PTROM_EINVAL;
  ctx->err.clear();
  if (n < 1 || n > kMaxN) return ctx->fail(PTROM_EINVAL, "n must be in [1, 2^30]");
  if (!(delta >= 0.0f) || !(dt > 0.0f) || nsteps < 0 || every < 1)
    return ctx->fail(PTROM_EINVAL, "need delta >= 0, dt > 0, nsteps >= 0, every >= 1");
  if (hipSetDevice(ctx->device) != hipSuccess) return ctx->fail(PTROM_EHIP, "hipSetDevice");
  return PTROM_OK;
}

}  // namespace

extern "C" int ptrom_rk4_fwd_ckpt(ptrom_ctx *ctx, int64_t n, const float *xy0, const float *gamma,
                                  float delta, float dt, int nsteps, int every, float *ckpt,
                                  float *xyT, ptrom_stream stream) {
  if (int rc = validate(ctx, n, delta, dt, nsteps, every)) return rc;
  if (!xy0 || !gamma || !xyT || (nsteps > 0 && !ckpt)) return ctx->fail(PTROM_EINVAL, "NULL array");
  const int64_t m = 2 * n;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(copy_kernel, g1(m), dim3(256), 0, st, m, xyT, xy0);
  for (int t0 = 0; t0 < nsteps; t0 += every) {
    hipLaunchKernelGGL(copy_kernel, g1(m), dim3(256), 0, st, m, ckpt + (size_t)(t0 / every) * m, xyT);
    const int len = std::min(every, nsteps - t0);
    if (int rc = ptrom_rk4(ctx, n, xyT, gamma, delta, dt, len, stream)) return rc;
  }
  PTROM_CHECK_HIP(ctx, hipGetLastError());
  return PTROM_OK;
}

extern "C" int ptrom_rk4_bwd(ptrom_ctx *ctx, int64_t n, const float *ckpt, const float *gamma,
                             float delta, float dt, int nsteps, int every, const float *lamT,
                             const float *ggamma_direct, float *lam0, float *ggamma,
                             ptrom_stream stream) {
  if (int rc = validate(ctx, n, delta, dt, nsteps, every)) return rc;
  if (!gamma || !lamT || !lam0 || !ggamma || (nsteps > 0 && !ckpt)) return ctx->fail(PTROM_EINVAL, "NULL array");
  const int64_t m = 2 * n;
  const int seg_len = std::min(every, std::max(nsteps, 1));
  const PairCfg vcfg = ctx->tune.get(OP_VEL, n), acfg = ctx->tune.get(OP_VJP, n);
  const size_t pwsf = std::max(pair_ws_floats(OP_VEL, vcfg, ctx->num_cus, n),
                               pair_ws_floats(OP_VJP, acfg, ctx->num_cus, n));
  const size_t vb = align256(m * sizeof(float)), nbq = align256(n * sizeof(float));
  const size_t need = vb * (size_t(4) * seg_len + 4 + 1 + 4 + 1) + 3 * nbq + align256(pwsf * sizeof(float)) + 1024;
  if (int rc = ctx->reserve(need)) return rc;
  Carver cv{static_cast<char *>(ctx->ws), ctx->ws_bytes};
  float *S = cv.take<float>(size_t(4) * seg_len * m);
  float *k[4];
  for (int q = 0; q < 4; ++q) k[q] = cv.take<float>(m);
  float *kap = cv.take<float>(m);
  float *a[4];
  for (int q = 0; q < 4; ++q) a[q] = cv.take<float>(m);
  float *lamc = cv.take<float>(m);
  float *gp = cv.take<float>(n), *ggc = cv.take<float>(n);
  float *pws = cv.take<float>(pwsf ? pwsf : 1);
  if (!S || !lamc || !ggc || !pws) return ctx->fail(PTROM_ENOMEM, "workspace carve");
  hipStream_t st = (hipStream_t)stream;
  const float h = dt;

  hipLaunchKernelGGL(copy_kernel, g1(m), dim3(256), 0, st, m, lam0, lamT);
  hipLaunchKernelGGL(fill_kernel, g1(m), dim3(256), 0, st, m, lamc, 0.0f);
  if (ggamma_direct)
    hipLaunchKernelGGL(copy_kernel, g1(n), dim3(256), 0, st, n, ggamma, ggamma_direct);
  else
    hipLaunchKernelGGL(fill_kernel, g1(n), dim3(256), 0, st, n, ggamma, 0.0f);
  hipLaunchKernelGGL(fill_kernel, g1(n), dim3(256), 0, st, n, ggc, 0.0f);

  auto vel = [&](const float *x, float *out) -> int {
    hipError_t e = launch_pair(OP_VEL, vcfg, ctx->num_cus, n, x, gamma, nullptr, delta, out, nullptr, pws, pwsf, st);
    return e == hipSuccess ? PTROM_OK : ctx->hip_fail(e, "velocity");
  };
  auto vjp = [&](const float *x, const float *w, float *out) -> int {
    hipError_t e = launch_pair(OP_VJP, acfg, ctx->num_cus, n, x, gamma, w, delta, out, gp, pws, pwsf, st);
    if (e != hipSuccess) return ctx->hip_fail(e, "vjp");
    hipLaunchKernelGGL(kahan_accum_kernel, g1(n), dim3(256), 0, st, n, ggamma, ggc, gp);
    return PTROM_OK;
  };

  const int nseg = (nsteps + every - 1) / every;
  for (int seg = nseg - 1; seg >= 0; --seg) {
    const int t0 = seg * every;
    const int len = std::min(every, nsteps - t0);
    // recompute the stage inputs of the segment
    hipLaunchKernelGGL(copy_kernel, g1(m), dim3(256), 0, st, m, S, ckpt + (size_t)seg * m);
    for (int s = 0; s < len; ++s) {
      float *s0 = S + (size_t)(4 * s) * m;
      float *sq[4] = {s0, s0 + m, s0 + 2 * m, s0 + 3 * m};
      // k4 only feeds the next step's start, so the segment's last step
      // skips it
      const int nk = s + 1 < len ? 4 : 3;
      for (int q = 0; q < nk; ++q) {
        if (int rc = vel(sq[q], k[q])) return rc;
        if (q < 3) PTROM_CHECK_HIP(ctx, launch_axpy(m, sq[q + 1], s0, (q < 2 ? 0.5f : 1.0f) * h, k[q], st));
      }
      if (s + 1 < len) {
        float *next = S + (size_t)(4 * (s + 1)) * m;
        hipLaunchKernelGGL(copy_kernel, g1(m), dim3(256), 0, st, m, next, s0);
        PTROM_CHECK_HIP(ctx, launch_rk4_combine(m, next, k[0], k[1], k[2], k[3], h, st));
      }
    }
    // reverse the segment's steps
    for (int s = len - 1; s >= 0; --s) {
      float *s0 = S + (size_t)(4 * s) * m;
      hipLaunchKernelGGL(kappa_kernel, g1(m), dim3(256), 0, st, m, kap, h / 6.0f, lam0, 0.0f, nullptr);
      if (int rc = vjp(s0 + 3 * m, kap, a[3])) return rc;
      hipLaunchKernelGGL(kappa_kernel, g1(m), dim3(256), 0, st, m, kap, h / 3.0f, lam0, h, a[3]);
      if (int rc = vjp(s0 + 2 * m, kap, a[2])) return rc;
      hipLaunchKernelGGL(kappa_kernel, g1(m), dim3(256), 0, st, m, kap, h / 3.0f, lam0, 0.5f * h, a[2]);
      if (int rc = vjp(s0 + m, kap, a[1])) return rc;
      hipLaunchKernelGGL(kappa_kernel, g1(m), dim3(256), 0, st, m, kap, h / 6.0f, lam0, 0.5f * h, a[1]);
      if (int rc = vjp(s0, kap, a[0])) return rc;
      hipLaunchKernelGGL(lam_update_kernel, g1(m), dim3(256), 0, st, m, lam0, lamc, a[0], a[1], a[2], a[3]);
    }
  }
  PTROM_CHECK_HIP(ctx, hipGetLastError());
  return PTROM_OK;
}
