// Online projection-tree ROM: HyperPair (Algorithm "HyperPair") and the
// Gauss-Newton loop around it (Algorithm "Gauss-Newton").
//
// Per Gauss-Newton iteration:
//   project   p_c = xqt0_c + Phit_c xhat  for every surrogate source, and
//             xbar = xbar0 + Phibar xhat  for the sampled rows (FP64);
//   gather    one wave64 per sampled target walks its interaction list
//             (lanes stride over the entries), forms r = xbar_i - p_c in FP64,
//             does the pair arithmetic in FP32 (velocity, the 2x2 self block
//             B_i, and in the exact mode sum_c G_ic Phit_c), reduces across the
//             wave with shuffles, and writes the trapezoid residual rows
//             rbar = xbar - xbar_prev - dt/2 (fbar + fbar_prev) and the rows of
//             C = (I - dt/2 dfbar/dx) Phibar in FP64;
//   solve     G = A C, b = A rbar (FP64), the relative reduced gradient
//             |G^T b| / |G_1^T b_1|, Householder QR of G in one wave and
//             xhat -= alpha G^+ b.
// ptrom_rom_run keeps the whole loop (all steps, all iterations) inside one
// workgroup, so a step costs no host round trip; ptrom_rom_hyperpair runs the
// projection and gather over many workgroups (large sample sets).
#include <cmath>
#include <vector>

#include "internal.h"

using namespace ptrom;

namespace {

constexpr int kMaxM = 32;
constexpr int kMaxMr = 64;
constexpr int kMaxNd = 1 << 21;
constexpr int kRunThreads = 1024;
constexpr double kInv2PiD = 0.15915494309189533576888376337251;

struct RomDev {
  int M, Mr, ns, nd, jac_mode, max_iter;
  int64_t Nc, nnz;
  float d2, dt;
  double tol, alpha;
  const float *Phibar, *xbar0, *xqt0, *Phit, *Gt;
  const int *off, *ids;
  const double *A;
  // scratch (device)
  double *pos, *xbar, *xbar_prev, *fbar, *fbar_prev, *rbar, *C, *xh;
};

__device__ __forceinline__ float wsum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wsumd(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// p_c for c in [c0, Nc) step cs and xbar rows for q in [q0, nd) step cs.
__device__ void project(const RomDev &d, const double *xh, int t0, int ts) {
  const int M = d.M;
  for (int64_t c = t0; c < 2 * d.Nc; c += ts) {
    double s = d.xqt0[c];
    const float *ph = d.Phit + c * M;
    for (int m = 0; m < M; ++m) s += (double)ph[m] * xh[m];
    d.pos[c] = s;
  }
  for (int q = t0; q < d.nd; q += ts) {
    double s = d.xbar0[q];
    const float *ph = d.Phibar + (size_t)q * M;
    for (int m = 0; m < M; ++m) s += (double)ph[m] * xh[m];
    d.xbar[q] = s;
  }
}

// HyperPair rows of sampled target i, computed by one whole wave.
template <bool EXACT>
__device__ void gather_target(const RomDev &d, int i, int lane, const double *xbar,
                              const double *xbar_prev, const double *fbar_prev, double *fbar_out,
                              double *rbar_out, double *C_out) {
  const int M = d.M, ns = d.ns;
  const double tx = xbar[i], ty = xbar[ns + i];
  float fx = 0.f, fy = 0.f, ba = 0.f, bb = 0.f, bc = 0.f;
  float ex[EXACT ? kMaxM : 1], ey[EXACT ? kMaxM : 1];
  if constexpr (EXACT) {
    for (int m = 0; m < kMaxM; ++m) ex[m] = ey[m] = 0.f;
  }
  const int e0 = d.off[i], e1 = d.off[i + 1];
  for (int e = e0 + lane; e < e1; e += 64) {
    const int c = d.ids[e];
    const float rx = (float)(tx - d.pos[2 * c]);
    const float ry = (float)(ty - d.pos[2 * c + 1]);
    const float q = fmaf(rx, rx, fmaf(ry, ry, d.d2));
    const float r = 1.0f / q;
    const float g = d.Gt[c] * r;
    fx = fmaf(-ry, g, fx);
    fy = fmaf(rx, g, fy);
    const float g2 = g * r;
    const float a2 = (rx + rx) * ry;
    const float dd = fmaf(ry, ry, -rx * rx);
    ba = fmaf(g2, a2, ba);
    bb = fmaf(g2, dd - d.d2, bb);
    bc = fmaf(g2, dd + d.d2, bc);
    if constexpr (EXACT) {
      const float *phx = d.Phit + (size_t)(2 * c) * M;
      const float *phy = phx + M;
      for (int m = 0; m < M; ++m) {
        ex[m] = fmaf(g2, fmaf(a2, phx[m], (dd - d.d2) * phy[m]), ex[m]);
        ey[m] = fmaf(g2, fmaf(dd + d.d2, phx[m], -a2 * phy[m]), ey[m]);
      }
    }
  }
  const double Fx = wsum(fx) * kInv2PiD, Fy = wsum(fy) * kInv2PiD;
  const double B00 = wsum(ba) * kInv2PiD, B01 = wsum(bb) * kInv2PiD, B10 = wsum(bc) * kInv2PiD;
  const double B11 = -B00;
  const double hdt = 0.5 * (double)d.dt;
  if (lane == 0) {
    if (fbar_out) {
      fbar_out[i] = Fx;
      fbar_out[ns + i] = Fy;
    }
    if (rbar_out) {
      rbar_out[i] = (tx - xbar_prev[i]) - hdt * (Fx + fbar_prev[i]);
      rbar_out[ns + i] = (ty - xbar_prev[ns + i]) - hdt * (Fy + fbar_prev[ns + i]);
    }
  }
  if (C_out) {
    for (int m = 0; m < M; ++m) {
      double e0v = 0.0, e1v = 0.0;
      if constexpr (EXACT) {
        e0v = wsum(ex[m]) * kInv2PiD;
        e1v = wsum(ey[m]) * kInv2PiD;
      }
      if (lane == m) {
        const double px = d.Phibar[(size_t)i * M + m], py = d.Phibar[(size_t)(ns + i) * M + m];
        C_out[(size_t)i * M + m] = px - hdt * (B00 * px + B01 * py - e0v);
        C_out[(size_t)(ns + i) * M + m] = py - hdt * (B10 * px + B11 * py - e1v);
      }
    }
  }
}

// ----------------------------------------------------------- hyperpair hook

__global__ void project_kernel(RomDev d, const double *__restrict__ xh) {
  project(d, xh, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

template <bool EXACT>
__global__ void __launch_bounds__(256)
    gather_kernel(RomDev d, const double *__restrict__ xbar_prev, const double *__restrict__ fbar_prev,
                  double *fbar, double *rbar, double *C) {
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (wave >= d.ns) return;
  gather_target<EXACT>(d, wave, lane, d.xbar, xbar_prev, fbar_prev, fbar, rbar, C);
}

// ----------------------------------------------------------- device-resident loop

template <bool EXACT>
__global__ void __launch_bounds__(kRunThreads)
    rom_run_kernel(RomDev d, int nsteps, double *__restrict__ xhat, double *__restrict__ hist,
                   int *__restrict__ iters) {
  __shared__ double xh[kMaxM];
  __shared__ double G[kMaxMr * kMaxM];
  __shared__ double b[kMaxMr];
  __shared__ double sol[kMaxM];
  __shared__ double s_eps, s_g1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = kRunThreads / 64;
  const int M = d.M, Mr = d.Mr, nd = d.nd;

  if (tid < M) xh[tid] = xhat[tid];
  __syncthreads();
  // previous-step terms for the first step: HyperPair at the initial xhat
  project(d, xh, tid, kRunThreads);
  __syncthreads();
  for (int i = wave; i < d.ns; i += nwaves)
    gather_target<EXACT>(d, i, lane, d.xbar, d.xbar, d.fbar_prev, d.fbar_prev, nullptr, nullptr);
  for (int q = tid; q < nd; q += kRunThreads) d.xbar_prev[q] = d.xbar[q];
  __syncthreads();

  for (int step = 0; step < nsteps; ++step) {
    int k = 1;
    for (;;) {
      project(d, xh, tid, kRunThreads);
      __syncthreads();
      for (int i = wave; i < d.ns; i += nwaves)
        gather_target<EXACT>(d, i, lane, d.xbar, d.xbar_prev, d.fbar_prev, d.fbar, d.rbar, d.C);
      __syncthreads();
      // G = A C, b = A rbar
      for (int t = tid; t < Mr * (M + 1); t += kRunThreads) {
        const int r = t / (M + 1), c = t % (M + 1);
        const double *a = d.A + (size_t)r * nd;
        double s = 0.0;
        if (c < M) {
          for (int q = 0; q < nd; ++q) s += a[q] * d.C[(size_t)q * M + c];
          G[r * M + c] = s;
        } else {
          for (int q = 0; q < nd; ++q) s += a[q] * d.rbar[q];
          b[r] = s;
        }
      }
      __syncthreads();
      if (wave == 0) {
        // relative reduced gradient |G^T b| / |G_1^T b_1|
        double gn = 0.0;
        if (lane < M) {
          double s = 0.0;
          for (int r = 0; r < Mr; ++r) s += G[r * M + lane] * b[r];
          gn = s * s;
        }
        gn = sqrt(wsumd(gn));
        if (k == 1) {
          if (lane == 0) s_g1 = gn;
        }
        const double g1 = (k == 1) ? gn : s_g1;
        const double eps = g1 > 0.0 ? gn / g1 : 0.0;
        // Householder QR of G (Mr x M, Mr <= 64: one row per lane) applied to b
        for (int kk = 0; kk < M; ++kk) {
          const double gkk = G[kk * M + kk];
          double v = (lane >= kk && lane < Mr) ? G[lane * M + kk] : 0.0;
          const double nrm = sqrt(wsumd(v * v));
          if (nrm == 0.0) continue;
          const double alpha = gkk > 0.0 ? -nrm : nrm;
          if (lane == kk) v -= alpha;
          const double vn2 = wsumd(v * v);
          for (int j = kk + 1; j < M; ++j) {
            const double gj = (lane < Mr) ? G[lane * M + j] : 0.0;
            const double s = wsumd(v * gj) * 2.0 / vn2;
            if (lane >= kk && lane < Mr) G[lane * M + j] = gj - s * v;
          }
          {
            const double bj = (lane < Mr) ? b[lane] : 0.0;
            const double s = wsumd(v * bj) * 2.0 / vn2;
            if (lane >= kk && lane < Mr) b[lane] = bj - s * v;
          }
          if (lane == kk) G[kk * M + kk] = alpha;
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
        if (lane == 0) {
          for (int kk = M - 1; kk >= 0; --kk) {
            double s = b[kk];
            for (int j = kk + 1; j < M; ++j) s -= G[kk * M + j] * sol[j];
            sol[kk] = s / G[kk * M + kk];
          }
          for (int m = 0; m < M; ++m) xh[m] -= d.alpha * sol[m];
          s_eps = eps;
        }
      }
      __syncthreads();
      ++k;
      if (!(s_eps > d.tol) || k > d.max_iter) break;
      __syncthreads();  // s_eps read by everyone before the next write
    }
    if (tid < M && hist) hist[(size_t)step * M + tid] = xh[tid];
    if (tid == 0 && iters) iters[step] = k - 1;
    __syncthreads();
    // previous-step terms: sampled rows at the accepted xhat, velocity of
    // the last HyperPair evaluation
    for (int q = tid; q < nd; q += kRunThreads) {
      double s = d.xbar0[q];
      const float *ph = d.Phibar + (size_t)q * M;
      for (int m = 0; m < M; ++m) s += (double)ph[m] * xh[m];
      d.xbar_prev[q] = s;
      d.fbar_prev[q] = d.fbar[q];
    }
    __syncthreads();
  }
  if (tid < M) xhat[tid] = xh[tid];
}

}  // namespace

struct ptrom_rom {
  ptrom_ctx *ctx = nullptr;
  RomDev d{};
  void *buf = nullptr;
};

extern "C" int ptrom_rom_create(ptrom_ctx *ctx, const ptrom_rom_desc *desc, ptrom_rom **out) {
  if (!ctx) return PTROM_EINVAL;
  ctx->err.clear();
  if (!desc || !out) return ctx->fail(PTROM_EINVAL, "NULL argument");
  const ptrom_rom_desc &s = *desc;
  const int nd = 2 * s.ns;
  if (s.M < 1 || s.M > kMaxM || s.Mr < s.M || s.Mr > kMaxMr || s.ns < 1 || nd > kMaxNd)
    return ctx->fail(PTROM_EINVAL, "need 1 <= M <= 32, M <= Mr <= 64, 1 <= ns <= 2^20");
  if (s.Nc < 0 || s.nnz < 0 || s.Nc > kMaxN || s.nnz > (int64_t(1) << 31) - 1)
    return ctx->fail(PTROM_EINVAL, "bad Nc / nnz");
  if (!s.Phibar || !s.xbar0 || !s.off || !s.A || (s.Nc > 0 && (!s.xqt0 || !s.Phit || !s.Gt)) ||
      (s.nnz > 0 && !s.ids))
    return ctx->fail(PTROM_EINVAL, "NULL artifact array");
  if (!(s.delta >= 0.0) || !(s.dt > 0.0) || !(s.tol >= 0.0) || !std::isfinite(s.alpha) ||
      s.max_iter < 1 || s.max_iter > 1000 || (s.jac_mode != PTROM_JAC_PAPER && s.jac_mode != PTROM_JAC_EXACT))
    return ctx->fail(PTROM_EINVAL, "bad delta/dt/tol/alpha/max_iter/jac_mode");
  if (s.off[0] != 0 || s.off[s.ns] != s.nnz) return ctx->fail(PTROM_EINVAL, "off must run from 0 to nnz");
  for (int i = 0; i < s.ns; ++i)
    if (s.off[i + 1] < s.off[i]) return ctx->fail(PTROM_EINVAL, "off must be non-decreasing");
  for (int64_t e = 0; e < s.nnz; ++e)
    if (s.ids[e] < 0 || s.ids[e] >= s.Nc) return ctx->fail(PTROM_EINVAL, "ids out of [0, Nc)");
  if (hipSetDevice(ctx->device) != hipSuccess) return ctx->fail(PTROM_EHIP, "hipSetDevice");

  const int M = s.M;
  const int64_t Nc = s.Nc > 0 ? s.Nc : 1;
  std::vector<float> phibar(size_t(nd) * M), xbar0(nd), xqt0(2 * Nc, 0.f), phit(2 * Nc * M, 0.f), gt(Nc, 0.f);
  std::vector<int> off(s.ns + 1), ids(s.nnz > 0 ? s.nnz : 1, 0);
  for (size_t q = 0; q < phibar.size(); ++q) phibar[q] = float(s.Phibar[q]);
  for (int q = 0; q < nd; ++q) xbar0[q] = float(s.xbar0[q]);
  for (int64_t c = 0; c < s.Nc; ++c) {
    xqt0[2 * c] = float(s.xqt0[2 * c]);
    xqt0[2 * c + 1] = float(s.xqt0[2 * c + 1]);
    gt[c] = float(s.Gt[c]);
    for (int q = 0; q < 2 * M; ++q) phit[2 * c * M + q] = float(s.Phit[2 * c * M + q]);
  }
  for (int i = 0; i <= s.ns; ++i) off[i] = int(s.off[i]);
  for (int64_t e = 0; e < s.nnz; ++e) ids[e] = int(s.ids[e]);

  auto rom = new ptrom_rom();
  rom->ctx = ctx;
  RomDev &d = rom->d;
  d.M = M; d.Mr = s.Mr; d.ns = s.ns; d.nd = nd; d.jac_mode = s.jac_mode; d.max_iter = s.max_iter;
  d.Nc = s.Nc; d.nnz = s.nnz;
  d.d2 = float(s.delta) * float(s.delta);
  d.dt = float(s.dt);
  d.tol = s.tol; d.alpha = s.alpha;

  const size_t bytes[] = {
      align256(phibar.size() * 4), align256(xbar0.size() * 4), align256(xqt0.size() * 4),
      align256(phit.size() * 4), align256(gt.size() * 4), align256(off.size() * 4),
      align256(ids.size() * 4), align256(size_t(s.Mr) * nd * 8),
      align256(2 * Nc * 8), align256(nd * 8), align256(nd * 8), align256(nd * 8), align256(nd * 8),
      align256(nd * 8), align256(size_t(nd) * M * 8), align256(kMaxM * 8)};
  size_t total = 0;
  for (size_t b : bytes) total += b;
  if (hipMalloc(&rom->buf, total) != hipSuccess) {
    delete rom;
    return ctx->fail(PTROM_ENOMEM, "rom allocation");
  }
  char *p = static_cast<char *>(rom->buf);
  void *ptrs[16];
  for (int q = 0; q < 16; ++q) {
    ptrs[q] = p;
    p += bytes[q];
  }
  d.Phibar = (float *)ptrs[0]; d.xbar0 = (float *)ptrs[1]; d.xqt0 = (float *)ptrs[2];
  d.Phit = (float *)ptrs[3]; d.Gt = (float *)ptrs[4]; d.off = (int *)ptrs[5]; d.ids = (int *)ptrs[6];
  d.A = (double *)ptrs[7]; d.pos = (double *)ptrs[8]; d.xbar = (double *)ptrs[9];
  d.xbar_prev = (double *)ptrs[10]; d.fbar = (double *)ptrs[11]; d.fbar_prev = (double *)ptrs[12];
  d.rbar = (double *)ptrs[13]; d.C = (double *)ptrs[14]; d.xh = (double *)ptrs[15];
  hipError_t e = hipMemcpy(ptrs[0], phibar.data(), phibar.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ptrs[1], xbar0.data(), xbar0.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ptrs[2], xqt0.data(), xqt0.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ptrs[3], phit.data(), phit.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ptrs[4], gt.data(), gt.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ptrs[5], off.data(), off.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ptrs[6], ids.data(), ids.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ptrs[7], s.A, size_t(s.Mr) * nd * 8, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hipFree(rom->buf);
    delete rom;
    return ctx->hip_fail(e, "rom upload");
  }
  *out = rom;
  return PTROM_OK;
}

extern "C" void ptrom_rom_destroy(ptrom_rom *rom) {
  if (!rom) return;
  hipSetDevice(rom->ctx->device);
  hipDeviceSynchronize();
  if (rom->buf) hipFree(rom->buf);
  delete rom;
}

extern "C" int ptrom_rom_hyperpair(ptrom_rom *rom, const double *xhat, const double *xbar_prev,
                                   const double *fbar_prev, double *xbar, double *fbar, double *rbar,
                                   double *C, ptrom_stream stream) {
  if (!rom) return PTROM_EINVAL;
  ptrom_ctx *ctx = rom->ctx;
  ctx->err.clear();
  if (!xhat || !xbar_prev || !fbar_prev) return ctx->fail(PTROM_EINVAL, "NULL input");
  if (hipSetDevice(ctx->device) != hipSuccess) return ctx->fail(PTROM_EHIP, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  const RomDev &d = rom->d;
  const int64_t work = std::max<int64_t>(2 * d.Nc, d.nd);
  const unsigned pg = (unsigned)std::min<int64_t>((work + 255) / 256, 4096);
  hipLaunchKernelGGL(project_kernel, dim3(pg), dim3(256), 0, st, d, xhat);
  const unsigned gg = (unsigned)((d.ns + 3) / 4);
  if (d.jac_mode == PTROM_JAC_EXACT)
    hipLaunchKernelGGL(gather_kernel<true>, dim3(gg), dim3(256), 0, st, d, xbar_prev, fbar_prev, fbar, rbar, C);
  else
    hipLaunchKernelGGL(gather_kernel<false>, dim3(gg), dim3(256), 0, st, d, xbar_prev, fbar_prev, fbar, rbar, C);
  if (xbar) PTROM_CHECK_HIP(ctx, hipMemcpyAsync(xbar, d.xbar, sizeof(double) * d.nd, hipMemcpyDeviceToDevice, st));
  PTROM_CHECK_HIP(ctx, hipGetLastError());
  return PTROM_OK;
}

extern "C" int ptrom_rom_run(ptrom_rom *rom, int nsteps, double *xhat, double *xhat_hist,
                             int32_t *iters, ptrom_stream stream) {
  if (!rom) return PTROM_EINVAL;
  ptrom_ctx *ctx = rom->ctx;
  ctx->err.clear();
  if (!xhat || nsteps < 0) return ctx->fail(PTROM_EINVAL, "xhat required and nsteps >= 0");
  if (hipSetDevice(ctx->device) != hipSuccess) return ctx->fail(PTROM_EHIP, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  if (rom->d.jac_mode == PTROM_JAC_EXACT)
    hipLaunchKernelGGL(rom_run_kernel<true>, dim3(1), dim3(kRunThreads), 0, st, rom->d, nsteps, xhat, xhat_hist, iters);
  else
    hipLaunchKernelGGL(rom_run_kernel<false>, dim3(1), dim3(kRunThreads), 0, st, rom->d, nsteps, xhat, xhat_hist, iters);
  PTROM_CHECK_HIP(ctx, hipGetLastError());
  return PTROM_OK;
}
