// Online projection-tree ROM: HyperPair (Algorithm "HyperPair") and the
// Gauss-Newton loop around it (Algorithm "Gauss-Newton").
//
// Entry layout.  Each interaction-list entry e = (target i, surrogate c) is
// stored as r0_e = xbar0_i - xqt0_c (2), Gamma~_c, pad, D_e = Phibar_i - Phit_c
// (2 x M), so that the pair separation at generalized coordinates xhat is
// r_e = r0_e + D_e xhat, which equals xbar_i - p_c with p_c = xqt0_c + Phit_c
// xhat (Algorithm "HyperPair" preamble).  The gather then streams contiguous
// entry rows (coalesced) with no projection pass and no indirection.
//
// Per Gauss-Newton iteration:
//   gather    one wave64 per sampled target walks its entries (lanes stride),
//             does the pair arithmetic in FP32 (velocity and the 2x2 self
//             block B_i; in the exact mode sum_e G_e D_e instead), reduces
//             across the wave with shuffles, and writes the trapezoid residual
//             rows rbar = xbar - xbar_prev - dt/2 (fbar + fbar_prev) and the
//             rows of C = Phibar - dt/2 dfbar/dxhat in FP64;
//   solve     G = A C, b = A rbar (FP64), the relative reduced gradient
//             |G^T b| / |G_1^T b_1|, Householder QR of G in one wave and
//             xhat -= alpha G^+ b.
// ptrom_rom_run keeps the whole loop (all steps, all iterations) inside one
// workgroup with A, C, rbar and the previous-step rows in LDS when they fit;
// ptrom_rom_hyperpair runs the gather over many workgroups (large sample sets).
#include <cmath>
#include <vector>

#include "internal.h"

using namespace ptrom;

namespace {

constexpr int kMaxM = 32;
constexpr int kMaxMr = 64;
constexpr int kRunThreads = 1024;
constexpr double kInv2PiD = 0.15915494309189533576888376337251;
constexpr size_t kMaxDynLds = 40 * 1024;  // keeps the workgroup under 64 KB of LDS

struct RomDev {
  int M, Mr, ns, nd, jac_mode, max_iter, ew;
  int64_t nnz;
  float d2, dt;
  double tol, alpha;
  const float *Phibar, *xbar0;  // [nd][M], [nd]
  const float *ent;             // [nnz][ew]: r0x r0y Gamma pad Dx[M] Dy[M]
  const int *off;               // [ns+1]
  const double *A;              // [Mr][nd]
  // scratch used when the LDS copies do not fit
  double *xbar_prev, *fbar, *fbar_prev, *rbar, *C;
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

// xbar_i (both rows) at xhat, FP64
__device__ __forceinline__ void sampled_position(const RomDev &d, int i, const double *xh, double &tx,
                                                 double &ty) {
  const int M = d.M, ns = d.ns;
  tx = d.xbar0[i];
  ty = d.xbar0[ns + i];
  const float *px = d.Phibar + (size_t)i * M, *py = d.Phibar + (size_t)(ns + i) * M;
  for (int m = 0; m < M; ++m) {
    tx += (double)px[m] * xh[m];
    ty += (double)py[m] * xh[m];
  }
}

// HyperPair rows of sampled target i, computed by one whole wave.
// xh: FP64 xhat, xf: FP32 copy.  Any output pointer may be null.
template <bool EXACT>
__device__ void gather_target(const RomDev &d, int i, int lane, const double *xh, const float *xf,
                              const double *xbar_prev, const double *fbar_prev, double *xbar_out,
                              double *fbar_out, double *rbar_out, double *C_out) {
  const int M = d.M, ns = d.ns, ew = d.ew;
  double tx, ty;
  sampled_position(d, i, xh, tx, ty);
  float fx = 0.f, fy = 0.f, ba = 0.f, bb = 0.f, bc = 0.f;
  float ex[EXACT ? kMaxM : 1], ey[EXACT ? kMaxM : 1];
  if constexpr (EXACT) {
    for (int m = 0; m < kMaxM; ++m) ex[m] = ey[m] = 0.f;
  }
  const int e0 = d.off[i], e1 = d.off[i + 1];
  for (int e = e0 + lane; e < e1; e += 64) {
    const float *E = d.ent + (size_t)e * ew;
    const float4 head = *reinterpret_cast<const float4 *>(E);
    float rx = head.x, ry = head.y;
    const float *Dx = E + 4, *Dy = E + 4 + M;
    for (int m = 0; m < M; ++m) {
      rx = fmaf(Dx[m], xf[m], rx);
      ry = fmaf(Dy[m], xf[m], ry);
    }
    const float q = fmaf(rx, rx, fmaf(ry, ry, d.d2));
    // a surrogate exactly on its target (possible at delta = 0) adds nothing
    const float r = q > 0.f ? 1.0f / q : 0.f;
    const float g = head.z * r;
    fx = fmaf(-ry, g, fx);
    fy = fmaf(rx, g, fy);
    const float g2 = g * r;
    const float a2 = (rx + rx) * ry;
    const float dd = fmaf(ry, ry, -rx * rx);
    if constexpr (EXACT) {
      const float h00 = g2 * a2, h01 = g2 * (dd - d.d2), h10 = g2 * (dd + d.d2);
      for (int m = 0; m < M; ++m) {
        ex[m] = fmaf(h00, Dx[m], fmaf(h01, Dy[m], ex[m]));
        ey[m] = fmaf(h10, Dx[m], fmaf(-h00, Dy[m], ey[m]));
      }
    } else {
      ba = fmaf(g2, a2, ba);
      bb = fmaf(g2, dd - d.d2, bb);
      bc = fmaf(g2, dd + d.d2, bc);
    }
  }
  const double Fx = wsum(fx) * kInv2PiD, Fy = wsum(fy) * kInv2PiD;
  const double hdt = 0.5 * (double)d.dt;
  if (lane == 0) {
    if (xbar_out) {
      xbar_out[i] = tx;
      xbar_out[ns + i] = ty;
    }
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
    if constexpr (EXACT) {
      // C_i = Phibar_i - dt/2 sum_e G_e (Phibar_i - Phit_c)
      for (int m = 0; m < M; ++m) {
        const double jx = wsum(ex[m]) * kInv2PiD, jy = wsum(ey[m]) * kInv2PiD;
        if (lane == m) {
          const double px = d.Phibar[(size_t)i * M + m], py = d.Phibar[(size_t)(ns + i) * M + m];
          C_out[(size_t)i * M + m] = px - hdt * jx;
          C_out[(size_t)(ns + i) * M + m] = py - hdt * jy;
        }
      }
    } else {
      // C_i = Phibar_i - dt/2 B_i Phibar_i (the paper's inexact Jacobian)
      const double B00 = wsum(ba) * kInv2PiD, B01 = wsum(bb) * kInv2PiD, B10 = wsum(bc) * kInv2PiD;
      if (lane < M) {
        const int m = lane;
        const double px = d.Phibar[(size_t)i * M + m], py = d.Phibar[(size_t)(ns + i) * M + m];
        C_out[(size_t)i * M + m] = px - hdt * (B00 * px + B01 * py);
        C_out[(size_t)(ns + i) * M + m] = py - hdt * (B10 * px - B00 * py);
      }
    }
  }
}

// ----------------------------------------------------------- hyperpair hook

template <bool EXACT>
__global__ void __launch_bounds__(256)
    gather_kernel(RomDev d, const double *__restrict__ xhat, const double *__restrict__ xbar_prev,
                  const double *__restrict__ fbar_prev, double *xbar, double *fbar, double *rbar, double *C) {
  __shared__ double xh[kMaxM];
  __shared__ float xf[kMaxM];
  if (threadIdx.x < d.M) {
    xh[threadIdx.x] = xhat[threadIdx.x];
    xf[threadIdx.x] = (float)xhat[threadIdx.x];
  }
  __syncthreads();
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (wave >= d.ns) return;
  gather_target<EXACT>(d, wave, lane, xh, xf, xbar_prev, fbar_prev, xbar, fbar, rbar, C);
}

// ----------------------------------------------------------- device-resident loop

template <bool EXACT>
__global__ void __launch_bounds__(kRunThreads)
    rom_run_kernel(RomDev d, int nsteps, int lds_arrays, double *__restrict__ xhat, double *__restrict__ hist,
                   int *__restrict__ iters) {
  __shared__ double xh[kMaxM];
  __shared__ float xf[kMaxM];
  __shared__ double G[kMaxMr * kMaxM];
  __shared__ double b[kMaxMr];
  __shared__ double sol[kMaxM];
  __shared__ double s_eps, s_g1;
  extern __shared__ double dyn[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = kRunThreads / 64;
  const int M = d.M, Mr = d.Mr, nd = d.nd;

  // A, C, rbar, fbar, fbar_prev, xbar_prev: LDS copies when they fit
  const double *A = d.A;
  double *C = d.C, *rbar = d.rbar, *fbar = d.fbar, *fbar_prev = d.fbar_prev, *xbar_prev = d.xbar_prev;
  if (lds_arrays) {
    double *p = dyn;
    double *Al = p; p += (size_t)Mr * nd;
    C = p; p += (size_t)nd * M;
    rbar = p; p += nd;
    fbar = p; p += nd;
    fbar_prev = p; p += nd;
    xbar_prev = p;
    for (int t = tid; t < Mr * nd; t += kRunThreads) Al[t] = d.A[t];
    A = Al;
  }
  if (tid < M) {
    xh[tid] = xhat[tid];
    xf[tid] = (float)xhat[tid];
  }
  __syncthreads();
  // previous-step terms for the first step: HyperPair at the initial xhat
  for (int i = wave; i < d.ns; i += nwaves)
    gather_target<EXACT>(d, i, lane, xh, xf, nullptr, nullptr, xbar_prev, fbar_prev, nullptr, nullptr);
  __syncthreads();

  for (int step = 0; step < nsteps; ++step) {
    int k = 1;
    for (;;) {
      for (int i = wave; i < d.ns; i += nwaves)
        gather_target<EXACT>(d, i, lane, xh, xf, xbar_prev, fbar_prev, nullptr, fbar, rbar, C);
      __syncthreads();
      // G = A C, b = A rbar
      for (int t = tid; t < Mr * (M + 1); t += kRunThreads) {
        const int r = t / (M + 1), c = t % (M + 1);
        const double *a = A + (size_t)r * nd;
        double s = 0.0;
        if (c < M) {
          for (int q = 0; q < nd; ++q) s += a[q] * C[(size_t)q * M + c];
          G[r * M + c] = s;
        } else {
          for (int q = 0; q < nd; ++q) s += a[q] * rbar[q];
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
        if (k == 1 && lane == 0) s_g1 = gn;
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
          for (int m = 0; m < M; ++m) {
            xh[m] -= d.alpha * sol[m];
            xf[m] = (float)xh[m];
          }
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
    // previous-step terms: sampled rows at the accepted xhat, velocity of
    // the last HyperPair evaluation
    for (int q = tid; q < nd; q += kRunThreads) {
      const int i = q < d.ns ? q : q - d.ns;
      double tx, ty;
      sampled_position(d, i, xh, tx, ty);
      xbar_prev[q] = q < d.ns ? tx : ty;
      fbar_prev[q] = fbar[q];
    }
    __syncthreads();
  }
  if (tid < M) xhat[tid] = xh[tid];
}

size_t run_lds_bytes(int M, int Mr, int nd) {
  return sizeof(double) * ((size_t)Mr * nd + (size_t)nd * M + 4 * (size_t)nd);
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
  if (s.M < 1 || s.M > kMaxM || s.Mr < s.M || s.Mr > kMaxMr || s.ns < 1 || s.ns > (1 << 20))
    return ctx->fail(PTROM_EINVAL, "need 1 <= M <= 32, M <= Mr <= 64, 1 <= ns <= 2^20");
  const int nd = 2 * s.ns;
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
  const int ew = 4 + (2 * M + 3) / 4 * 4;
  std::vector<float> phibar(size_t(nd) * M), xbar0(nd);
  std::vector<int> off32(s.ns + 1);
  for (size_t q = 0; q < phibar.size(); ++q) phibar[q] = float(s.Phibar[q]);
  for (int q = 0; q < nd; ++q) xbar0[q] = float(s.xbar0[q]);
  for (int i = 0; i <= s.ns; ++i) off32[i] = int(s.off[i]);
  // entry rows: r0 = xbar0_i - xqt0_c, Gamma~_c, D = Phibar_i - Phit_c (differences in FP64)
  std::vector<float> ent(size_t(s.nnz > 0 ? s.nnz : 1) * ew, 0.0f);
  for (int i = 0; i < s.ns; ++i)
    for (int64_t e = s.off[i]; e < s.off[i + 1]; ++e) {
      const int64_t c = s.ids[e];
      float *E = ent.data() + (size_t)e * ew;
      E[0] = float(s.xbar0[i] - s.xqt0[2 * c]);
      E[1] = float(s.xbar0[s.ns + i] - s.xqt0[2 * c + 1]);
      E[2] = float(s.Gt[c]);
      for (int m = 0; m < M; ++m) {
        E[4 + m] = float(s.Phibar[(size_t)i * M + m] - s.Phit[(size_t)(2 * c) * M + m]);
        E[4 + M + m] = float(s.Phibar[(size_t)(s.ns + i) * M + m] - s.Phit[(size_t)(2 * c + 1) * M + m]);
      }
    }

  auto rom = new ptrom_rom();
  rom->ctx = ctx;
  RomDev &d = rom->d;
  d.M = M; d.Mr = s.Mr; d.ns = s.ns; d.nd = nd; d.jac_mode = s.jac_mode; d.max_iter = s.max_iter;
  d.ew = ew; d.nnz = s.nnz;
  d.d2 = float(s.delta) * float(s.delta);
  d.dt = float(s.dt);
  d.tol = s.tol; d.alpha = s.alpha;

  const size_t bytes[] = {align256(phibar.size() * 4), align256(xbar0.size() * 4), align256(ent.size() * 4),
                          align256(off32.size() * 4), align256(size_t(s.Mr) * nd * 8),
                          align256(nd * 8), align256(nd * 8), align256(nd * 8), align256(nd * 8),
                          align256(size_t(nd) * M * 8)};
  constexpr int NB = sizeof(bytes) / sizeof(bytes[0]);
  size_t total = 0;
  for (size_t b : bytes) total += b;
  if (hipMalloc(&rom->buf, total) != hipSuccess) {
    delete rom;
    return ctx->fail(PTROM_ENOMEM, "rom allocation");
  }
  char *p = static_cast<char *>(rom->buf);
  void *ptrs[NB];
  for (int q = 0; q < NB; ++q) {
    ptrs[q] = p;
    p += bytes[q];
  }
  d.Phibar = (float *)ptrs[0]; d.xbar0 = (float *)ptrs[1]; d.ent = (float *)ptrs[2]; d.off = (int *)ptrs[3];
  d.A = (double *)ptrs[4]; d.xbar_prev = (double *)ptrs[5]; d.fbar = (double *)ptrs[6];
  d.fbar_prev = (double *)ptrs[7]; d.rbar = (double *)ptrs[8]; d.C = (double *)ptrs[9];
  hipError_t e = hipMemcpy(ptrs[0], phibar.data(), phibar.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ptrs[1], xbar0.data(), xbar0.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ptrs[2], ent.data(), ent.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ptrs[3], off32.data(), off32.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ptrs[4], s.A, size_t(s.Mr) * nd * 8, hipMemcpyHostToDevice);
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
  if (!xhat || (rbar && (!xbar_prev || !fbar_prev))) return ctx->fail(PTROM_EINVAL, "NULL input");
  if (hipSetDevice(ctx->device) != hipSuccess) return ctx->fail(PTROM_EHIP, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  const RomDev &d = rom->d;
  const unsigned gg = (unsigned)((d.ns + 3) / 4);
  if (d.jac_mode == PTROM_JAC_EXACT)
    hipLaunchKernelGGL(gather_kernel<true>, dim3(gg), dim3(256), 0, st, d, xhat, xbar_prev, fbar_prev, xbar, fbar,
                       rbar, C);
  else
    hipLaunchKernelGGL(gather_kernel<false>, dim3(gg), dim3(256), 0, st, d, xhat, xbar_prev, fbar_prev, xbar,
                       fbar, rbar, C);
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
  const RomDev &d = rom->d;
  const size_t lds = run_lds_bytes(d.M, d.Mr, d.nd);
  const int use_lds = lds <= kMaxDynLds;
  const size_t shmem = use_lds ? lds : 0;
  if (d.jac_mode == PTROM_JAC_EXACT)
    hipLaunchKernelGGL(rom_run_kernel<true>, dim3(1), dim3(kRunThreads), shmem, st, d, nsteps, use_lds, xhat,
                       xhat_hist, iters);
  else
    hipLaunchKernelGGL(rom_run_kernel<false>, dim3(1), dim3(kRunThreads), shmem, st, d, nsteps, use_lds, xhat,
                       xhat_hist, iters);
  PTROM_CHECK_HIP(ctx, hipGetLastError());
  return PTROM_OK;
}
