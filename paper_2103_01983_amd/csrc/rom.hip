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
//             across the wave with DPP row reductions, and writes the
//             trapezoid residual rows rbar = xbar - xbar_prev - dt/2 (fbar +
//             fbar_prev) and the rows of C = Phibar - dt/2 dfbar/dxhat (FP64);
//   solve     G' = A [C | rbar] (FP64, four columns per thread), the Gram
//             matrix G'^T G' = [G^T G, G^T b; ...], the relative reduced
//             gradient |G^T b| / |G_1^T b_1|, and in one wave a Cholesky
//             factorisation of G^T G held one row per lane, forward and back
//             substitution by lane broadcasts, and one refinement step on the
//             true residual b - G x (corrected semi-normal equations), then
//             xhat -= alpha x.
// ptrom_rom_run keeps the whole loop (all steps, all iterations) inside one
// workgroup with A, [C | rbar] and the previous-step rows in LDS when they
// fit; ptrom_rom_hyperpair runs the gather over many workgroups (large sample
// sets).
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

using namespace ptrom;

namespace {

constexpr int kMaxM = 32;
constexpr int kMaxMr = 64;
constexpr int kMaxLdc = 36;   // columns of [C | rbar] rounded up to 4
constexpr int kLt = kMaxM + 1;  // row stride of the transposed factor in LDS (bank spread)
constexpr int kRunThreads = 1024;
constexpr double kInv2PiD = 0.15915494309189533576888376337251;

struct RomDev {
  int M, Mr, ns, nd, jac_mode, max_iter, ew, ldc;
  int64_t nnz;
  float d2, dt;
  double tol, alpha;
  const float *Phibar, *xbar0;  // [nd][M], [nd]
  const float *ent;             // [nnz][ew]: r0x r0y Gamma pad Dx[M] Dy[M]
  const int *off;               // [ns+1]
  const double *A;              // [Mr][nd]
  // scratch used when the LDS copies do not fit; C holds [C | rbar | 0] with
  // leading dimension ldc
  double *xbar_prev, *fbar, *fbar_prev, *C;
};

// Wave-wide sums by DPP: within each row of 16 lanes swap neighbours
// (quad_perm [1,0,3,2] and [2,3,0,1]), then mirror the half row and the row,
// so every lane holds its row's sum; the four row sums are then read out and
// added in a fixed order.  Must be called with all 64 lanes active.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __builtin_bit_cast(float, dpp_i<CTRL>(__builtin_bit_cast(int, v)));
}

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)dpp_i<CTRL>((int)(unsigned)(u & 0xffffffffull));
  const unsigned hi = (unsigned)dpp_i<CTRL>((int)(unsigned)(u >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ float lane_f(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

__device__ __forceinline__ double lane_d(double v, int l) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffull), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ float wsum(float v) {
  v += dpp_f<0xB1>(v);
  v += dpp_f<0x4E>(v);
  v += dpp_f<0x141>(v);
  v += dpp_f<0x140>(v);
  return (lane_f(v, 0) + lane_f(v, 16)) + (lane_f(v, 32) + lane_f(v, 48));
}

__device__ __forceinline__ double wsumd(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x141>(v);
  v += dpp_d<0x140>(v);
  return (lane_d(v, 0) + lane_d(v, 16)) + (lane_d(v, 32) + lane_d(v, 48));
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
// xh: FP64 xhat, xf: FP32 copy.  Any output pointer may be null.  Row q of
// rbar is rbar_out[q * rs], row q of C is C_out[q * ldc .. + M).
template <bool EXACT>
__device__ void gather_target(const RomDev &d, int i, int lane, const double *xh, const float *xf,
                              const double *xbar_prev, const double *fbar_prev, double *xbar_out,
                              double *fbar_out, double *rbar_out, int rs, double *C_out, int ldc) {
  const int M = d.M, ns = d.ns, ew = d.ew;
  double tx, ty;
  sampled_position(d, i, xh, tx, ty);
  float fx = 0.f, fy = 0.f, ba = 0.f, bb = 0.f, bc = 0.f;
  float ex[EXACT ? kMaxM : 1], ey[EXACT ? kMaxM : 1];
  if constexpr (EXACT) {
#pragma unroll
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
#pragma unroll
      for (int m = 0; m < kMaxM; ++m) {
        if (m < M) {
          ex[m] = fmaf(h00, Dx[m], fmaf(h01, Dy[m], ex[m]));
          ey[m] = fmaf(h10, Dx[m], fmaf(-h00, Dy[m], ey[m]));
        }
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
      rbar_out[(size_t)i * rs] = (tx - xbar_prev[i]) - hdt * (Fx + fbar_prev[i]);
      rbar_out[(size_t)(ns + i) * rs] = (ty - xbar_prev[ns + i]) - hdt * (Fy + fbar_prev[ns + i]);
    }
  }
  if (C_out) {
    if constexpr (EXACT) {
      // C_i = Phibar_i - dt/2 sum_e G_e (Phibar_i - Phit_c)
      double jx = 0.0, jy = 0.0;
#pragma unroll
      for (int m = 0; m < kMaxM; ++m) {
        if (m < M) {
          const float sx = wsum(ex[m]), sy = wsum(ey[m]);
          if (lane == m) {
            jx = sx * kInv2PiD;
            jy = sy * kInv2PiD;
          }
        }
      }
      if (lane < M) {
        const int m = lane;
        const double px = d.Phibar[(size_t)i * M + m], py = d.Phibar[(size_t)(ns + i) * M + m];
        C_out[(size_t)i * ldc + m] = px - hdt * jx;
        C_out[(size_t)(ns + i) * ldc + m] = py - hdt * jy;
      }
    } else {
      // C_i = Phibar_i - dt/2 B_i Phibar_i (the paper's inexact Jacobian)
      const double B00 = wsum(ba) * kInv2PiD, B01 = wsum(bb) * kInv2PiD, B10 = wsum(bc) * kInv2PiD;
      if (lane < M) {
        const int m = lane;
        const double px = d.Phibar[(size_t)i * M + m], py = d.Phibar[(size_t)(ns + i) * M + m];
        C_out[(size_t)i * ldc + m] = px - hdt * (B00 * px + B01 * py);
        C_out[(size_t)(ns + i) * ldc + m] = py - hdt * (B10 * px - B00 * py);
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
  gather_target<EXACT>(d, wave, lane, xh, xf, xbar_prev, fbar_prev, xbar, fbar, rbar, 1, C, d.M);
}

// ----------------------------------------------------------- device-resident loop

// Solves (L L^T) x = rhs for the factor held one row per lane (a[j] = L_lj on
// lane l, j <= l) and its transpose in LDS (Lt[i * kLt + k] = L_ki).  rhs_i is
// given on lane i; x is written to xs[] and lane i's component returned.  A
// zero pivot drops its direction (component 0).
__device__ __forceinline__ double chol_solve(const double (&a)[kMaxM], const double *Lt, int M, int lane,
                                             double rhs, double *xs) {
  // forward: L y = rhs; lane i keeps rhs_i - sum_{j<k} L_ij y_j
  double acc = rhs, ymine = 0.0;
#pragma unroll
  for (int k = 0; k < kMaxM; ++k) {
    if (k < M) {
      const double lkk = lane_d(a[k], k);
      const double yk = lkk != 0.0 ? lane_d(acc, k) / lkk : 0.0;
      if (lane == k) ymine = yk;
      acc = fma(-a[k], yk, acc);
    }
  }
  // backward: L^T x = y; lane i keeps y_i - sum_{j>k} L_ji x_j
  double acc2 = ymine, xmine = 0.0;
#pragma unroll
  for (int k = kMaxM - 1; k >= 0; --k) {
    if (k < M) {
      const double ukk = lane_d(a[k], k);
      const double xk = ukk != 0.0 ? lane_d(acc2, k) / ukk : 0.0;
      if (lane == k) xmine = xk;
      if (lane == 0) xs[k] = xk;
      if (lane < k) acc2 = fma(-Lt[lane * kLt + k], xk, acc2);
    }
  }
  return xmine;
}

template <bool EXACT>
__global__ void __launch_bounds__(kRunThreads)
    rom_run_kernel(RomDev d, int nsteps, int lds_arrays, double *__restrict__ xhat, double *__restrict__ hist,
                   int *__restrict__ iters) {
  __shared__ double xh[kMaxM];
  __shared__ float xf[kMaxM];
  __shared__ double Gp[kMaxMr * kMaxLdc];          // G' = A [C | rbar | 0]
  __shared__ double Nw[(kMaxM + 1) * (kMaxM + 1)];  // G'^T G', then L^T
  __shared__ double rr[kMaxMr], xs[kMaxM], dxs[kMaxM];
  __shared__ double s_eps, s_g1;
  extern __shared__ double dyn[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = kRunThreads / 64;
  const int M = d.M, Mr = d.Mr, nd = d.nd, ldc = d.ldc, M1 = M + 1;

  // A, [C | rbar], fbar, fbar_prev, xbar_prev: LDS copies when they fit
  const double *A = d.A;
  double *Cp = d.C, *fbar = d.fbar, *fbar_prev = d.fbar_prev, *xbar_prev = d.xbar_prev;
  if (lds_arrays) {
    double *p = dyn;
    double *Al = p; p += (size_t)Mr * nd;
    Cp = p; p += (size_t)nd * ldc;
    fbar = p; p += nd;
    fbar_prev = p; p += nd;
    xbar_prev = p;
    for (int t = tid; t < Mr * nd; t += kRunThreads) Al[t] = d.A[t];
    A = Al;
  }
  for (int t = tid; t < nd * ldc; t += kRunThreads) Cp[t] = 0.0;  // padding columns stay zero
  if (tid < M) {
    xh[tid] = xhat[tid];
    xf[tid] = (float)xhat[tid];
  }
  __syncthreads();
  // previous-step terms for the first step: HyperPair at the initial xhat
  for (int i = wave; i < d.ns; i += nwaves)
    gather_target<EXACT>(d, i, lane, xh, xf, nullptr, nullptr, xbar_prev, fbar_prev, nullptr, 0, nullptr, 0);
  __syncthreads();

  const int nblk = ldc / 4;
  const int npair = M1 * (M1 + 1) / 2;
  for (int step = 0; step < nsteps; ++step) {
    int k = 1;
    for (;;) {
      for (int i = wave; i < d.ns; i += nwaves)
        gather_target<EXACT>(d, i, lane, xh, xf, xbar_prev, fbar_prev, nullptr, fbar, Cp + M, ldc, Cp, ldc);
      __syncthreads();
      // G' = A [C | rbar | 0], four columns per thread
      for (int t = tid; t < Mr * nblk; t += kRunThreads) {
        const int r = t / nblk, c0 = (t - r * nblk) * 4;
        const double *arow = A + (size_t)r * nd;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        for (int q = 0; q < nd; ++q) {
          const double av = arow[q];
          const double *c = Cp + (size_t)q * ldc + c0;
          s0 = fma(av, c[0], s0);
          s1 = fma(av, c[1], s1);
          s2 = fma(av, c[2], s2);
          s3 = fma(av, c[3], s3);
        }
        double *g = Gp + r * ldc + c0;
        g[0] = s0;
        g[1] = s1;
        g[2] = s2;
        g[3] = s3;
      }
      __syncthreads();
      // G'^T G' over the first M + 1 columns (lower triangle, mirrored)
      for (int t = tid; t < npair; t += kRunThreads) {
        int i = 0;
        while ((i + 1) * (i + 2) / 2 <= t) ++i;
        const int j = t - i * (i + 1) / 2;
        double sum = 0.0;
        for (int r = 0; r < Mr; ++r) sum = fma(Gp[r * ldc + i], Gp[r * ldc + j], sum);
        Nw[i * M1 + j] = sum;
        Nw[j * M1 + i] = sum;
      }
      __syncthreads();
      if (wave == 0) {
        // relative reduced gradient |G^T b| / |G_1^T b_1|
        const double gl = lane < M ? Nw[lane * M1 + M] : 0.0;
        const double gn = sqrt(wsumd(gl * gl));
        const double g1 = (k == 1) ? gn : s_g1;
        const double eps = g1 > 0.0 ? gn / g1 : 0.0;
        // Cholesky of G^T G, row `lane` in registers
        double a[kMaxM];
#pragma unroll
        for (int j = 0; j < kMaxM; ++j) a[j] = (j < M && lane < M) ? Nw[lane * M1 + j] : 0.0;
#pragma unroll
        for (int kk = 0; kk < kMaxM; ++kk) {
          if (kk < M) {
            const double piv = lane_d(a[kk], kk);
            const bool pos = piv > 0.0;
            const double lkk = pos ? sqrt(piv) : 0.0;
            const double inv = pos ? 1.0 / lkk : 0.0;
            a[kk] = lane == kk ? lkk : a[kk] * inv;
#pragma unroll
            for (int j = kk + 1; j < kMaxM; ++j) {
              if (j < M) {
                const double ljk = lane_d(a[kk], j);
                a[j] = fma(-a[kk], ljk, a[j]);
              }
            }
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // all reads of Nw done
        // L^T into LDS: Lt[i * kLt + k] = L_ki for k >= i
#pragma unroll
        for (int j = 0; j < kMaxM; ++j)
          if (j < M && lane < M && lane >= j) Nw[j * kLt + lane] = a[j];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        double xl = chol_solve(a, Nw, M, lane, gl, xs);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        // one refinement step on the true residual: r' = b - G x, G^T r'
        if (lane < Mr) {
          double rv = Gp[lane * ldc + M];
#pragma unroll
          for (int j = 0; j < kMaxM; ++j)
            if (j < M) rv = fma(-Gp[lane * ldc + j], xs[j], rv);
          rr[lane] = rv;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        double g2 = 0.0;
        if (lane < M)
          for (int r = 0; r < Mr; ++r) g2 = fma(Gp[r * ldc + lane], rr[r], g2);
        xl += chol_solve(a, Nw, M, lane, g2, dxs);
        if (lane < M) {
          xh[lane] -= d.alpha * xl;
          xf[lane] = (float)xh[lane];
        }
        if (lane == 0) {
          if (k == 1) s_g1 = gn;
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

size_t run_lds_bytes(int Mr, int nd, int ldc) {
  return sizeof(double) * ((size_t)Mr * nd + (size_t)nd * ldc + 3 * (size_t)nd);
}

}  // namespace

struct ptrom_rom {
  ptrom_ctx *ctx = nullptr;
  RomDev d{};
  void *buf = nullptr;
  size_t max_dyn_lds = 0;  // dynamic LDS the run kernel may take on this device
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
  {
    // dynamic LDS the run kernel may request: the device's per-workgroup
    // limit minus the kernel's static LDS
    int maxsh = 0;
    if (hipDeviceGetAttribute(&maxsh, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device) != hipSuccess)
      maxsh = 64 * 1024;
    size_t stat = 0;
    const void *kernels[2] = {reinterpret_cast<const void *>(rom_run_kernel<false>),
                              reinterpret_cast<const void *>(rom_run_kernel<true>)};
    for (const void *k : kernels) {
      hipFuncAttributes fa{};
      if (hipFuncGetAttributes(&fa, k) == hipSuccess) stat = std::max(stat, fa.sharedSizeBytes);
    }
    size_t dyn = size_t(maxsh) > stat ? size_t(maxsh) - stat : 0;
    for (const void *k : kernels)
      if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, int(dyn)) != hipSuccess) {
        dyn = 64 * 1024 > stat ? 64 * 1024 - stat : 0;
        (void)hipGetLastError();
        break;
      }
    rom->max_dyn_lds = dyn;
  }
  RomDev &d = rom->d;
  d.M = M; d.Mr = s.Mr; d.ns = s.ns; d.nd = nd; d.jac_mode = s.jac_mode; d.max_iter = s.max_iter;
  d.ew = ew; d.nnz = s.nnz;
  d.ldc = (M + 1 + 3) / 4 * 4;
  d.d2 = float(s.delta) * float(s.delta);
  d.dt = float(s.dt);
  d.tol = s.tol; d.alpha = s.alpha;

  const size_t bytes[] = {align256(phibar.size() * 4), align256(xbar0.size() * 4), align256(ent.size() * 4),
                          align256(off32.size() * 4), align256(size_t(s.Mr) * nd * 8),
                          align256(nd * 8), align256(nd * 8), align256(nd * 8),
                          align256(size_t(nd) * ((M + 4) / 4 * 4) * 8)};
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
  d.fbar_prev = (double *)ptrs[7]; d.C = (double *)ptrs[8];
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
  const size_t lds = run_lds_bytes(d.Mr, d.nd, d.ldc);
  const int use_lds = lds <= rom->max_dyn_lds;
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
