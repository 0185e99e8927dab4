// Implicit one-step schemes of the linear multistep residual (eq. "linKstep"
// with k = 1): r(xi) = xi - x_prev - dt (beta0 f(xi) + beta1 f(x_prev)).
// Newton's method on the increment D = xi - x_prev (keeps the small
// difference out of FP32 cancellation), each Newton system
// (I - dt beta0 J(xi)) d = -r solved by restarted GMRES whose matrix-vector
// products are the Jacobian-product pair kernel.  Krylov vectors live in
// HBM (FP32); dot products accumulate in FP64 on the device, and so does the
// small Hessenberg least-squares problem (Givens rotations, back
// substitution).  With
// the paper's inexact Jacobian the Newton systems are instead the per-body
// 2x2 blocks (I - dt beta0 B_i) d_i = -r_i, the blocks coming from the same
// pair pass as the velocity (fused velocity + block-Jacobian operation).
// For vectors of up to 16384 entries the residual and its norm are one
// kernel.  The Newton convergence test runs on the device; the host waits
// about once per Newton iteration with GMRES (when the Arnoldi steps it issued
// were enough) and about once per step with the block model.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

using namespace ptrom;

namespace {

// out = a + b
__global__ void add_kernel(int64_t m, float *__restrict__ out, const float *__restrict__ a,
                           const float *__restrict__ b) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < m) out[q] = a[q] + b[q];
}

// r = D - dt (b0 f + b1 fp) - dt (b0 + b1) u, u (background velocity) may be null
__global__ void residual_kernel(int64_t m, float *__restrict__ r, const float *__restrict__ D,
                                const float *__restrict__ f, const float *__restrict__ fp, float dtb0,
                                float dtb1, const float *__restrict__ u, float dtu) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < m) r[q] = D[q] - (dtb0 * f[q] + dtb1 * fp[q] + (u ? dtu * u[q] : 0.0f));
}

constexpr int kDotParts = 64;

// part[v][p] = sum over the p-th strided slice of X_v . y (FP64 accumulation);
// grid (kDotParts, nvec).
__global__ void __launch_bounds__(256)
    dot_partial_kernel(int64_t m, const float *__restrict__ X, int64_t ldx, const float *__restrict__ y,
                       double *__restrict__ part) {
  __shared__ double red[256];
  const float *x = X + (size_t)blockIdx.y * ldx;
  double s = 0.0;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < m; q += (int64_t)kDotParts * 256)
    s += (double)x[q] * (double)y[q];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.y * kDotParts + blockIdx.x] = red[0];
}

// out[v] = sum_p part[v][p], in a fixed order
__global__ void __launch_bounds__(64)
    dot_final_kernel(const double *__restrict__ part, double *__restrict__ out) {
  __shared__ double red[kDotParts];
  red[threadIdx.x] = part[blockIdx.x * kDotParts + threadIdx.x];
  __syncthreads();
  for (int w = kDotParts / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// Newton state of the current step on the device (block model): the squared
// norms of the first and latest residuals, the Newton iterations done, and
// done = 1 (converged) or 2 (iteration cap hit), 0 while iterating.  The
// host issues several iterations without waiting; an iteration issued after
// the step has finished changes nothing.
struct NewtonDev {
  double r0sq, rnsq, it, done;
};

// Update of the state from the latest residual's squared norm s (one thread):
// the first residual sets r0; converged when |r| <= tol |r0| or r0 = 0;
// otherwise the cap, otherwise one more iteration follows.
__device__ __forceinline__ void newton_update(NewtonDev *st, double s, double tol, int max_newton) {
  if (st->done != 0.0) return;
  if (st->r0sq < 0.0) st->r0sq = s;
  st->rnsq = s;
  if (st->r0sq == 0.0 || std::sqrt(s) <= tol * std::sqrt(st->r0sq))
    st->done = 1.0;
  else if (st->it >= double(max_newton))
    st->done = 2.0;
  else
    st->it += 1.0;
}

__global__ void newton_state_kernel(NewtonDev *st, const double *__restrict__ s, double tol, int max_newton) {
  if (threadIdx.x == 0 && blockIdx.x == 0) newton_update(st, s[0], tol, max_newton);
}

__global__ void newton_reset_kernel(NewtonDev *st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *st = NewtonDev{-1.0, 0.0, 0.0, 0.0};
}

// The paper's inexact Newton correction: per body, solve
// (I - c B_i) d_i = -r_i with B_i = [B0 B1; B2 B3] (layout [4][n]) by
// Cramer's rule in FP64, add d_i to the increment D and form the next
// iterate xi = x_prev + D.  With a device state, nothing changes once the
// step has finished.
__global__ void block_solve_kernel(int64_t n, float *__restrict__ D, float *__restrict__ xi,
                                   const float *__restrict__ xprev, const float *__restrict__ r,
                                   const float *__restrict__ B, float c, const NewtonDev *__restrict__ st) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (st && st->done != 0.0) return;
  const double cc = c;
  const double a00 = 1.0 - cc * B[i], a01 = -cc * B[n + i];
  const double a10 = -cc * B[2 * n + i], a11 = 1.0 - cc * B[3 * n + i];
  const double det = a00 * a11 - a01 * a10;
  const double bx = -(double)r[i], by = -(double)r[n + i];
  const float dx = (float)((double)D[i] + (bx * a11 - a01 * by) / det);
  const float dy = (float)((double)D[n + i] + (a00 * by - a10 * bx) / det);
  D[i] = dx;
  D[n + i] = dy;
  xi[i] = xprev[i] + dx;
  xi[n + i] = xprev[n + i] + dy;
}

// Start of a step: x_prev = x, D = 0, xi = x.
__global__ void step_start_kernel(int64_t m, float *__restrict__ xprev, float *__restrict__ D,
                                  float *__restrict__ xi, const float *__restrict__ x) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  const float v = x[q];
  xprev[q] = v;
  xi[q] = v;
  D[q] = 0.0f;
}

// out[v] = X_v . y for short vectors: one workgroup per vector, the whole
// sum in a fixed order (strided FP64 partials, then a tree over the block).
constexpr int64_t kShortDot = 16384;

__global__ void __launch_bounds__(256)
    dot_short_kernel(int64_t m, const float *__restrict__ X, int64_t ldx, const float *__restrict__ y,
                     double *__restrict__ out) {
  __shared__ double red[256];
  const float *x = X + (size_t)blockIdx.x * ldx;
  double s = 0.0;
  for (int64_t q = threadIdx.x; q < m; q += 256) s += (double)x[q] * (double)y[q];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

constexpr int kMaxRestart = 200;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One Arnoldi orthogonalisation for short vectors (m <= kFusedGS), in one
// workgroup with w held in LDS: classical Gram-Schmidt against V_0 .. V_k
// applied twice, the two coefficient sets to c1[0, k] and c2[0, k], |w|^2 to
// c2[k + 1], and V_{k+1} = w / |w| when |w| > 0.  Dot products are FP64
// (per-lane strided partials, then a butterfly over the wave); the update of
// each element adds the projections in vector order.
constexpr int kFusedGS = 12288;
constexpr int kGSThreads = 1024;

// GMRES state on the device: |b| of the Newton system, the current cycle's
// initial residual norm beta, the Arnoldi columns formed in this cycle and
// done = 1 once the cycle meets the tolerance (or the Krylov space is
// exhausted).  The Hessenberg matrix, the Givens rotations and the
// right-hand side g live next to it in device memory.
struct GmresDev {
  double bn, beta, kdone, done;
};

__device__ __forceinline__ bool gmres_idle(const NewtonDev *ns, const GmresDev *gs) {
  return (ns && ns->done != 0.0) || gs->done != 0.0;
}

// One whole Arnoldi step for short vectors (m <= kFusedGS), in one workgroup
// with w held in LDS: w = v_k - c Jv_k (Jv_k from the Jacobian-product
// kernel), classical Gram-Schmidt against V_0 .. V_k applied twice (the two
// coefficient sets to c1[0, k] and c2[0, k], |w|^2 to c2[k + 1]),
// V_{k+1} = w / |w| when |w| > 0, then the Hessenberg column, its Givens
// rotation and the convergence test (as arnoldi_kernel).  Dot products are
// FP64 (per-lane strided partials, then a butterfly over the wave); the
// update of each element adds the projections in vector order.
__device__ void arnoldi_column(int k, int R, GmresDev *gs, double *__restrict__ H, double *__restrict__ cs,
                               double *__restrict__ sn, double *__restrict__ g, const double *c1, const double *c2,
                               double hn2, double rtol);

__global__ void __launch_bounds__(kGSThreads)
    gs_fused_kernel(int m, int k, float *__restrict__ V, const float *__restrict__ jv, float c,
                    double *__restrict__ c1, double *__restrict__ c2, const NewtonDev *ns, GmresDev *gsd, int R,
                    double *__restrict__ H, double *__restrict__ gcs, double *__restrict__ gsn, double *__restrict__ gg,
                    double rtol) {
  constexpr int NW = kGSThreads / 64;
  __shared__ float wl[kFusedGS];
  __shared__ double cs[2][kMaxRestart + 1];
  __shared__ double red[NW];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (gmres_idle(ns, gsd)) return;
  const float *vk = V + (size_t)k * m;
  for (int q = tid; q < m; q += kGSThreads) wl[q] = vk[q] - c * jv[q];
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {
    double *cout = pass ? c2 : c1;
    for (int v = wv; v <= k; v += NW) {
      const float *x = V + (size_t)v * m;
      double s = 0.0;
      for (int q = lane; q < m; q += 64) s += (double)x[q] * (double)wl[q];
      s = wave_sum(s);
      if (lane == 0) {
        cs[pass][v] = s;
        cout[v] = s;
      }
    }
    __syncthreads();
    for (int q = tid; q < m; q += kGSThreads) {
      double s = 0.0;
      for (int v = 0; v <= k; ++v) s += cs[pass][v] * (double)V[(size_t)v * m + q];
      wl[q] = (float)((double)wl[q] - s);
    }
    __syncthreads();
  }
  double s = 0.0;
  for (int q = tid; q < m; q += kGSThreads) s += (double)wl[q] * (double)wl[q];
  s = wave_sum(s);
  if (lane == 0) red[wv] = s;
  __syncthreads();
  double nn = 0.0;
  for (int i = 0; i < NW; ++i) nn += red[i];
  if (tid == 0) {
    c2[k + 1] = nn;
    arnoldi_column(k, R, gsd, H, gcs, gsn, gg, cs[0], cs[1], nn, rtol);
  }
  if (nn > 0.0) {
    const float a = float(1.0 / sqrt(nn));
    float *out = V + (size_t)(k + 1) * m;
    for (int q = tid; q < m; q += kGSThreads) out[q] = a * wl[q];
  }
}

// The residual (as residual_kernel) and its squared norm for short vectors
// (m <= kShortDot): one workgroup, the norm summed as dot_short_kernel sums.
__global__ void __launch_bounds__(256)
    residual_norm_kernel(int64_t m, float *__restrict__ r, const float *__restrict__ D, const float *__restrict__ f,
                         const float *__restrict__ fp, float dtb0, float dtb1, const float *__restrict__ u, float dtu,
                         double *__restrict__ out, NewtonDev *st, double tol, int max_newton) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t q = threadIdx.x; q < m; q += 256) {
    const float v = D[q] - (dtb0 * f[q] + dtb1 * fp[q] + (u ? dtu * u[q] : 0.0f));
    r[q] = v;
    s += (double)v * (double)v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = red[0];
    if (st) newton_update(st, red[0], tol, max_newton);
  }
}

// One whole block-Newton iteration for short vectors (m <= kShortDot), in
// one workgroup: the residual and its squared norm (as residual_norm_kernel),
// the device state update, then, unless the step has finished, every body's
// 2x2 correction (as block_solve_kernel).
__global__ void __launch_bounds__(256)
    block_newton_kernel(int64_t n, float *__restrict__ r, float *__restrict__ D, float *__restrict__ xi,
                        const float *__restrict__ xprev, const float *__restrict__ f, const float *__restrict__ fp,
                        const float *__restrict__ B, float dtb0, float dtb1, const float *__restrict__ u, float dtu,
                        NewtonDev *st, double tol, int max_newton) {
  __shared__ double red[256];
  __shared__ int proceed;
  const int64_t m = 2 * n;
  if (threadIdx.x == 0) proceed = st->done == 0.0;
  __syncthreads();
  if (!proceed) return;
  double s = 0.0;
  for (int64_t q = threadIdx.x; q < m; q += 256) {
    const float v = D[q] - (dtb0 * f[q] + dtb1 * fp[q] + (u ? dtu * u[q] : 0.0f));
    r[q] = v;
    s += (double)v * (double)v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    newton_update(st, red[0], tol, max_newton);
    proceed = st->done == 0.0;
  }
  __syncthreads();
  if (!proceed) return;
  const double cc = dtb0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double a00 = 1.0 - cc * B[i], a01 = -cc * B[n + i];
    const double a10 = -cc * B[2 * n + i], a11 = 1.0 - cc * B[3 * n + i];
    const double det = a00 * a11 - a01 * a10;
    const double bx = -(double)r[i], by = -(double)r[n + i];
    const float dx = (float)((double)D[i] + (bx * a11 - a01 * by) / det);
    const float dy = (float)((double)D[n + i] + (a00 * by - a10 * bx) / det);
    D[i] = dx;
    D[n + i] = dy;
    xi[i] = xprev[i] + dx;
    xi[n + i] = xprev[n + i] + dy;
  }
}

// y -= sum_v c[v] X_v  (c on the device), or y = scale * y + sum_v c[v] X_v when accumulate.
__global__ void multi_axpy_kernel(int64_t m, int nvec, const float *__restrict__ X, int64_t ldx,
                                  const double *__restrict__ c, float sign, float *__restrict__ y) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  double s = 0.0;
  for (int v = 0; v < nvec; ++v) s += c[v] * (double)X[(size_t)v * ldx + q];
  y[q] = (float)((double)y[q] + sign * s);
}

__global__ void scale_kernel(int64_t m, float *__restrict__ out, const float *__restrict__ x, float a) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < m) out[q] = a * x[q];
}

__global__ void lincomb_kernel(int64_t m, float *__restrict__ out, const float *__restrict__ v,
                               float c, const float *__restrict__ w) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < m) out[q] = v[q] - c * w[q];
}

// Start of a GMRES cycle: beta = sqrt(sq[0]); the first cycle also takes
// |b| = beta.  A later cycle is done at once when beta <= rtol |b|.
__global__ void gmres_init_kernel(GmresDev *gs, double *__restrict__ g, int R, const double *__restrict__ sq,
                                  int first, double rtol, const NewtonDev *ns) {
  if (threadIdx.x != 0 || (ns && ns->done != 0.0)) return;
  const double beta = std::sqrt(sq[0]);
  if (first) gs->bn = beta;
  gs->beta = beta;
  gs->kdone = 0.0;
  gs->done = (beta == 0.0 || (!first && beta <= rtol * gs->bn)) ? 1.0 : 0.0;
  g[0] = beta;
  for (int i = 1; i <= R; ++i) g[i] = 0.0;
}

// out = in / beta (V_0 of a cycle)
__global__ void scale_beta_kernel(int64_t m, float *__restrict__ out, const float *__restrict__ in,
                                  const GmresDev *gs, const NewtonDev *ns) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m || gmres_idle(ns, gs)) return;
  out[q] = float(1.0 / gs->beta) * in[q];
}

// V_{k+1} = w / |w| from |w|^2 on the device (separate Gram-Schmidt path)
__global__ void scale_norm_kernel(int64_t m, float *__restrict__ out, const float *__restrict__ w,
                                  const double *__restrict__ nsq, const GmresDev *gs, const NewtonDev *ns) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m || gmres_idle(ns, gs) || !(nsq[0] > 0.0)) return;
  out[q] = float(1.0 / std::sqrt(nsq[0])) * w[q];
}

// Column k of the Hessenberg matrix from both Gram-Schmidt passes and |w|^2,
// the earlier Givens rotations applied to it, a new rotation, the updated
// right-hand side g and the convergence test |g_{k+1}| <= rtol |b|.  H is
// row-major [R + 1][R].  One thread.
__device__ void arnoldi_column(int k, int R, GmresDev *gs, double *__restrict__ H, double *__restrict__ cs,
                               double *__restrict__ sn, double *__restrict__ g, const double *c1, const double *c2,
                               double hn2, double rtol) {
  const double hn = std::sqrt(hn2);
  for (int i = 0; i <= k; ++i) H[i * R + k] = c1[i] + c2[i];
  H[(k + 1) * R + k] = hn;
  for (int i = 0; i < k; ++i) {
    const double a = H[i * R + k], b = H[(i + 1) * R + k];
    H[i * R + k] = cs[i] * a + sn[i] * b;
    H[(i + 1) * R + k] = -sn[i] * a + cs[i] * b;
  }
  const double a = H[k * R + k], b = H[(k + 1) * R + k];
  const double rr = std::sqrt(a * a + b * b);
  cs[k] = rr == 0.0 ? 1.0 : a / rr;
  sn[k] = rr == 0.0 ? 0.0 : b / rr;
  H[k * R + k] = rr;
  H[(k + 1) * R + k] = 0.0;
  g[k + 1] = -sn[k] * g[k];
  g[k] = cs[k] * g[k];
  gs->kdone = double(k + 1);
  if (std::fabs(g[k + 1]) <= rtol * gs->bn || hn == 0.0) gs->done = 1.0;
}

__global__ void arnoldi_kernel(int k, int R, GmresDev *gs, double *__restrict__ H, double *__restrict__ cs,
                               double *__restrict__ sn, double *__restrict__ g, const double *__restrict__ c1,
                               const double *__restrict__ c2, double rtol, const NewtonDev *ns) {
  if (threadIdx.x != 0 || gmres_idle(ns, gs)) return;
  arnoldi_column(k, R, gs, H, cs, sn, g, c1, c2, c2[k + 1], rtol);
}

// y = R^{-1} g over the kdone columns of this cycle (back substitution)
__global__ void gmres_solve_kernel(int R, const GmresDev *gs, const double *__restrict__ H,
                                   const double *__restrict__ g, double *__restrict__ y, const NewtonDev *ns) {
  if (threadIdx.x != 0 || (ns && ns->done != 0.0)) return;
  const int k = int(gs->kdone);
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int j = i + 1; j < k; ++j) s -= H[i * R + j] * y[j];
    y[i] = s / H[i * R + i];
  }
}

// d += sum_{v < kdone} y[v] V_v
__global__ void update_kernel(int64_t m, const float *__restrict__ V, const double *__restrict__ y,
                              const GmresDev *gs, const NewtonDev *ns, float *__restrict__ d) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m || (ns && ns->done != 0.0)) return;
  const int k = int(gs->kdone);
  double s = 0.0;
  for (int v = 0; v < k; ++v) s += y[v] * (double)V[(size_t)v * m + q];
  d[q] = (float)((double)d[q] + s);
}

inline dim3 g1(int64_t m) { return dim3((unsigned)((m + 255) / 256)); }

// Matrix-free GMRES for (I - c J(xi)) d = b.  The Gram-Schmidt coefficients,
// the Hessenberg matrix, the Givens rotations and the convergence test stay
// on the device; the host reads the small state once per batch of Arnoldi
// steps.
struct Solver {
  ptrom_ctx *ctx;
  hipStream_t st;
  int64_t n, m;
  const float *gamma;
  float delta;
  PairCfg jcfg;
  float *pws;
  size_t pwsf;
  float *xi, *tmp, *w, *V;
  double *dd;     // device: |r|^2, then the coefficients [restart + 1] twice and |w|^2
  double *hp;     // pinned host scratch (the state copies at hp + 3 restart + 4)
  double *dot_part;
  int restart;

  // w = (I - c J(xi)) v
  int apply(const float *v, float c, float *out) {
    hipError_t e = launch_pair(OP_JVP, jcfg, ctx->num_cus, n, xi, gamma, v, delta, tmp, nullptr,
                               pws, pwsf, st);
    if (e != hipSuccess) return ctx->hip_fail(e, "jvp");
    hipLaunchKernelGGL(lincomb_kernel, g1(m), dim3(256), 0, st, m, out, v, c, tmp);
    return PTROM_OK;
  }

  // dev[v] = X_v . y for v < nvec (stays on the device)
  void dots(const float *X, int nvec, const float *y, double *dev) {
    if (m <= kShortDot) {
      hipLaunchKernelGGL(dot_short_kernel, dim3(nvec), dim3(256), 0, st, m, X, m, y, dev);
      return;
    }
    hipLaunchKernelGGL(dot_partial_kernel, dim3(kDotParts, nvec), dim3(256), 0, st, m, X, m, y, dot_part);
    hipLaunchKernelGGL(dot_final_kernel, dim3(nvec), dim3(kDotParts), 0, st, dot_part, dev);
  }

  // The residual, its squared norm and the device Newton state update, with
  // no host wait.
  void residual_state(float *r, const float *D, const float *f, const float *fp, float dtb0, float dtb1,
                      const float *u, float dtu, NewtonDev *ns, double tol, int max_newton) {
    if (m <= kShortDot) {
      hipLaunchKernelGGL(residual_norm_kernel, dim3(1), dim3(256), 0, st, m, r, D, f, fp, dtb0, dtb1, u, dtu, dd, ns,
                         tol, max_newton);
      return;
    }
    hipLaunchKernelGGL(residual_kernel, g1(m), dim3(256), 0, st, m, r, D, f, fp, dtb0, dtb1, u, dtu);
    dots(r, 1, r, dd);
    hipLaunchKernelGGL(newton_state_kernel, dim3(1), dim3(64), 0, st, ns, dd, tol, max_newton);
  }

  // Device GMRES state: GmresDev, then H [(R + 1) R], cs [R], sn [R], g [R + 1], y [R].
  GmresDev *gsd;
  double *H, *gcs, *gsn, *gg, *gy;

  // Host copies of both device states (one wait).
  int fetch_states(const NewtonDev *ns, NewtonDev *hn, GmresDev *hg) {
    double *h = hp + (3 * restart + 4);
    PTROM_CHECK_HIP(ctx, hipMemcpyAsync(h, ns, sizeof(NewtonDev), hipMemcpyDeviceToHost, st));
    PTROM_CHECK_HIP(ctx, hipMemcpyAsync(h + 4, gsd, sizeof(GmresDev), hipMemcpyDeviceToHost, st));
    PTROM_CHECK_HIP(ctx, hipStreamSynchronize(st));
    std::memcpy(hn, h, sizeof(NewtonDev));
    std::memcpy(hg, h + 4, sizeof(GmresDev));
    return PTROM_OK;
  }

  // Solve (I - c J) d = b from d = 0 to relative tolerance rtol by restarted
  // GMRES whose Hessenberg matrix, rotations and convergence test stay on the
  // device.  |b|^2 is in dd[0] (the Newton residual's).  The host issues
  // `predict` Arnoldi steps (more if needed) and then reads the state once;
  // steps issued after convergence change nothing.  Nothing runs when the
  // Newton state says the step has finished (*newton_done then true).
  // *used = Jacobian products that counted, *cols = Arnoldi columns of the
  // first cycle.
  int gmres(const float *b, float *d, float c, double rtol, int maxit, int predict, const NewtonDev *ns,
            NewtonDev *hns, bool *newton_done, int *used, int *cols) {
    *used = 0;
    *cols = 0;
    *newton_done = false;
    const int R = restart;
    double *d1 = dd, *d2 = dd + (R + 1);
    hipLaunchKernelGGL(scale_kernel, g1(m), dim3(256), 0, st, m, d, b, 0.0f);
    hipLaunchKernelGGL(gmres_init_kernel, dim3(1), dim3(64), 0, st, gsd, gg, R, dd, 1, rtol, ns);
    hipLaunchKernelGGL(scale_beta_kernel, g1(m), dim3(256), 0, st, m, V, b, gsd, ns);
    int issued = 0;
    for (int cycle = 0;; ++cycle) {
      GmresDev hg{};
      int k = 0;
      for (;;) {
        const int batch = k == 0 ? std::max(1, predict) : std::max(1, predict / 2);
        for (int q = 0; q < batch && k < R && issued < maxit; ++q, ++k, ++issued) {
          float *vk = V + (size_t)k * m;
          if (m <= kFusedGS) {
            // the Jacobian product, then one kernel for the rest of the step
            const hipError_t e = launch_pair(OP_JVP, jcfg, ctx->num_cus, n, xi, gamma, vk, delta, tmp, nullptr, pws,
                                             pwsf, st);
            if (e != hipSuccess) return ctx->hip_fail(e, "jvp");
            hipLaunchKernelGGL(gs_fused_kernel, dim3(1), dim3(kGSThreads), 0, st, int(m), k, V, tmp, c, d1, d2, ns,
                               gsd, R, H, gcs, gsn, gg, rtol);
            continue;
          }
          if (int rc = apply(vk, c, w)) return rc;
          {
            // classical Gram-Schmidt, applied twice, coefficients on the device
            dots(V, k + 1, w, d1);
            hipLaunchKernelGGL(multi_axpy_kernel, g1(m), dim3(256), 0, st, m, k + 1, V, m, d1, -1.0f, w);
            dots(V, k + 1, w, d2);
            hipLaunchKernelGGL(multi_axpy_kernel, g1(m), dim3(256), 0, st, m, k + 1, V, m, d2, -1.0f, w);
            dots(w, 1, w, d2 + (k + 1));
            hipLaunchKernelGGL(scale_norm_kernel, g1(m), dim3(256), 0, st, m, V + (size_t)(k + 1) * m, w,
                               d2 + (k + 1), gsd, ns);
            hipLaunchKernelGGL(arnoldi_kernel, dim3(1), dim3(64), 0, st, k, R, gsd, H, gcs, gsn, gg, d1, d2, rtol,
                               ns);
          }
        }
        if (int rc = fetch_states(ns, hns, &hg)) return rc;
        if (hns->done != 0.0) {
          *newton_done = true;
          return PTROM_OK;
        }
        if (hg.done != 0.0 || k >= R || issued >= maxit) break;
      }
      const int kd = int(hg.kdone);
      *used += kd;
      if (cycle == 0) *cols = kd;
      hipLaunchKernelGGL(gmres_solve_kernel, dim3(1), dim3(64), 0, st, R, gsd, H, gg, gy, ns);
      hipLaunchKernelGGL(update_kernel, g1(m), dim3(256), 0, st, m, V, gy, gsd, ns, d);
      if (hg.done != 0.0 || issued >= maxit) break;
      // restart from the true residual b - A d
      if (int rc = apply(d, c, w)) return rc;
      ++issued;
      ++*used;
      hipLaunchKernelGGL(lincomb_kernel, g1(m), dim3(256), 0, st, m, w, b, 1.0f, w);  // w = b - A d
      dots(w, 1, w, dd);
      hipLaunchKernelGGL(gmres_init_kernel, dim3(1), dim3(64), 0, st, gsd, gg, R, dd, 0, rtol, ns);
      hipLaunchKernelGGL(scale_beta_kernel, g1(m), dim3(256), 0, st, m, V, w, gsd, ns);
      if (int rc = fetch_states(ns, hns, &hg)) return rc;
      if (hg.done != 0.0) break;
    }
    return PTROM_OK;
  }
};

}  // namespace

extern "C" int ptrom_implicit_forced(ptrom_ctx *ctx, int64_t n, float *xy, const float *gamma, float delta,
                                     const float *uinf, float dt, int nsteps, int scheme,
                                     const ptrom_newton_opts *opts, ptrom_newton_stats *stats,
                                     ptrom_stream stream) {
  if (!ctx) return PTROM_EINVAL;
  ctx->err.clear();
  if (n < 1 || n > kMaxN) return ctx->fail(PTROM_EINVAL, "n must be in [1, 2^30]");
  if (!(delta >= 0.0f) || !(dt > 0.0f) || nsteps < 0) return ctx->fail(PTROM_EINVAL, "bad delta/dt/nsteps");
  if (!xy || !gamma) return ctx->fail(PTROM_EINVAL, "NULL array");
  if (scheme != PTROM_BACKWARD_EULER && scheme != PTROM_TRAPEZOID) return ctx->fail(PTROM_EINVAL, "bad scheme");
  ptrom_newton_opts o{1e-6, 20, 20, 60, PTROM_NEWTON_GMRES, 1e-3, 0, 0};
  if (opts) o = *opts;
  if (o.gmres_restart < 1 || o.gmres_restart > kMaxRestart || o.max_newton < 0 || o.gmres_maxit < 1 ||
      (o.linear_solver != PTROM_NEWTON_GMRES && o.linear_solver != PTROM_NEWTON_BLOCK) || o.jac_period < 0)
    return ctx->fail(PTROM_EINVAL, "bad Newton/GMRES options");
  const bool block = o.linear_solver == PTROM_NEWTON_BLOCK;
  if (hipSetDevice(ctx->device) != hipSuccess) return ctx->fail(PTROM_EHIP, "hipSetDevice");
  ptrom_newton_stats stl{};
  const int64_t m = 2 * n;
  const float b0 = scheme == PTROM_BACKWARD_EULER ? 1.0f : 0.5f;
  const float b1 = scheme == PTROM_BACKWARD_EULER ? 0.0f : 0.5f;
  const PairCfg vcfg = ctx->tune.get(OP_VEL, n), jcfg = ctx->tune.get(OP_JVP, n);
  const PairCfg bcfg = ctx->tune.get(OP_VBJ, n);
  const size_t pwsf = std::max({pair_ws_floats(OP_VEL, vcfg, ctx->num_cus, n),
                                pair_ws_floats(OP_JVP, jcfg, ctx->num_cus, n),
                                block ? pair_ws_floats(OP_VBJ, bcfg, ctx->num_cus, n) : size_t(0)});
  const int R = o.gmres_restart;
  const size_t vb = align256(m * sizeof(float));
  const size_t need = vb * (9 + R + 1) + align256(pwsf * sizeof(float)) + align256(sizeof(double) * (3 * R + 4)) +
                      align256(sizeof(double) * (R + 2) * kDotParts) + align256(4 * n * sizeof(float)) +
                      align256(sizeof(NewtonDev)) + align256(sizeof(double) * (4 + (R + 1) * R + 4 * R + 1)) +
                      1024;
  if (int rc = ctx->reserve(need)) return rc;
  Carver cv{static_cast<char *>(ctx->ws), ctx->ws_bytes};
  float *xprev = cv.take<float>(m), *D = cv.take<float>(m), *xi = cv.take<float>(m);
  float *f = cv.take<float>(m), *fp = cv.take<float>(m), *r = cv.take<float>(m);
  float *tmp = cv.take<float>(m), *d = cv.take<float>(m), *w = cv.take<float>(m);
  float *V = cv.take<float>(m * (R + 1));
  float *pws = cv.take<float>(pwsf ? pwsf : 1);
  double *dd = cv.take<double>(3 * R + 4);
  double *dpart = cv.take<double>(size_t(R + 2) * kDotParts);
  float *Bj = cv.take<float>(4 * n);
  NewtonDev *nst = cv.take<NewtonDev>(1);
  GmresDev *gdev = reinterpret_cast<GmresDev *>(cv.take<double>(4 + size_t(R + 1) * R + 4 * size_t(R) + 1));
  if (!w || !V || !pws || !dd || !dpart || !Bj || !nst || !gdev) return ctx->fail(PTROM_ENOMEM, "workspace carve");
  double *hp = ctx->pinned_doubles(3 * R + 12);  // the Newton and GMRES state copies at 3 R + 4
  if (!hp) return ctx->fail(PTROM_ENOMEM, "pinned host scratch");
  hipStream_t st = (hipStream_t)stream;
  Solver S{ctx, st, n, m, gamma, delta, jcfg, pws, pwsf, xi, tmp, w, V, dd, hp, dpart, R};
  S.gsd = gdev;
  S.H = reinterpret_cast<double *>(gdev + 1);
  S.gcs = S.H + (R + 1) * R;
  S.gsn = S.gcs + R;
  S.gg = S.gsn + R;
  S.gy = S.gg + (R + 1);

  // velocity at x (and, for the block model, the self blocks in the same pass)
  auto rhs = [&](const float *x, float *fo, bool blocks) -> int {
    const hipError_t e = blocks ? launch_pair(OP_VBJ, bcfg, ctx->num_cus, n, x, gamma, nullptr, delta, fo, Bj,
                                              pws, pwsf, st)
                                : launch_pair(OP_VEL, vcfg, ctx->num_cus, n, x, gamma, nullptr, delta, fo, nullptr,
                                              pws, pwsf, st);
    return e == hipSuccess ? PTROM_OK : ctx->hip_fail(e, blocks ? "velocity and block jacobian" : "velocity");
  };
  // Block model: the convergence test runs on the device, and the host issues
  // as many Newton iterations as the previous step needed (plus the final
  // residual) before it reads the state once; iterations issued beyond the
  // step's end change nothing.
  int predicted = 2;
  for (int step = 0; block && step < nsteps; ++step) {
    hipLaunchKernelGGL(step_start_kernel, g1(m), dim3(256), 0, st, m, xprev, D, xi, xy);
    hipLaunchKernelGGL(newton_reset_kernel, dim3(1), dim3(64), 0, st, nst);
    const bool refresh = o.jac_period == 0 || step % o.jac_period == 0;
    if (int rc = rhs(xprev, fp, refresh)) return rc;
    int issued = 0;
    NewtonDev hs{};
    for (;;) {
      const int batch = issued == 0 ? predicted : std::max(1, predicted / 4);
      for (int q = 0; q < batch && issued <= o.max_newton; ++q, ++issued) {
        if (issued > 0)
          if (int rc = rhs(xi, f, o.jac_period == 0)) return rc;
        const float *fc = issued == 0 ? fp : f;
        if (m <= kShortDot) {
          hipLaunchKernelGGL(block_newton_kernel, dim3(1), dim3(256), 0, st, n, r, D, xi, xprev, fc, fp, Bj, dt * b0,
                             dt * b1, uinf, dt * (b0 + b1), nst, o.newton_tol, o.max_newton);
          continue;
        }
        S.residual_state(r, D, fc, fp, dt * b0, dt * b1, uinf, dt * (b0 + b1), nst, o.newton_tol, o.max_newton);
        hipLaunchKernelGGL(block_solve_kernel, g1(n), dim3(256), 0, st, n, D, xi, xprev, r, Bj, dt * b0, nst);
      }
      double *hst = hp + (3 * R + 4);
      PTROM_CHECK_HIP(ctx, hipMemcpyAsync(hst, nst, sizeof(NewtonDev), hipMemcpyDeviceToHost, st));
      PTROM_CHECK_HIP(ctx, hipStreamSynchronize(st));
      std::memcpy(&hs, hst, sizeof(NewtonDev));
      if (hs.done != 0.0 || issued > o.max_newton) break;
    }
    const int it = int(hs.it);
    if (hs.done != 1.0) stl.nonconverged_steps++;
    stl.newton_iters += it;
    const double rel = hs.r0sq > 0.0 ? std::sqrt(hs.rnsq / hs.r0sq) : 0.0;
    if (rel > stl.max_final_rel_residual) stl.max_final_rel_residual = rel;
    predicted = it + 1;
    hipLaunchKernelGGL(add_kernel, g1(m), dim3(256), 0, st, m, xy, xprev, D);
  }
  // GMRES model: the Newton test runs on the device too.  The host issues an
  // iteration's GMRES without waiting for its residual while the step is
  // expected to continue (fewer iterations than the previous step took), and
  // reads both states once per Newton iteration.
  // (speculative Arnoldi steps are cheap for short vectors; for long ones a
  // wasted Jacobian product costs far more than a wait, so start from one)
  int predicted_newton = 1, predicted_cols = m <= kFusedGS ? 4 : 1;
  for (int step = 0; !block && step < nsteps; ++step) {
    hipLaunchKernelGGL(step_start_kernel, g1(m), dim3(256), 0, st, m, xprev, D, xi, xy);
    hipLaunchKernelGGL(newton_reset_kernel, dim3(1), dim3(64), 0, st, nst);
    if (int rc = rhs(xprev, fp, false)) return rc;
    NewtonDev hs{};
    for (int it = 0;; ++it) {
      if (it > 0) {
        hipLaunchKernelGGL(add_kernel, g1(m), dim3(256), 0, st, m, xi, xprev, D);  // xi = x_prev + D
        if (int rc = rhs(xi, f, false)) return rc;
      }
      S.residual_state(r, D, it == 0 ? fp : f, fp, dt * b0, dt * b1, uinf, dt * (b0 + b1), nst, o.newton_tol,
                       o.max_newton);
      if (it >= predicted_newton) {
        GmresDev hg{};
        if (int rc = S.fetch_states(nst, &hs, &hg)) return rc;
        if (hs.done != 0.0) break;
      }
      hipLaunchKernelGGL(scale_kernel, g1(m), dim3(256), 0, st, m, r, r, -1.0f);
      int used = 0, cols = 0;
      bool newton_done = false;
      if (int rc = S.gmres(r, d, dt * b0, o.gmres_tol, o.gmres_maxit, predicted_cols, nst, &hs, &newton_done, &used,
                           &cols))
        return rc;
      if (newton_done) break;
      stl.krylov_iters += used;
      if (cols > 0) predicted_cols = cols;
      hipLaunchKernelGGL(add_kernel, g1(m), dim3(256), 0, st, m, D, D, d);
    }
    const int it = int(hs.it);
    if (hs.done != 1.0) stl.nonconverged_steps++;
    stl.newton_iters += it;
    const double rel = hs.r0sq > 0.0 ? std::sqrt(hs.rnsq / hs.r0sq) : 0.0;
    if (rel > stl.max_final_rel_residual) stl.max_final_rel_residual = rel;
    predicted_newton = it;
    hipLaunchKernelGGL(add_kernel, g1(m), dim3(256), 0, st, m, xy, xprev, D);
  }
  PTROM_CHECK_HIP(ctx, hipGetLastError());
  PTROM_CHECK_HIP(ctx, hipStreamSynchronize(st));
  if (stats) *stats = stl;
  return stl.nonconverged_steps ? PTROM_ENOCONV : PTROM_OK;
}

extern "C" int ptrom_implicit(ptrom_ctx *ctx, int64_t n, float *xy, const float *gamma, float delta,
                              float dt, int nsteps, int scheme, const ptrom_newton_opts *opts,
                              ptrom_newton_stats *stats, ptrom_stream stream) {
  return ptrom_implicit_forced(ctx, n, xy, gamma, delta, nullptr, dt, nsteps, scheme, opts, stats, stream);
}
