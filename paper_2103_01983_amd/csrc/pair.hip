// All-pairs kernels of the regularized 2D Biot-Savart sum (kernel equation
// of the problem formulation) and its derivatives: velocity, per-body 2x2
// self blocks (the paper's inexact Jacobian), both in one pass, the
// Jacobian-vector product, the vector-Jacobian product with the circulation
// gradient, and the stream function of the Hamiltonian.
//
// Work decomposition: a workgroup of 4 wave64 owns 256*K consecutive targets
// (K per lane, kept in VGPRs) and one contiguous chunk of sources (grid.y
// splits the sources so that small N still fills 256 CUs).  Sources arrive
// either through LDS tiles (cooperative coalesced loads, broadcast reads) or
// through the scalar cache (wave-uniform loads feeding SGPR operands); both
// are FP32 vector-ALU bound.  Each target accumulates a plain FP32 partial
// per 256-source tile and adds it to a Kahan-compensated running sum.  With
// more than one source chunk, the chunks' compensated sums go to a
// workspace and a second kernel adds them in chunk order, so results are
// bitwise reproducible.  Self pairs are removed by index in the tiles that
// overlap the workgroup's targets (needed for delta = 0).
#include <algorithm>

#include "pair_core.h"

namespace ptrom {
namespace {

template <int OP, int K, int STAGING>
__global__ void __launch_bounds__(kBlock)
    pair_kernel(int n, const float *__restrict__ xy, const float *__restrict__ gam,
                const float *__restrict__ aux, float d2, int chunk, int partial,
                float *__restrict__ out, float *__restrict__ out2) {
  constexpr int NA = Traits<OP>::NACC;
  __shared__ float lds[STAGING == STAGE_LDS ? Traits<OP>::NSRC * kTile : 1];
  const int tgt0 = blockIdx.x * (kBlock * K);
  const int sb = blockIdx.y * chunk;
  const int se = min(n, sb + chunk);
  float res[K][NA];
  pair_block<OP, K, STAGING>(n, xy, gam, aux, d2, tgt0, sb, se, lds, res);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = tgt0 + k * kBlock + threadIdx.x;
    if (i >= n) continue;
    if (partial) {
#pragma unroll
      for (int a = 0; a < NA; ++a) out[(size_t)(blockIdx.y * NA + a) * n + i] = res[k][a];
    } else {
      store_final<OP>(n, i, res[k], out, out2);
    }
  }
}

// Adds the per-chunk partials in chunk order (compensated) and stores.  The
// partials are loaded kRedBatch chunks at a time, all loads issued before the
// additions, so a small launch waits on a few memory round trips rather than
// one per chunk; the order of the additions is the chunk order.
constexpr int kRedBatch = 8;

template <int OP>
__global__ void __launch_bounds__(256)
    reduce_kernel(int n, int nsplit, const float *__restrict__ ws, float *__restrict__ out,
                  float *__restrict__ out2) {
  constexpr int NA = Traits<OP>::NACC;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s[NA], c[NA];
#pragma unroll
  for (int a = 0; a < NA; ++a) s[a] = c[a] = 0.0f;
  for (int p0 = 0; p0 < nsplit; p0 += kRedBatch) {
    const int cnt = min(kRedBatch, nsplit - p0);
    float t[kRedBatch][NA];
#pragma unroll
    for (int u = 0; u < kRedBatch; ++u)
#pragma unroll
      for (int a = 0; a < NA; ++a) t[u][a] = u < cnt ? ws[(size_t)((p0 + u) * NA + a) * n + i] : 0.0f;
#pragma unroll
    for (int u = 0; u < kRedBatch; ++u)
      if (u < cnt) {
#pragma unroll
        for (int a = 0; a < NA; ++a) kahan_add(s[a], c[a], t[u][a]);
      }
  }
  float v[NA];
#pragma unroll
  for (int a = 0; a < NA; ++a) v[a] = s[a] - c[a];
  store_final<OP>(n, i, v, out, out2);
}

// Velocity at arbitrary points: kPtsK points per lane, sources read at
// wave-uniform addresses (full tiles unrolled so the scalar loads batch),
// 256-source tiles added with Kahan compensation.
// blockIdx.y takes sources [y chunk, (y + 1) chunk); with several chunks
// each writes its unscaled partial sums to out[(2 y + a) nt + t], added in
// chunk order by reduce_kernel<OP_VEL>.
constexpr int kPtsK = 4;  // field points per lane

__global__ void __launch_bounds__(kBlock)
    points_velocity_kernel(int nt, const float *__restrict__ p, int n, const float *__restrict__ xy,
                           const float *__restrict__ gam, float d2, int chunk, int partial,
                           float *__restrict__ out) {
  constexpr int K = kPtsK;
  float tg[K][2];
  const int t0 = blockIdx.x * (kBlock * K);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int t = t0 + k * kBlock + threadIdx.x;
    const int tc = t < nt ? t : nt - 1;
    tg[k][0] = p[tc];
    tg[k][1] = p[nt + tc];
  }
  float sum[K][2] = {}, cmp[K][2] = {};
  const int sb = blockIdx.y * chunk, se = min(n, sb + chunk);
  for (int ts = sb; ts < se; ts += kTile) {
    const int cnt = min(kTile, se - ts);
    float part[K][2] = {};
    if (cnt == kTile) {
#pragma unroll 4
      for (int jj = 0; jj < kTile; ++jj) {
        const float s[3] = {xy[ts + jj], xy[n + ts + jj], gam[ts + jj]};
#pragma unroll
        for (int k = 0; k < K; ++k) interact<OP_VEL, false>(tg[k], s, d2, part[k], false);
      }
    } else {
      for (int jj = 0; jj < cnt; ++jj) {
        const float s[3] = {xy[ts + jj], xy[n + ts + jj], gam[ts + jj]};
#pragma unroll
        for (int k = 0; k < K; ++k) interact<OP_VEL, false>(tg[k], s, d2, part[k], false);
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      kahan_add(sum[k][0], cmp[k][0], part[k][0]);
      kahan_add(sum[k][1], cmp[k][1], part[k][1]);
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int t = t0 + k * kBlock + threadIdx.x;
    if (t < nt) {
      if (partial) {
        out[(size_t)(2 * blockIdx.y) * nt + t] = sum[k][0] - cmp[k][0];
        out[(size_t)(2 * blockIdx.y + 1) * nt + t] = sum[k][1] - cmp[k][1];
      } else {
        out[t] = (sum[k][0] - cmp[k][0]) * kInv2Pi;
        out[nt + t] = (sum[k][1] - cmp[k][1]) * kInv2Pi;
      }
    }
  }
}

template <int OP>
hipError_t dispatch(const PairCfg &cfg, dim3 grid, hipStream_t st, int n, const float *xy,
                    const float *gam, const float *aux, float d2, int chunk, int partial,
                    float *out, float *out2) {
#define PTROM_LAUNCH(KK, SS)                                                                     \
  hipLaunchKernelGGL((pair_kernel<OP, KK, SS>), grid, dim3(kBlock), 0, st, n, xy, gam, aux, d2, \
                     chunk, partial, out, out2)
  if (cfg.staging == STAGE_LDS) {
    if (cfg.k == 1) PTROM_LAUNCH(1, STAGE_LDS);
    else if (cfg.k == 2) PTROM_LAUNCH(2, STAGE_LDS);
    else PTROM_LAUNCH(4, STAGE_LDS);
  } else {
    if (cfg.k == 1) PTROM_LAUNCH(1, STAGE_SCALAR);
    else if (cfg.k == 2) PTROM_LAUNCH(2, STAGE_SCALAR);
    else PTROM_LAUNCH(4, STAGE_SCALAR);
  }
#undef PTROM_LAUNCH
  return hipGetLastError();
}

// Plain FP64 velocity: one target per thread, IEEE division, sequential sum.
__global__ void __launch_bounds__(256)
    velocity_f64_kernel(int n, const double *__restrict__ xy, const double *__restrict__ gam,
                        double d2, double *__restrict__ f) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double xi = xy[i], yi = xy[n + i];
  double sx = 0.0, sy = 0.0;
  for (int j = 0; j < n; ++j) {
    const double dx = xi - xy[j], dy = yi - xy[n + j];
    const double s = dx * dx + dy * dy + d2;
    const double g = (j == i) ? 0.0 : gam[j] / s;
    sx += -dy * g;
    sy += dx * g;
  }
  const double inv2pi = 0.15915494309189533576888376337251;
  f[i] = sx * inv2pi;
  f[n + i] = sy * inv2pi;
}

__global__ void axpy_kernel(int64_t m, float *__restrict__ out, const float *__restrict__ x, float a,
                            const float *__restrict__ y) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < m) out[q] = fmaf(a, y[q], x[q]);
}

__global__ void rk4_combine_kernel(int64_t m, float *__restrict__ x, const float *__restrict__ k1,
                                   const float *__restrict__ k2, const float *__restrict__ k3,
                                   const float *__restrict__ k4, float h6) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < m) x[q] = fmaf(h6, (k1[q] + k4[q]) + 2.0f * (k2[q] + k3[q]), x[q]);
}

__global__ void axpy_f64_kernel(int64_t m, double *__restrict__ out, const double *__restrict__ x,
                                double a, const double *__restrict__ y) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < m) out[q] = x[q] + a * y[q];
}

__global__ void rk4_combine_f64_kernel(int64_t m, double *__restrict__ x,
                                       const double *__restrict__ k1, const double *__restrict__ k2,
                                       const double *__restrict__ k3, const double *__restrict__ k4,
                                       double h) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < m) x[q] += h / 6.0 * (k1[q] + 2.0 * k2[q] + 2.0 * k3[q] + k4[q]);
}

}  // namespace

int size_class(int64_t n) {
  int c = 0;
  while ((int64_t(1) << (c + 1)) <= n && c < 30) ++c;
  return c < 8 ? 8 : (c > 24 ? 24 : c);
}

PairCfg large_n_cfg() {
  PairCfg c;
  c.staging = STAGE_LDS;
  c.k = 2;
  c.waves_per_simd = 8;
  c.sym = 0;
  return c;
}

PairCfg Tuning::get(int op, int64_t n) const {
  PairCfg c = get_table(op, n);
  if (c.sym && uint64_t(pair_sym_ws_floats(op, c.k, n)) * sizeof(float) > ws_cap_bytes) c = large_n_cfg();
  return c;
}

PairCfg Tuning::get_batched(int64_t nbar) const {
  // nearest tuned class; without any batched entry K = 2, 8 workgroups per CU
  PairCfg c = get_table(OP_BATCH, nbar);
  c.staging = STAGE_LDS;
  c.sym = 1;
  return c;
}

int64_t batched_size(int nb, const int64_t *offsets) {
  double s1 = 0.0, s2 = 0.0;
  for (int b = 0; b < nb; ++b) {
    const double n = double(offsets[b + 1] - offsets[b]);
    s1 += n;
    s2 += n * n;
  }
  const double v = s1 > 0.0 ? s2 / s1 : 1.0;
  return v < 1.0 ? 1 : int64_t(v);
}

PairCfg Tuning::get_table(int op, int64_t n) const {
  const int cls = size_class(n);
  const PairCfg *best = nullptr;
  int bestd = 1 << 30;
  for (const auto &kv : table) {
    if (kv.first.first != op) continue;
    const int dd = kv.first.second > cls ? kv.first.second - cls : cls - kv.first.second;
    if (dd < bestd) {
      bestd = dd;
      best = &kv.second;
    }
  }
  if (best) return *best;
  PairCfg c;
  c.staging = STAGE_SCALAR;
  c.k = (op == OP_VJP) ? 1 : 2;
  c.waves_per_simd = 8;
  return c;
}

// Source chunks per launch.  Chunks are whole 256-source tiles unless that
// leaves fewer than 4 waves per SIMD (small n): then they shrink to multiples
// of kSubChunk sources, at most kMaxSubSplits of them, so that each lane's
// source loop stays short and the launch's latency is a few microseconds.
constexpr int kSubChunk = 32;
constexpr int kMaxSubSplits = 64;

int64_t pair_chunk(const PairCfg &cfg, int num_cus, int64_t n) {
  const int64_t blocks_x = (n + kBlock * cfg.k - 1) / (kBlock * cfg.k);
  const int64_t want_waves = int64_t(num_cus) * 4 * cfg.waves_per_simd;
  int64_t s = (want_waves + blocks_x * 4 - 1) / (blocks_x * 4);
  const int64_t tiles = (n + kTile - 1) / kTile;
  int64_t unit = kTile, max_s = tiles;
  if (blocks_x * tiles * 4 < int64_t(num_cus) * 16) {
    unit = kSubChunk;
    max_s = std::min<int64_t>((n + kSubChunk - 1) / kSubChunk, kMaxSubSplits);
  }
  if (cfg.max_splits > 0 && max_s > cfg.max_splits) max_s = cfg.max_splits;
  if (s < 1) s = 1;
  if (s > max_s) s = max_s;
  return ((n + s - 1) / s + unit - 1) / unit * unit;
}

int pair_splits(int op, const PairCfg &cfg, int num_cus, int64_t n) {
  (void)op;
  const int64_t chunk = pair_chunk(cfg, num_cus, n);
  return int((n + chunk - 1) / chunk);
}

size_t pair_ws_floats(int op, const PairCfg &cfg, int num_cus, int64_t n) {
  if (cfg.sym) return pair_sym_ws_floats(op, cfg.k, n);
  const int s = pair_splits(op, cfg, num_cus, n);
  return s > 1 ? size_t(s) * nacc(op) * size_t(n) : 0;
}

hipError_t launch_pair(int op, const PairCfg &cfg, int num_cus, int64_t n64, const float *xy,
                       const float *gamma, const float *aux, float delta, float *out, float *out2,
                       float *ws, size_t ws_floats, hipStream_t stream) {
  if (cfg.sym)
    return launch_pair_sym(op, cfg.k, cfg.waves_per_simd, num_cus, n64, xy, gamma, aux, delta, out, out2, ws,
                           ws_floats, stream);
  const int n = int(n64);
  const int64_t chunk = pair_chunk(cfg, num_cus, n64);
  const int s = int((n64 + chunk - 1) / chunk);
  if (s > 1 && ws_floats < size_t(s) * nacc(op) * size_t(n)) return hipErrorInvalidValue;
  const dim3 grid((n + kBlock * cfg.k - 1) / (kBlock * cfg.k), s);
  const float d2 = delta * delta;
  const int partial = s > 1;
  float *o1 = partial ? ws : out;
  hipError_t e;
  switch (op) {
    case OP_VEL: e = dispatch<OP_VEL>(cfg, grid, stream, n, xy, gamma, aux, d2, int(chunk), partial, o1, out2); break;
    case OP_BJAC: e = dispatch<OP_BJAC>(cfg, grid, stream, n, xy, gamma, aux, d2, int(chunk), partial, o1, out2); break;
    case OP_JVP: e = dispatch<OP_JVP>(cfg, grid, stream, n, xy, gamma, aux, d2, int(chunk), partial, o1, out2); break;
    case OP_PSI: e = dispatch<OP_PSI>(cfg, grid, stream, n, xy, gamma, aux, d2, int(chunk), partial, o1, out2); break;
    case OP_VBJ: e = dispatch<OP_VBJ>(cfg, grid, stream, n, xy, gamma, aux, d2, int(chunk), partial, o1, out2); break;
    default: e = dispatch<OP_VJP>(cfg, grid, stream, n, xy, gamma, aux, d2, int(chunk), partial, o1, out2); break;
  }
  if (e != hipSuccess || !partial) return e;
  const dim3 rg((n + 255) / 256);
  switch (op) {
    case OP_VEL: hipLaunchKernelGGL(reduce_kernel<OP_VEL>, rg, dim3(256), 0, stream, n, s, ws, out, out2); break;
    case OP_BJAC: hipLaunchKernelGGL(reduce_kernel<OP_BJAC>, rg, dim3(256), 0, stream, n, s, ws, out, out2); break;
    case OP_JVP: hipLaunchKernelGGL(reduce_kernel<OP_JVP>, rg, dim3(256), 0, stream, n, s, ws, out, out2); break;
    case OP_PSI: hipLaunchKernelGGL(reduce_kernel<OP_PSI>, rg, dim3(256), 0, stream, n, s, ws, out, out2); break;
    case OP_VBJ: hipLaunchKernelGGL(reduce_kernel<OP_VBJ>, rg, dim3(256), 0, stream, n, s, ws, out, out2); break;
    default: hipLaunchKernelGGL(reduce_kernel<OP_VJP>, rg, dim3(256), 0, stream, n, s, ws, out, out2); break;
  }
  return hipGetLastError();
}

// Source chunks for the field-point kernel: enough workgroups for 16 waves
// per CU, whole 256-source tiles per chunk.
int points_splits(int num_cus, int64_t nt, int64_t n) {
  const int64_t blocks_x = (nt + kPtsK * kBlock - 1) / (kPtsK * kBlock);
  const int64_t want_waves = int64_t(num_cus) * 16;
  int64_t s = (want_waves + blocks_x * 4 - 1) / (blocks_x * 4);
  const int64_t max_s = (n + kTile - 1) / kTile;
  s = std::max<int64_t>(1, std::min(s, max_s));
  const int64_t chunk = ((n + s - 1) / s + kTile - 1) / kTile * kTile;
  return int((n + chunk - 1) / chunk);
}

size_t points_ws_floats(int num_cus, int64_t nt, int64_t n) {
  const int s = points_splits(num_cus, nt, n);
  return s > 1 ? size_t(s) * 2 * size_t(nt) : 0;
}

hipError_t launch_velocity_points(int64_t nt, const float *p, int64_t n, const float *xy, const float *gamma,
                                  float delta, float *out, float *ws, size_t ws_floats, int num_cus,
                                  hipStream_t stream) {
  const int s = points_splits(num_cus, nt, n);
  const int64_t chunk = ((n + s - 1) / s + kTile - 1) / kTile * kTile;
  if (s > 1 && ws_floats < size_t(s) * 2 * size_t(nt)) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((nt + kPtsK * kBlock - 1) / (kPtsK * kBlock)), s);
  hipLaunchKernelGGL(points_velocity_kernel, grid, dim3(kBlock), 0, stream, int(nt), p, int(n), xy, gamma,
                     delta * delta, int(chunk), s > 1 ? 1 : 0, s > 1 ? ws : out);
  if (s == 1) return hipGetLastError();
  hipLaunchKernelGGL(reduce_kernel<OP_VEL>, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, stream, int(nt), s, ws,
                     out, nullptr);
  return hipGetLastError();
}

hipError_t launch_velocity_f64(int64_t n, const double *xy, const double *gamma, double delta,
                               double *f, hipStream_t stream) {
  hipLaunchKernelGGL(velocity_f64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                     int(n), xy, gamma, delta * delta, f);
  return hipGetLastError();
}

static dim3 ew_grid(int64_t m) { return dim3((unsigned)((m + 255) / 256)); }

hipError_t launch_axpy(int64_t m, float *out, const float *x, float a, const float *y, hipStream_t s) {
  hipLaunchKernelGGL(axpy_kernel, ew_grid(m), dim3(256), 0, s, m, out, x, a, y);
  return hipGetLastError();
}

hipError_t launch_rk4_combine(int64_t m, float *x, const float *k1, const float *k2,
                              const float *k3, const float *k4, float h, hipStream_t s) {
  hipLaunchKernelGGL(rk4_combine_kernel, ew_grid(m), dim3(256), 0, s, m, x, k1, k2, k3, k4, h / 6.0f);
  return hipGetLastError();
}

hipError_t launch_axpy_f64(int64_t m, double *out, const double *x, double a, const double *y,
                           hipStream_t s) {
  hipLaunchKernelGGL(axpy_f64_kernel, ew_grid(m), dim3(256), 0, s, m, out, x, a, y);
  return hipGetLastError();
}

hipError_t launch_rk4_combine_f64(int64_t m, double *x, const double *k1, const double *k2,
                                  const double *k3, const double *k4, double h, hipStream_t s) {
  hipLaunchKernelGGL(rk4_combine_f64_kernel, ew_grid(m), dim3(256), 0, s, m, x, k1, k2, k3, k4, h);
  return hipGetLastError();
}

}  // namespace ptrom
