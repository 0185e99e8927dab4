// Online projection-tree ROM: HyperPair (Algorithm "HyperPair") and the
// Gauss-Newton loop around it (Algorithm "Gauss-Newton").
//
// Entry layout.  Each interaction-list entry e = (target i, surrogate c) is
// stored as r0_e = xbar0_i - xqt0_c (2), Gamma~_c, pad, then the columns of
// D_e = Phibar_i - Phit_c as (x, y) pairs (2 x M), so that the pair separation at generalized coordinates xhat is
// r_e = r0_e + D_e xhat, which equals xbar_i - p_c with p_c = xqt0_c + Phit_c
// xhat (Algorithm "HyperPair" preamble).  The gather then streams contiguous
// entry rows (coalesced) with no projection pass and no indirection.
//
// Per Gauss-Newton iteration (ptrom_rom_run, one workgroup of 512 threads):
//   gather    paper Jacobian, when the per-entry terms fit in LDS: one thread
//             per list entry computes the pair terms in FP32 (each entry row
//             is loaded whole), groups of 16/32/64 lanes add them per target
//             (DPP row reductions) and write the velocity and trapezoid
//             residual rows rbar = xbar - xbar_prev - dt/2 (fbar + fbar_prev)
//             and the 2x2 blocks B_i, then one thread per element forms
//             C = Phibar - dt/2 B Phibar (FP64).  Otherwise (exact Jacobian,
//             long lists) a group of lanes per target does all of that.
//   solve     G' = A [C | rbar] and the Gram matrix G'^T G' = [G^T G, G^T b;
//             ...] on the FP64 matrix cores, the relative reduced gradient
//             |G^T b| / |G_1^T b_1|, Gauss-Jordan inversion of G^T G inside
//             one wave (columns in registers, pivot columns broadcast from
//             their lanes, no barriers), x = (G^T G)^+ G^T b and one
//             refinement step on the true residual b - G x, then
//             xhat -= alpha x.
// A, [C | rbar], Phibar, xbar0 and the previous-step rows live in LDS when
// they fit.  ptrom_rom_hyperpair runs the gather over many workgroups, one
// wave per target (large sample sets).
#include <algorithm>
#include <array>
#include <cmath>
#include <functional>
#include <cstring>
#include <vector>

#include "internal.h"

using namespace ptrom;

namespace {

// Small bases (M <= 32, M_r <= 64) take the register/single-wave path; larger
// ones (paper Jacobian) the blocked path, up to kMaxM / kMaxMr.
constexpr int kSmallM = 32;
constexpr int kSmallMr = 64;
constexpr int kMaxM = 112;
constexpr int kMaxMr = 256;
constexpr int kRunThreads = 512;  // 8 waves: up to 256 VGPRs per lane
constexpr double kInv2PiD = 0.15915494309189533576888376337251;

struct RomDev {
  int M, Mr, ns, nd, jac_mode, max_iter, ew, ldc, glanes, maxlen, Nc;
  int64_t nnz;
  float d2, dt;
  double tol, alpha;
  const float *Phibar, *xbar0;  // [nd][M], [nd]
  const float *ent;             // entry rows r0x r0y Gamma~ surrogate-id, then (Dx_m Dy_m)
                                // pairs; paper Jacobian: chunk-major, float4 chunk c of
                                // entry e at ((float4 *)ent)[c * nnz + e]; exact
                                // Jacobian: row-major, ent[e * ew ..]
  const int *off;               // [ns+1]
  // point form used by the larger-basis kernel: P = nd + 2 Nc coordinates
  // (the sampled rows, then x and y of every surrogate), basis rows stored
  // mode-major pt[m][p] and reference positions p0[p], both FP64; per entry
  // its target (etg) and surrogate (eid); gt0 the trained Gamma~
  int P;
  const double *ubar;  // [nd] background velocity at the sampled rows (zeros without inflow)
  const double *pt, *p0;
  const int *etg, *eid;
  const float *gt0;
  double *pos;  // [P] point-form positions of the hook's last evaluation
  double *spk;  // [Nc][4] the same surrogate positions packed with Gamma~: x, y, Gamma~, 0,
                // surrogate c at record rec[c] (Morton order of the reference positions)
  const int *rec;   // [Nc]
  const int *erec;  // [nnz] records of each target's surrogates, ascending within the target,
                    // targets in the hook's order (tord), target tord[r] at toff[r] .. toff[r + 1)
  const int *toff;  // [ns + 1]
  const int *tord;  // [ns] the order in which the hook takes the sampled targets (lists sharing
                    // their far-field surrogates adjacent)
  // the hook's target groups: group g holds targets tord[gstart[g] .. gstart[g + 1]) (at most
  // kGroupTargets) and the union of their records urec[ustart[g] .. ustart[g + 1]) (ascending);
  // eloc[e] is entry e's record (erec[e]) as an index into its group's union
  int ngroups, umax;  // umax: the largest union held in LDS (the launch's LDS, in records)
  const int *gstart, *ustart, *urec;
  const unsigned short *eloc;
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

// xbar_i (both rows) at xhat, FP64; Phibar [nd][M] and xbar0 [nd] (FP32)
__device__ __forceinline__ void sampled_position(const float *Phibar, const float *xbar0, int M, int ns, int i,
                                                 const double *xh, double &tx, double &ty) {
  tx = xbar0[i];
  ty = xbar0[ns + i];
  const float *px = Phibar + (size_t)i * M, *py = Phibar + (size_t)(ns + i) * M;
  for (int m = 0; m < M; ++m) {
    tx += (double)px[m] * xh[m];
    ty += (double)py[m] * xh[m];
  }
}

// One entry row in registers: r0x r0y Gamma~ pad, then (Dx_m, Dy_m) pairs,
// padded to whole float4 chunks.  With the paper's Jacobian the table stores
// the rows chunk-major (CM), so lanes reading consecutive entries read one
// contiguous span per chunk; the exact Jacobian re-reads D from its row while
// it accumulates, and keeps the rows whole (row-major), where one address
// serves every chunk.
constexpr int kMaxEw = 4 + 2 * kSmallM;

constexpr int kShortEw = 36;  // rows of bases with M <= 16
constexpr int kTinyEw = 20;   // rows of bases with M <= 8

template <bool CM, int EW>
__device__ __forceinline__ void load_entry(const float *ent, int ew, int64_t nnz, int e, float (&v)[EW]) {
  const float4 *p = reinterpret_cast<const float4 *>(CM ? ent : ent + (size_t)e * ew) + (CM ? e : 0);
#pragma unroll
  for (int c = 0; c < EW / 4; ++c) {
    float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
    if (c * 4 < ew) q = p[CM ? (size_t)c * nnz : (size_t)c];
    v[4 * c] = q.x;
    v[4 * c + 1] = q.y;
    v[4 * c + 2] = q.z;
    v[4 * c + 3] = q.w;
  }
}

// MB: the compile-time bound on the basis size (8, 16, 24 or 32) of the small
// kernels, which sizes every unrolled mode loop, so a small basis runs
// proportionally less code
template <bool EXACT, int MB = kSmallM>
struct GatherAcc {
  float fx = 0.f, fy = 0.f, ba = 0.f, bb = 0.f, bc = 0.f;
  float ex[EXACT ? MB : 1] = {}, ey[EXACT ? MB : 1] = {};
};

// Velocity and Jacobian terms of one (target, surrogate) entry at xhat:
// r = r0 + D xhat; the 2x2 block (or, exact mode, its product with D).
template <bool EXACT, int EW, int MB>
__device__ __forceinline__ void entry_terms(const float (&v)[EW], const float *ent, int ew, int e, const float *xf,
                                            const float *gt, int M, float d2, GatherAcc<EXACT, MB> &a) {
  static_assert(!EXACT || (EW - 4) / 2 <= MB, "accumulators for every mode of the row");
  float rx = v[0], ry = v[1];
#pragma unroll
  for (int m = 0; m < (EW - 4) / 2; ++m)
    if (m < M) {
      rx = fmaf(v[4 + 2 * m], xf[m], rx);
      ry = fmaf(v[5 + 2 * m], xf[m], ry);
    }
  const float q = fmaf(rx, rx, fmaf(ry, ry, d2));
  // a surrogate exactly on its target (possible at delta = 0) adds nothing
  const float r = q > 0.f ? 1.0f / q : 0.f;
  // Gamma~ of the training parameter, or of the query (table indexed by the
  // surrogate id kept in the row)
  const float g = (gt ? gt[__builtin_bit_cast(int, v[3])] : v[2]) * r;
  a.fx = fmaf(-ry, g, a.fx);
  a.fy = fmaf(rx, g, a.fy);
  const float g2 = g * r;
  const float a2 = (rx + rx) * ry;
  const float dd = fmaf(ry, ry, -rx * rx);
  if constexpr (EXACT) {
    // D re-read from the row (cache hit) so the register copy is not kept live
    const float h00 = g2 * a2, h01 = g2 * (dd - d2), h10 = g2 * (dd + d2);
    const float *row = ent + (size_t)e * ew;
#pragma unroll
    for (int m = 0; m < (EW - 4) / 2; ++m)
      if (m < M) {
        const float dx = row[4 + 2 * m], dy = row[5 + 2 * m];
        a.ex[m] = fmaf(h00, dx, fmaf(h01, dy, a.ex[m]));
        a.ey[m] = fmaf(h10, dx, fmaf(-h00, dy, a.ey[m]));
      }
  } else {
    a.ba = fmaf(g2, a2, a.ba);
    a.bb = fmaf(g2, dd - d2, a.bb);
    a.bc = fmaf(g2, dd + d2, a.bc);
  }
}

// The same terms for an entry row read straight from memory in float4 chunks
// (bases with M > 32, paper Jacobian): r = r0 + D xhat, then the velocity and
// the 2x2 block.
__device__ __forceinline__ void entry_terms_stream(const float *ent, int64_t nnz, int e, const float *xf, const float *gt,
                                                   int M, float d2, GatherAcc<false> &a) {
  const float4 *row = reinterpret_cast<const float4 *>(ent) + e;
  const float4 head = row[0];
  float rx = head.x, ry = head.y;
  const int nq = (2 * M + 3) / 4;  // chunks of two modes
#pragma unroll 4
  for (int c = 0; c < nq; ++c) {
    const float4 q = row[(size_t)(1 + c) * nnz];
    const int m = 2 * c;
    rx = fmaf(q.x, xf[m], rx);
    ry = fmaf(q.y, xf[m], ry);
    if (m + 1 < M) {
      rx = fmaf(q.z, xf[m + 1], rx);
      ry = fmaf(q.w, xf[m + 1], ry);
    }
  }
  const float qq = fmaf(rx, rx, fmaf(ry, ry, d2));
  const float r = qq > 0.f ? 1.0f / qq : 0.f;
  const float g = (gt ? gt[__builtin_bit_cast(int, head.w)] : head.z) * r;
  a.fx = fmaf(-ry, g, a.fx);
  a.fy = fmaf(rx, g, a.fy);
  const float g2 = g * r;
  const float a2 = (rx + rx) * ry;
  const float dd = fmaf(ry, ry, -rx * rx);
  a.ba = fmaf(g2, a2, a.ba);
  a.bb = fmaf(g2, dd - d2, a.bb);
  a.bc = fmaf(g2, dd + d2, a.bc);
}

// Sum over an aligned group of G = 16, 32 or 64 lanes (G uniform); every lane
// of the group receives the same value.  All 64 lanes must be active.
__device__ __forceinline__ float gsum(float v, int G) {
  v += dpp_f<0xB1>(v);
  v += dpp_f<0x4E>(v);
  v += dpp_f<0x141>(v);
  v += dpp_f<0x140>(v);
  if (G >= 32) v += __shfl_xor(v, 16, 64);
  if (G == 64) v += __shfl_xor(v, 32, 64);
  return v;
}

// HyperPair rows of sampled target t, computed by a group of G lanes (gl =
// lane in the group).  Lanes of invalid groups (t >= ns) take part in the
// group sums only.  xh: FP64 xhat, xf: FP32 copy; Phibar / xbar0 may be LDS
// copies.  Any output pointer may be null.  Row q of rbar is rbar_out[q * rs],
// row q of C is C_out[q * ldc .. + M).
template <bool EXACT, int MB = kSmallM>
__device__ void gather_group(const RomDev &d, const float *Phibar, const float *xbar0, const float *gt, int t,
                             bool valid, int gl, int G, const double *xh, const float *xf, const double *xbar_prev,
                             const double *fbar_prev, double *xbar_out, double *fbar_out, double *rbar_out, int rs,
                             double *C_out, int ldc, const double *ubar) {
  const int M = d.M, ns = d.ns;
  constexpr int EWB = 4 + 2 * MB;  // the longest row of the bound
  GatherAcc<EXACT, MB> a;
  if (valid) {
    // two (four for M <= 8) entries per lane per pass: the rows are
    // requested before any is used, cutting the exposed load latency on long
    // lists; each lane still adds its entries in list order
    const int e1 = d.off[t + 1];
    int e = d.off[t] + gl;
    if constexpr (!EXACT) {
      bool streamed = false;
      if constexpr (MB == kSmallM) {
        if (M > kSmallM) {
          for (; e < e1; e += G) entry_terms_stream(d.ent, d.nnz, e, xf, gt, M, d.d2, a);
          streamed = true;
        }
      }
      if (!streamed && d.ew <= kShortEw) {
        if (d.ew <= kTinyEw) {
          // four rows in flight per lane for the smallest bases
          for (; e + 3 * G < e1; e += 4 * G) {
            float v0[kTinyEw], v1[kTinyEw], v2[kTinyEw], v3[kTinyEw];
            load_entry<true>(d.ent, d.ew, d.nnz, e, v0);
            load_entry<true>(d.ent, d.ew, d.nnz, e + G, v1);
            load_entry<true>(d.ent, d.ew, d.nnz, e + 2 * G, v2);
            load_entry<true>(d.ent, d.ew, d.nnz, e + 3 * G, v3);
            entry_terms<false>(v0, nullptr, 0, 0, xf, gt, M, d.d2, a);
            entry_terms<false>(v1, nullptr, 0, 0, xf, gt, M, d.d2, a);
            entry_terms<false>(v2, nullptr, 0, 0, xf, gt, M, d.d2, a);
            entry_terms<false>(v3, nullptr, 0, 0, xf, gt, M, d.d2, a);
          }
        }
        if constexpr (MB > 8) {
          for (; e + G < e1; e += 2 * G) {
            float v0[kShortEw], v1[kShortEw];
            load_entry<true>(d.ent, d.ew, d.nnz, e, v0);
            load_entry<true>(d.ent, d.ew, d.nnz, e + G, v1);
            entry_terms<false>(v0, nullptr, 0, 0, xf, gt, M, d.d2, a);
            entry_terms<false>(v1, nullptr, 0, 0, xf, gt, M, d.d2, a);
          }
        }
      }
    }
    for (; e < e1; e += G) {
      float v[EWB];
      load_entry<!EXACT>(d.ent, d.ew, d.nnz, e, v);
      entry_terms<EXACT>(v, d.ent, d.ew, e, xf, gt, M, d.d2, a);
    }
  }
  const double Fx = gsum(a.fx, G) * kInv2PiD + (valid ? ubar[t] : 0.0);
  const double Fy = gsum(a.fy, G) * kInv2PiD + (valid ? ubar[ns + t] : 0.0);
  const double hdt = 0.5 * (double)d.dt;
  if (valid && gl == 0) {
    double tx, ty;
    sampled_position(Phibar, xbar0, M, ns, t, xh, tx, ty);
    if (xbar_out) {
      xbar_out[t] = tx;
      xbar_out[ns + t] = ty;
    }
    if (fbar_out) {
      fbar_out[t] = Fx;
      fbar_out[ns + t] = Fy;
    }
    if (rbar_out) {
      rbar_out[(size_t)t * rs] = (tx - xbar_prev[t]) - hdt * (Fx + fbar_prev[t]);
      rbar_out[(size_t)(ns + t) * rs] = (ty - xbar_prev[ns + t]) - hdt * (Fy + fbar_prev[ns + t]);
    }
  }
  if (C_out) {
    if constexpr (EXACT) {
      // C_t = Phibar_t - dt/2 sum_e G_e (Phibar_t - Phit_c)
#pragma unroll
      for (int m = 0; m < MB; ++m) {
        if (m < M) {
          const double jx = gsum(a.ex[m], G) * kInv2PiD, jy = gsum(a.ey[m], G) * kInv2PiD;
          if (valid && gl == (m & (G - 1))) {
            const double px = Phibar[(size_t)t * M + m], py = Phibar[(size_t)(ns + t) * M + m];
            C_out[(size_t)t * ldc + m] = px - hdt * jx;
            C_out[(size_t)(ns + t) * ldc + m] = py - hdt * jy;
          }
        }
      }
    } else {
      // C_t = Phibar_t - dt/2 B_t Phibar_t (the paper's inexact Jacobian)
      const double B00 = gsum(a.ba, G) * kInv2PiD, B01 = gsum(a.bb, G) * kInv2PiD,
                   B10 = gsum(a.bc, G) * kInv2PiD;
      if (valid)
        for (int m = gl; m < M; m += G) {
          const double px = Phibar[(size_t)t * M + m], py = Phibar[(size_t)(ns + t) * M + m];
          C_out[(size_t)t * ldc + m] = px - hdt * (B00 * px + B01 * py);
          C_out[(size_t)(ns + t) * ldc + m] = py - hdt * (B10 * px - B00 * py);
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
  gather_group<EXACT>(d, d.Phibar, d.xbar0, nullptr, wave, true, lane, 64, xh, xf, xbar_prev, fbar_prev, xbar, fbar,
                      rbar, 1, C, d.M, d.ubar);
}

// Point form of the hook (paper Jacobian).  First every coordinate of the
// point form at xhat, in FP64 (one thread per coordinate, mode-major basis,
// coalesced): the sampled rows xbar = xbar0 + Phibar xhat, then each
// surrogate's p_c = xqt0_c + Phit_c xhat.  Then one wave per sampled target
// walks its list reading only the surrogate id (4 bytes per entry; the
// positions and circulations of the surrogates stay in L2), forms the
// separation in FP64 and the pair terms in FP32.
__global__ void __launch_bounds__(256)
    point_positions_kernel(RomDev d, const double *__restrict__ xhat, double *__restrict__ pos) {
  __shared__ double xh[kMaxM];
  if (threadIdx.x < d.M) xh[threadIdx.x] = xhat[threadIdx.x];
  __syncthreads();
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= d.P) return;
  double v = d.p0[q];
  for (int m = 0; m < d.M; ++m) v = fma(d.pt[(size_t)m * d.P + q], xh[m], v);
  pos[q] = v;
  if (q >= d.nd) {
    // one 32-byte record per surrogate: a list entry touches one cache line,
    // and spatially close surrogates (a target's near field) share lines
    const int c = (q - d.nd) >> 1, k = (q - d.nd) & 1, rc = d.rec[c];
    d.spk[4 * rc + k] = v;
    if (k == 0) {
      d.spk[4 * rc + 2] = (double)d.gt0[c];
      d.spk[4 * rc + 3] = 0.0;
    }
  }
}

typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void point_terms(double tx, double ty, const dbl4 p, float d2, GatherAcc<false> &a) {
  const float rx = float(tx - p.x), ry = float(ty - p.y);
  const float q = fmaf(rx, rx, fmaf(ry, ry, d2));
  const float r = q > 0.f ? 1.0f / q : 0.f;  // a surrogate on its target adds nothing
  const float g = float(p.z) * r;
  a.fx = fmaf(-ry, g, a.fx);
  a.fy = fmaf(rx, g, a.fy);
  const float g2 = g * r;
  const float a2 = (rx + rx) * ry;
  const float dd = fmaf(ry, ry, -rx * rx);
  a.ba = fmaf(g2, a2, a.ba);
  a.bb = fmaf(g2, dd - d2, a.bb);
  a.bc = fmaf(g2, dd + d2, a.bc);
}

constexpr int kGroupTargets = 8;   // targets per group: one wave each
constexpr int kUnionCap = 1024;    // records of a group held in LDS (at most 32 KB)

// One workgroup per target group: the union of the group's records is
// copied to LDS once (targets whose lists share their far-field surrogates
// are grouped, so the union is a fraction of the lists' total), then one
// wave per target walks its list by 2-byte union indices.  The entries are
// stored in group order, so a wave's index loads depend on nothing but its
// slot; they, the target's own operands and the union copy are all in
// flight before the barrier.  A group whose union passes kUnionCap (a single
// target's long list) reads its records from the global table instead.
constexpr int kGatherKU = 6;  // list entries per lane in flight
__global__ void __launch_bounds__(64 * kGroupTargets) __attribute__((amdgpu_waves_per_eu(8, 8)))
    gather_point_kernel(RomDev d, const double *__restrict__ pos, const double *__restrict__ xbar_prev,
                        const double *__restrict__ fbar_prev, double *xbar, double *fbar, double *rbar, double *C) {
  extern __shared__ __align__(16) double ulds[];
  dbl4 *ur = reinterpret_cast<dbl4 *>(ulds);
  const dbl4 *sp = reinterpret_cast<const dbl4 *>(d.spk);
  const int g = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  const int ns = d.ns, M = d.M;
  const int r = d.gstart[g] + (tid >> 6);
  const bool valid = r < d.gstart[g + 1];
  const int u0 = d.ustart[g], nu = d.ustart[g + 1] - u0;
  const bool in_lds = nu <= kUnionCap;
  int t = 0, e0 = 0, e1 = 0;
  if (valid) {
    t = d.tord[r];
    e0 = d.toff[r];
    e1 = d.toff[r + 1];
  }
  if (in_lds)
    for (int u = tid; u < nu; u += 64 * kGroupTargets) ur[u] = sp[d.urec[u0 + u]];
  // the first round of this lane's entries (lane + 64 k of the list)
  int c[kGatherKU];
#pragma unroll
  for (int k = 0; k < kGatherKU; ++k) {
    const int e = e0 + lane + 64 * k;
    c[k] = e < e1 ? (in_lds ? (int)d.eloc[e] : d.erec[e]) : -1;
  }
  // the target's own operands
  double tx = 0.0, ty = 0.0, u_x = 0.0, u_y = 0.0, xp_x = 0.0, xp_y = 0.0, fp_x = 0.0, fp_y = 0.0;
  float phx = 0.f, phy = 0.f;
  if (valid) {
    tx = pos[t];
    ty = pos[ns + t];
    u_x = d.ubar[t];
    u_y = d.ubar[ns + t];
    if (rbar) {
      xp_x = xbar_prev[t];
      xp_y = xbar_prev[ns + t];
      fp_x = fbar_prev[t];
      fp_y = fbar_prev[ns + t];
    }
    if (C && lane < M) {
      phx = d.Phibar[(size_t)t * M + lane];
      phy = d.Phibar[(size_t)(ns + t) * M + lane];
    }
  }
  __syncthreads();
  if (!valid) return;
  const double hdt = 0.5 * (double)d.dt;
  GatherAcc<false> a;
  // each lane adds its entries in list order (the two record sources in
  // separate loops, so each keeps its own address space)
  auto walk = [&](auto rec_at, auto idx_at) {
    for (int eb = e0;;) {
#pragma unroll
      for (int k = 0; k < kGatherKU; ++k)
        if (c[k] >= 0) point_terms(tx, ty, rec_at(c[k]), d.d2, a);
      eb += 64 * kGatherKU;
      if (eb >= e1) break;
#pragma unroll
      for (int k = 0; k < kGatherKU; ++k) {
        const int e = eb + lane + 64 * k;
        c[k] = e < e1 ? idx_at(e) : -1;
      }
    }
  };
  if (in_lds)
    walk([&](int q) { return ur[q]; }, [&](int e) { return (int)d.eloc[e]; });
  else
    walk([&](int q) { return sp[q]; }, [&](int e) { return d.erec[e]; });
  const double Fx = gsum(a.fx, 64) * kInv2PiD + u_x;
  const double Fy = gsum(a.fy, 64) * kInv2PiD + u_y;
  if (lane == 0) {
    if (xbar) {
      xbar[t] = tx;
      xbar[ns + t] = ty;
    }
    if (fbar) {
      fbar[t] = Fx;
      fbar[ns + t] = Fy;
    }
    if (rbar) {
      rbar[t] = (tx - xp_x) - hdt * (Fx + fp_x);
      rbar[ns + t] = (ty - xp_y) - hdt * (Fy + fp_y);
    }
  }
  if (C) {
    const double B00 = gsum(a.ba, 64) * kInv2PiD, B01 = gsum(a.bb, 64) * kInv2PiD, B10 = gsum(a.bc, 64) * kInv2PiD;
    for (int m = lane; m < M; m += 64) {
      // the lane's first mode was loaded above
      const double px = m == lane ? (double)phx : (double)d.Phibar[(size_t)t * M + m];
      const double py = m == lane ? (double)phy : (double)d.Phibar[(size_t)(ns + t) * M + m];
      C[(size_t)t * M + m] = px - hdt * (B00 * px + B01 * py);
      C[(size_t)(ns + t) * M + m] = py - hdt * (B10 * px - B00 * py);
    }
  }
}

// ----------------------------------------------------------- device-resident loop

// One 16 x 16 tile of D = X Y (X: rows x K, Y: K x cols) on one wave with the
// FP64 matrix-core instruction (16 x 16 x 4 per step): lane l supplies
// X(l % 16, k0 + l / 16) and Y(k0 + l / 16, l % 16) and receives, in register
// r, D(4 r + l / 16, l % 16) (tile-local indices).  xa / yb return 0 outside
// the matrices.  Whole groups of four k-steps go to four independent
// accumulators, so consecutive products do not wait on each other; the four
// are added at the end.  The wave must be fully active.
template <class FX, class FY>
__device__ __forceinline__ dbl4 mfma_tile(int K, int lane, FX xa, FY yb, dbl4 acc = dbl4{0.0, 0.0, 0.0, 0.0}) {
  const int r = lane & 15, kq = lane >> 4;
  dbl4 c1 = dbl4{0.0, 0.0, 0.0, 0.0}, c2 = c1, c3 = c1;
  int k0 = 0;
  for (; k0 + 16 <= K; k0 += 16) {
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = xa(r, k0 + 4 * u + kq);
      b[u] = yb(k0 + 4 * u + kq, r);
    }
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], acc, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1], b[1], c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[2], b[2], c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[3], b[3], c3, 0, 0, 0);
  }
  for (; k0 < K; k0 += 4) {
    const int k = k0 + kq;
    const double a = k < K ? xa(r, k) : 0.0;
    const double b = k < K ? yb(k, r) : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  return (acc + c1) + (c2 + c3);
}

// Sum over aligned groups of 8 lanes (all lanes active); every lane of the
// group receives the sum.
__device__ __forceinline__ double sum8(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x141>(v);
  return v;
}

// Split runs (paper Jacobian, arrays in LDS): the W workgroups of one query
// each hold a contiguous slice of the entry rows in LDS (slice w: entries
// [w L, (w + 1) L)).  Per HyperPair evaluation b every workgroup sums its
// slice's terms for each target whose list meets the slice and publishes the
// five sums, each as one 64-bit word (FP32 bits, and b + 1 in the high half);
// then it reads, for every target, the words of the slices its list spans,
// until all carry b + 1, and adds them in slice order.  The tags make each
// word its own completion flag: no counter, no fences.  Words alternate
// between two buffers by the parity of b: a workgroup writes evaluation b + 2
// only after it has read everyone's b + 1, which each wrote after reading b.
// Each workgroup then runs the whole solve itself.  The workgroups run the
// same instructions on the same data, so their xhat, and with it every
// convergence decision, agree bit for bit, and they take part in the same
// evaluations.  A workgroup whose wait fails max_polls checks (the grid is
// launched cooperatively, so every workgroup is resident and a wait ends)
// raises the abort flag; every workgroup of the launch then leaves at its
// next wait, and the query reports iters = -1.
struct SplitArgs {
  int W = 1;                           // workgroups per query
  int L = 0;                           // entries per slice, ceil(nnz / W)
  unsigned long long *part = nullptr;  // [2][nq][W][5 ns] tagged slice sums, zero at launch
  unsigned *abort = nullptr;           // [1] zero at launch
  unsigned max_polls = 0;              // failed checks of one wait before the abort
  int nt = 0;                          // most targets whose lists meet one slice
};
constexpr unsigned kSplitPolls = 1u << 20;  // about a second of polling

// LDSA: the arrays' LDS copies are used (a compile-time choice, so every
// access to them is an LDS instruction); otherwise they are read in place.
// SPLIT: the split form above (requires !EXACT and LDSA).  MB: the basis
// bound (M <= MB).
template <bool EXACT, bool LDSA, bool SPLIT, int MB>
__global__ void __launch_bounds__(kRunThreads)
    rom_run_kernel(RomDev d, int nsteps, int entry_par, const float *__restrict__ gtq,
                   double *__restrict__ xhat, double *__restrict__ hist, int *__restrict__ iters, SplitArgs sp) {
  static_assert(!SPLIT || (!EXACT && LDSA), "split runs use the paper Jacobian with LDS copies");
  __shared__ double xh[kSmallM];
  __shared__ float xf[kSmallM];
  __shared__ double rr[kSmallMr], gq[kSmallM], xs[kSmallM], gvec[kSmallM];
  __shared__ double s_eps, s_g1, s_gn;
  __shared__ int s_ab[2];  // split: the abort flag as read at each poll (alternating)
  extern __shared__ __align__(16) double dyn[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = kRunThreads / 64;
  // query and slice of this workgroup
  const int qi = SPLIT ? (int)blockIdx.x / sp.W : (int)blockIdx.x;
  const int wpart = SPLIT ? (int)blockIdx.x - qi * sp.W : 0;
  const int M = d.M, Mr = d.Mr, nd = d.nd, ns = d.ns, ldc = d.ldc, M1 = M + 1;
  const int lg = M1;  // row stride of G'
  const double hdt = 0.5 * (double)d.dt;
  // G' = A [C | rbar] (Mr x (M + 1)) and the Gauss-Jordan tableau [N | I]
  // (rows padded to MB, columns to 64: one column per lane of a wave) at the
  // front of the dynamic LDS
  double *Gp = dyn, *T0 = Gp + (size_t)Mr * lg;

  // A, [C | rbar], fbar, fbar_prev, xbar_prev, the per-target 2x2 blocks,
  // Phibar, xbar0 and the per-entry terms: LDS copies when they fit.  The
  // copy of A has an odd row stride (n_d + 1 doubles), so the 16 lanes that
  // read one matrix-core operand column hit distinct banks.
  const double *A = d.A;
  const int lda = LDSA ? nd + 1 : nd;
  const float *Phibar = d.Phibar, *xbar0 = d.xbar0;
  double *Cp = d.C, *fbar = d.fbar, *fbar_prev = d.fbar_prev, *xbar_prev = d.xbar_prev, *bt = nullptr,
         *xcur = nullptr;
  float *ct = nullptr;
  const float *gt = nullptr;
  const double *ubar = d.ubar;
  double *psum = nullptr;            // split: [5][ns] sums over all slices
  int *wsp = nullptr;                // split: [ns][4] first and last slice of each target's list, and
                                     // the list's local range in this slice (empty when it misses it)
  float *wp = nullptr;               // split: [8 waves][sp.nt][5] each wave's sums per slice target
  const float *rows = nullptr;       // split: this slice's entry rows, chunk-major, stride sp.L
  int e0 = 0, ln = 0, ta = 0, tb = -1;  // split: entries [e0, e0 + ln), of targets ta..tb
  xhat += (size_t)qi * M;
  if (hist) hist += (size_t)qi * nsteps * M;
  if (iters) iters += (size_t)qi * nsteps;
  if constexpr (LDSA) {
    double *p = T0 + (size_t)MB * 64;
    double *Al = p; p += (size_t)Mr * (nd + 1);
    Cp = p; p += (size_t)nd * ldc;
    fbar = p; p += nd;
    fbar_prev = p; p += nd;
    xbar_prev = p; p += nd;
    bt = p; p += 3 * (size_t)ns;
    xcur = p; p += nd;
    {
      double *ul = p;
      p += nd;
      for (int t = tid; t < nd; t += kRunThreads) ul[t] = d.ubar[t];
      ubar = ul;
    }
    if constexpr (SPLIT) {
      psum = p;
      p += 5 * (size_t)ns;
      wsp = reinterpret_cast<int *>(p);
      p += 2 * (size_t)ns;
    }
    float *f = reinterpret_cast<float *>(p);
    float *Pl = f; f += (size_t)nd * M;
    float *xl = f; f += nd;
    ct = f; f += SPLIT ? 5 * (size_t)sp.L : entry_par ? 5 * (size_t)d.nnz : 0;
    if constexpr (SPLIT) {
      wp = f;
      f += (size_t)nwaves * sp.nt * 5;
    }
    if (gtq) {
      // this query's clustered circulations (one workgroup per query)
      float *gl_ = f;
      for (int t = tid; t < d.Nc; t += kRunThreads) gl_[t] = gtq[(size_t)qi * d.Nc + t];
      gt = gl_;
      f += d.Nc;
    }
    if constexpr (SPLIT) {
      // the slice's rows, 16-byte aligned, chunk c of local entry l at
      // float4 index c * L + l (the table's chunk-major form)
      // (offsets from the 16-byte aligned base, so the pointer stays an LDS one)
      const size_t fo = (reinterpret_cast<char *>(f) - reinterpret_cast<char *>(dyn) + 15) & ~size_t(15);
      float4 *r4 = reinterpret_cast<float4 *>(reinterpret_cast<char *>(dyn) + fo);
      const int nnz = (int)d.nnz;
      e0 = min(wpart * sp.L, nnz);
      ln = min(sp.L, nnz - e0);
      const int nch = d.ew / 4;
      const float4 *g4 = reinterpret_cast<const float4 *>(d.ent);
      for (int t = tid; t < nch * ln; t += kRunThreads) {
        const int c = t / ln, l = t - c * ln;
        r4[(size_t)c * sp.L + l] = g4[(size_t)c * nnz + e0 + l];
      }
      rows = reinterpret_cast<const float *>(r4);
      for (int t = tid; t < ns; t += kRunThreads) {
        const int a = d.off[t], b = d.off[t + 1];
        wsp[4 * t] = b > a ? a / sp.L : 1;
        wsp[4 * t + 1] = b > a ? (b - 1) / sp.L : 0;
        wsp[4 * t + 2] = min(max(a - e0, 0), ln);
        wsp[4 * t + 3] = min(max(b - e0, 0), ln);
      }
      if (ln > 0) {
        // first target whose list ends past e0, last one whose list starts
        // before e0 + ln
        int lo = 0, hi = ns - 1;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (d.off[mid + 1] > e0) hi = mid;
          else lo = mid + 1;
        }
        ta = lo;
        hi = ns - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (d.off[mid] < e0 + ln) lo = mid;
          else hi = mid - 1;
        }
        tb = lo;
      }
    }
    for (int t = tid; t < Mr * nd; t += kRunThreads) Al[(t / nd) * (nd + 1) + t % nd] = d.A[t];
    for (int t = tid; t < nd * M; t += kRunThreads) Pl[t] = d.Phibar[t];
    for (int t = tid; t < nd; t += kRunThreads) xl[t] = d.xbar0[t];
    A = Al;
    Phibar = Pl;
    xbar0 = xl;
  }
  for (int t = tid; t < nd * ldc; t += kRunThreads) Cp[t] = 0.0;  // padding columns stay zero
  if (tid < M) {
    xh[tid] = xhat[tid];
    xf[tid] = (float)xhat[tid];
  }
  __syncthreads();
  // targets are taken by groups of G lanes, 64 / G per wave
  const int G = d.glanes, tpw = 64 / G, gl = lane & (G - 1), slot = lane / G;

  // split: the slice's terms at xhat, its per-target sums, the barrier, then
  // psum[k * ns + t] = the sums of all slices (FP64, added in slice order).
  // Returns false when the launch is aborted.
  int nbar = 0;
  auto split_sums = [&]() -> bool {
    const int L = sp.L;
    for (int l = tid; l < ln; l += kRunThreads) {
      float v[4 + 2 * MB];
      load_entry<true>(rows, d.ew, L, l, v);
      GatherAcc<false> a;
      entry_terms<false>(v, nullptr, 0, 0, xf, gt, M, d.d2, a);
      ct[l] = a.fx;
      ct[L + l] = a.fy;
      ct[2 * L + l] = a.ba;
      ct[3 * L + l] = a.bb;
      ct[4 * L + l] = a.bc;
    }
    __syncthreads();
    // this evaluation's buffer; words of slice w of this query at [w][5 ns]
    unsigned long long *par = sp.part + ((size_t)(nbar & 1) * gridDim.x + (size_t)qi * sp.W) * 5 * (size_t)ns;
    const unsigned long long tag = (unsigned long long)(unsigned)(nbar + 1) << 32;
    unsigned long long *mine = par + (size_t)wpart * 5 * ns;
    // each wave sums its share [c0, c1) of the slice per target; the waves'
    // sums are then added in wave order
    {
      const int cw = (ln + nwaves - 1) / nwaves, c0 = min(wave * cw, ln), c1 = min(c0 + cw, ln);
      for (int i = 0; i <= tb - ta; ++i) {
        const int t = ta + i, r0 = max(wsp[4 * t + 2], c0), r1 = min(wsp[4 * t + 3], c1);
        float sv[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
        if (r0 < r1) {
          for (int e = r0 + lane; e < r1; e += 64)
#pragma unroll
            for (int k = 0; k < 5; ++k) sv[k] += ct[k * L + e];
#pragma unroll
          for (int k = 0; k < 5; ++k) sv[k] = gsum(sv[k], 64);
        }
        if (lane == 0)
#pragma unroll
          for (int k = 0; k < 5; ++k) wp[((size_t)wave * sp.nt + i) * 5 + k] = sv[k];
      }
    }
    __syncthreads();
    for (int q = tid; q < 5 * (tb - ta + 1); q += kRunThreads) {
      const int i = q / 5, k = q - 5 * i;
      float sm = 0.f;
      for (int v = 0; v < nwaves; ++v) sm += wp[((size_t)v * sp.nt + i) * 5 + k];
      __hip_atomic_store(mine + k * ns + ta + i, tag | __float_as_uint(sm), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    // every target's sums from the slices its list spans, in slice order,
    // once all of them carry this evaluation's tag
    for (unsigned polls = 0;; ++polls) {
      if (tid == 0) s_ab[polls & 1] = (int)__hip_atomic_load(sp.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      int ok = 1;
      for (int q = tid; q < 5 * ns; q += kRunThreads) {
        const int t = q - (q / ns) * ns;
        double s = 0.0;
        for (int w = wsp[4 * t]; w <= wsp[4 * t + 1]; ++w) {
          const unsigned long long v =
              __hip_atomic_load(par + (size_t)w * 5 * ns + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok &= (v >> 32) == (tag >> 32);
          s += (double)__uint_as_float((unsigned)v);
        }
        psum[q] = s;
      }
      if (__syncthreads_and(ok)) break;
      if (s_ab[polls & 1] || polls + 1 >= sp.max_polls) {
        if (tid == 0) __hip_atomic_store(sp.abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return false;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    ++nbar;
    return true;
  };
  // an aborted split launch: the query reports iters = -1 and a NaN xhat
  auto split_abort = [&]() {
    if (wpart != 0) return;
    if (iters)
      for (int s = tid; s < nsteps; s += kRunThreads) iters[s] = -1;
    if (tid < M) xhat[tid] = __builtin_nan("");
  };

  // previous-step terms for the first step: HyperPair at the initial xhat
  if constexpr (SPLIT) {
    if (!split_sums()) {
      split_abort();
      return;
    }
    for (int q = tid; q < nd; q += kRunThreads) {
      const int i = q < ns ? q : q - ns;
      double tx, ty;
      sampled_position(Phibar, xbar0, M, ns, i, xh, tx, ty);
      xbar_prev[q] = q < ns ? tx : ty;
      fbar_prev[q] = psum[q] * kInv2PiD + ubar[q];
    }
  } else {
    for (int base = wave * tpw; base < ns; base += nwaves * tpw)
      gather_group<EXACT, MB>(d, Phibar, xbar0, gt, base + slot, base + slot < ns, gl, G, xh, xf, nullptr, nullptr,
                              xbar_prev, fbar_prev, nullptr, 0, nullptr, 0, ubar);
  }
  __syncthreads();

  const int tr = (Mr + 15) / 16, tc = (M1 + 15) / 16;
  const int nnz = (int)d.nnz;
  for (int step = 0; step < nsteps; ++step) {
    int k = 1;
    for (;;) {
      // ---- HyperPair: velocity rows, residual rows (column M of [C | rbar]) and C
      if (!EXACT && (SPLIT || entry_par)) {
        if constexpr (SPLIT) {
          if (!split_sums()) {
            split_abort();
            return;
          }
        } else {
          // one thread per entry; the five per-entry terms go to LDS
          for (int e = tid; e < nnz; e += kRunThreads) {
            float v[4 + 2 * MB];
            load_entry<true>(d.ent, d.ew, d.nnz, e, v);
            GatherAcc<false> a;
            entry_terms<false>(v, nullptr, 0, 0, xf, gt, M, d.d2, a);
            ct[e] = a.fx;
            ct[nnz + e] = a.fy;
            ct[2 * nnz + e] = a.ba;
            ct[3 * nnz + e] = a.bb;
            ct[4 * nnz + e] = a.bc;
          }
        }
        // the sampled rows at the current xhat
        for (int q = tid; q < nd; q += kRunThreads) {
          double x = xbar0[q];
          const float *ph = Phibar + (size_t)q * M;
          for (int m = 0; m < M; ++m) x += (double)ph[m] * xh[m];
          xcur[q] = x;
        }
        __syncthreads();
        // per-target sums (one thread per target for lists of at most 8, else
        // groups of G lanes), residual rows and the 2x2 blocks
        auto finish = [&](int t, double s0, double s1, double s2, double s3, double s4) {
          const double Fx = s0 * kInv2PiD + ubar[t], Fy = s1 * kInv2PiD + ubar[ns + t];
          fbar[t] = Fx;
          fbar[ns + t] = Fy;
          Cp[(size_t)t * ldc + M] = (xcur[t] - xbar_prev[t]) - hdt * (Fx + fbar_prev[t]);
          Cp[(size_t)(ns + t) * ldc + M] = (xcur[ns + t] - xbar_prev[ns + t]) - hdt * (Fy + fbar_prev[ns + t]);
          bt[3 * t] = s2 * kInv2PiD;
          bt[3 * t + 1] = s3 * kInv2PiD;
          bt[3 * t + 2] = s4 * kInv2PiD;
        };
        if constexpr (SPLIT) {
          for (int t = tid; t < ns; t += kRunThreads)
            finish(t, psum[t], psum[ns + t], psum[2 * ns + t], psum[3 * ns + t], psum[4 * ns + t]);
        } else if (d.maxlen <= 8) {
          for (int t = tid; t < ns; t += kRunThreads) {
            float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f, s4 = 0.f;
            const int e1 = d.off[t + 1];
            for (int e = d.off[t]; e < e1; ++e) {
              s0 += ct[e];
              s1 += ct[nnz + e];
              s2 += ct[2 * nnz + e];
              s3 += ct[3 * nnz + e];
              s4 += ct[4 * nnz + e];
            }
            finish(t, s0, s1, s2, s3, s4);
          }
        } else {
          for (int base = wave * tpw; base < ns; base += nwaves * tpw) {
            const int t = base + slot;
            const bool valid = t < ns;
            float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f, s4 = 0.f;
            if (valid) {
              const int e1 = d.off[t + 1];
              for (int e = d.off[t] + gl; e < e1; e += G) {
                s0 += ct[e];
                s1 += ct[nnz + e];
                s2 += ct[2 * nnz + e];
                s3 += ct[3 * nnz + e];
                s4 += ct[4 * nnz + e];
              }
            }
            s0 = gsum(s0, G);
            s1 = gsum(s1, G);
            s2 = gsum(s2, G);
            s3 = gsum(s3, G);
            s4 = gsum(s4, G);
            if (valid && gl == 0) finish(t, s0, s1, s2, s3, s4);
          }
        }
        __syncthreads();
        // C = Phibar - dt/2 B Phibar (the paper's inexact Jacobian), one element per thread
        for (int q = tid; q < nd * M; q += kRunThreads) {
          const int row = q / M, m = q - row * M;
          const int t = row < ns ? row : row - ns;
          const double px = Phibar[(size_t)t * M + m], py = Phibar[(size_t)(ns + t) * M + m];
          const double B00 = bt[3 * t], B01 = bt[3 * t + 1], B10 = bt[3 * t + 2];
          Cp[(size_t)row * ldc + m] = row < ns ? px - hdt * (B00 * px + B01 * py) : py - hdt * (B10 * px - B00 * py);
        }
      } else {
        for (int base = wave * tpw; base < ns; base += nwaves * tpw)
          gather_group<EXACT, MB>(d, Phibar, xbar0, gt, base + slot, base + slot < ns, gl, G, xh, xf, xbar_prev,
                                  fbar_prev, nullptr, fbar, Cp + M, ldc, Cp, ldc, ubar);
      }
      __syncthreads();
      // ---- G' = A [C | rbar] on the matrix cores (Mr x (M + 1))
      for (int tile = wave; tile < tr * tc; tile += nwaves) {
        const int i0 = (tile / tc) * 16, j0 = (tile % tc) * 16;
        const dbl4 acc = mfma_tile(
            nd, lane, [&](int i, int q) { return i0 + i < Mr ? A[(size_t)(i0 + i) * lda + q] : 0.0; },
            [&](int q, int j) { return j0 + j < ldc ? Cp[(size_t)q * ldc + j0 + j] : 0.0; });
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = i0 + 4 * r + (lane >> 4), col = j0 + (lane & 15);
          if (row < Mr && col < M1) Gp[row * lg + col] = acc[r];
        }
      }
      __syncthreads();
      // ---- Gram G'^T G' into the tableau [N | I | g]: N = G^T G, g = G^T b
      for (int tile = wave; tile < tc * tc; tile += nwaves) {
        const int i0 = (tile / tc) * 16, j0 = (tile % tc) * 16;
        const dbl4 acc = mfma_tile(
            Mr, lane, [&](int i, int q) { return i0 + i < M1 ? Gp[q * lg + i0 + i] : 0.0; },
            [&](int q, int j) { return j0 + j < M1 ? Gp[q * lg + j0 + j] : 0.0; });
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = i0 + 4 * r + (lane >> 4), col = j0 + (lane & 15);
          if (row < M && col < M) T0[row * 64 + col] = acc[r];
          if (row < M && col == M) gvec[row] = acc[r];
        }
      }
      // identity block and zero padding of the tableau
      for (int t = tid; t < MB * 64; t += kRunThreads) {
        const int i = t >> 6, j = t & 63;
        if (i >= M || j >= M) T0[t] = (i < M && j - M == i) ? 1.0 : 0.0;
      }
      __syncthreads();
      // ---- in wave 0: the relative reduced gradient |G^T b| / |G_1^T b_1|,
      // then Gauss-Jordan inversion of N = G^T G (symmetric positive
      // semi-definite) on the tableau [N | I], lane j owning column j in
      // registers (rows past M are zero padding and stay zero).  The pivot
      // loop is unrolled, so every row index is static; each step reads the
      // pivot column's entries from lane kk (lane_d) and updates the
      // lane's own column.  A non-positive pivot leaves its direction out
      // (its row of the inverse is zero).
      if (wave == 0) {
        const double gv = lane < M ? gvec[lane] : 0.0;
        const double gn = sqrt(wsumd(gv * gv));
        if (lane == 0) s_gn = gn;
        double col[MB];
#pragma unroll
        for (int u = 0; u < MB; ++u) col[u] = T0[u * 64 + lane];
#pragma unroll
        for (int kk = 0; kk < MB; ++kk) {
          if (kk < M) {
            const double piv = lane_d(col[kk], kk);
            double ip = 0.0;
            if (piv > 0.0) {
              // reciprocal: hardware estimate refined by two Newton steps
              ip = __builtin_amdgcn_rcp(piv);
              ip = fma(ip, fma(-piv, ip, 1.0), ip);
              ip = fma(ip, fma(-piv, ip, 1.0), ip);
            }
            const double rk = col[kk] * ip;
            // rows in blocks of 8; blocks wholly past M are padding.  A
            // block's pivot-column entries are all read before any is used,
            // so the scalar-register hazard of each read is hidden.
#pragma unroll
            for (int i0 = 0; i0 < MB; i0 += 8) {
              if (i0 < M) {
                double cb[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) cb[u] = lane_d(col[i0 + u], kk);
#pragma unroll
                for (int u = 0; u < 8; ++u)
                  col[i0 + u] = i0 + u == kk ? rk : fma(-cb[u], rk, col[i0 + u]);
              }
            }
          }
        }
#pragma unroll
        for (int u = 0; u < MB; ++u) T0[u * 64 + lane] = col[u];
      }
      __syncthreads();
      // ---- x = N^+ g, then one refinement step: r' = b - G x, g' = G^T r',
      // x += N^+ g' (8 lanes per dot product)
      const double *Pc = T0;
      {
        const int o = tid >> 3, part = tid & 7;
        double s = 0.0;
        if (o < M)
          for (int j = part; j < M; j += 8) s = fma(Pc[o * 64 + M + j], gvec[j], s);
        s = sum8(s);
        if (o < M && part == 0) xs[o] = s;
      }
      __syncthreads();
      {
        const int o = tid >> 3, part = tid & 7;
        double s = 0.0;
        if (o < Mr)
          for (int j = part; j < M; j += 8) s = fma(Gp[o * lg + j], xs[j], s);
        s = sum8(s);
        if (o < Mr && part == 0) rr[o] = Gp[o * lg + M] - s;
      }
      __syncthreads();
      {
        const int o = tid >> 3, part = tid & 7;
        double s = 0.0;
        if (o < M)
          for (int r = part; r < Mr; r += 8) s = fma(Gp[r * lg + o], rr[r], s);
        s = sum8(s);
        if (o < M && part == 0) gq[o] = s;
      }
      __syncthreads();
      {
        const int o = tid >> 3, part = tid & 7;
        double s = 0.0;
        if (o < M)
          for (int j = part; j < M; j += 8) s = fma(Pc[o * 64 + M + j], gq[j], s);
        s = sum8(s);
        if (o < M && part == 0) xs[o] += s;
      }
      __syncthreads();
      if (tid < M) {
        xh[tid] -= d.alpha * xs[tid];
        xf[tid] = (float)xh[tid];
      }
      if (tid == 0) {
        const double gn = s_gn;
        if (k == 1) s_g1 = gn;
        const double g1 = k == 1 ? gn : s_g1;
        s_eps = g1 > 0.0 ? gn / g1 : 0.0;
      }
      __syncthreads();
      ++k;
      if (!(s_eps > d.tol) || k > d.max_iter) break;
      __syncthreads();  // s_eps read by everyone before the next write
    }
    if (wpart == 0 && tid < M && hist) hist[(size_t)step * M + tid] = xh[tid];
    if (wpart == 0 && tid == 0 && iters) iters[step] = k - 1;
    // previous-step terms: sampled rows at the accepted xhat, velocity of
    // the last HyperPair evaluation
    for (int q = tid; q < nd; q += kRunThreads) {
      const int i = q < ns ? q : q - ns;
      double tx, ty;
      sampled_position(Phibar, xbar0, M, ns, i, xh, tx, ty);
      xbar_prev[q] = q < ns ? tx : ty;
      fbar_prev[q] = fbar[q];
    }
    __syncthreads();
  }
  if (wpart == 0 && tid < M) xhat[tid] = xh[tid];
}

// ----------------------------------------------------------- larger bases

// Bases with M > 32 or M_r > 64 (paper Jacobian; M <= 112, M_r <= 256).  One
// workgroup per query; per Gauss-Newton iteration:
//   gather    the sampled-row and surrogate positions at xhat in FP64 (one
//             thread per coordinate over a mode-major basis), then each
//             target's list by a group of 8 lanes: velocity, residual rows
//             rbar and the 2x2 blocks; C = (I - dt/2 B) Phibar in FP32,
//             formed in place over a copy of Phibar left by the positions;
//   normal    N' = G'^T G' with G' = A [C | rbar] accumulated over 16-row
//   matrix    blocks of A: the block is staged in LDS, G'_blk = A_blk [C |
//             rbar] and N' += G'_blk^T G'_blk run on the FP64 matrix cores,
//             each wave keeping its (lower-triangle) tiles of N' in registers;
//   solve     N = G^T G is inverted in place by blocked Gauss-Jordan over
//             16 x 16 blocks of its lower block triangle: one wave inverts
//             the pivot block in registers (a non-positive pivot leaves its
//             direction out), the row and column panels and the rank-16
//             trailing update run on the FP64 matrix cores; then x = N^-1 g
//             with g = G^T b.
// C enters only the step direction, never the residual, so its FP32 rounding
// leaves the Gauss-Newton fixed point where it is.
// LDS: region 1 holds C and rbar and then N; region 2 holds the positions
// during the gather, the A / G' row blocks during the product and the panels
// during the inversion; the tail holds the previous-step rows, this query's
// Gamma~ and the entries' surrogate ids.
constexpr int kMaxTiles = 5;  // lower-triangle tiles of N' per wave
constexpr int kPf = 4;        // A elements per thread prefetched a block ahead (n_d <= 128; the rest is loaded in place)
static_assert(((kMaxM + 17) / 16) * ((kMaxM + 17) / 16 + 1) / 2 <= kMaxTiles * (kRunThreads / 64),
              "every lower-triangle tile of N' needs an owner");

// LDS row strides chosen so that the 16 lanes of a quarter-wave reading one
// matrix-core operand column hit distinct banks: odd (in doubles) for the A
// block, the pivot block and the tableau; an odd multiple of 16 floats for the
// FP32 [C | rbar] rows (rows kq = 0..3 of one k-step then start 16 banks
// apart).
__host__ __device__ inline int c_stride(int M1p) { return (M1p / 16) % 2 ? M1p : M1p + 16; }

struct BigLayout {
  size_t r1, r2, total;  // doubles
};

__host__ __device__ inline BigLayout big_layout(int M, int Mr, int nd, int ns, int64_t nnz, int Nc) {
  (void)Mr;
  const int M1p = (M + 2 + 15) / 16 * 16, Mp = (M + 15) / 16 * 16;
  BigLayout L;
  const size_t tab = (size_t)Mp * (Mp + 1);  // padded tableau, odd row stride
  const size_t ndp = (nd + 3) / 4 * 4, ldcf = c_stride(M1p);
  const size_t crb = (ndp * ldcf + 1) / 2;  // [C | rbar_hi | rbar_lo] in FP32
  L.r1 = crb > tab ? crb : tab;
  const size_t gather = 3 * (size_t)ns + nd + 2 * (size_t)Nc;
  const size_t blocks = 16 * (ndp + 1) + 16 * (size_t)M1p;
  const size_t inv = 2 * 16 * (size_t)Mp + 16 * 17 + 2 * (size_t)Mp;  // row / column panels, block inverse, g
  L.r2 = gather > blocks ? gather : blocks;
  L.r2 = L.r2 > inv ? L.r2 : inv;
  L.total = L.r1 + L.r2 + 3 * (size_t)nd + ((size_t)Nc + 1) / 2 + ((size_t)nnz + 1) / 2;
  return L;
}

// SPILL = 0: every array in LDS; 1: region 1 ([C | rbar], then N) of query q
// at spill + q r1 in global memory (L2-resident), the rest in LDS; 2: all of
// them at spill + q total.  __syncthreads orders the workgroup's global
// accesses as it orders LDS ones (one CU, one vector cache).
template <int SPILL>
__global__ void __launch_bounds__(kRunThreads)
    rom_run_large_kernel(RomDev d, int nsteps, const float *__restrict__ gtq, double *__restrict__ xhat,
                         double *__restrict__ hist, int *__restrict__ iters, double *__restrict__ spill) {
  __shared__ double xh[kMaxM + 32], xs[kMaxM];  // xh is zero beyond M
  __shared__ double s_eps, s_g1, s_gn;
  extern __shared__ double dyn[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = kRunThreads / 64;
  // columns of [C | rbar]: M of C, rbar's FP32 high part (M) and low part
  // (M + 1), zeros up to M1p
  const int M = d.M, Mr = d.Mr, nd = d.nd, ns = d.ns, M1p = (M + 2 + 15) / 16 * 16;
  const int nnz = (int)d.nnz;
  const double hdt = 0.5 * (double)d.dt;
  const BigLayout L = big_layout(M, Mr, nd, ns, d.nnz, d.Nc);
  // (a compile-time choice: with every array in LDS the compiler emits LDS
  // instructions for all of them)
  double *R1 = SPILL == 0 ? dyn : spill + blockIdx.x * (SPILL == 1 ? L.r1 : L.total);
  double *R2 = SPILL == 1 ? dyn : R1 + L.r1;
  double *fbar = R2 + L.r2, *fbar_prev = fbar + nd, *xbar_prev = fbar_prev + nd;
  // region 1: [C | rbar_hi | rbar_lo | 0] as FP32 (ndp rows of stride ldcf,
  // zero padded; the two parts of rbar keep its FP64 value to 2^-48, and A
  // times their sum is the sum of the two product columns), then N (Mp x Mp,
  // stride ldT)
  const int ndp = (nd + 3) / 4 * 4, ldcf = c_stride(M1p), lda = ndp + 1;
  float *Cf = reinterpret_cast<float *>(R1);
  double *T = R1;
  double *bt = R2, *pos = R2 + 3 * ns;           // gather phase: pos[0, nd) are the sampled rows
  double *Ab = R2, *Gb = R2 + 16 * (size_t)lda;  // product phase (A block rows of stride lda)
  const int Mp = (M + 15) / 16 * 16, ldT = Mp + 1;
  double *Rp = R2, *Cpn = R2 + 16 * (size_t)Mp, *Pinv = Cpn + 16 * (size_t)Mp;  // inversion
  double *gb = Pinv + 16 * 17, *gb2 = gb + Mp;  // g from rbar's high and low parts
  xhat += (size_t)blockIdx.x * M;
  if (hist) hist += (size_t)blockIdx.x * nsteps * M;
  if (iters) iters += (size_t)blockIdx.x * nsteps;
  float *gt = reinterpret_cast<float *>(xbar_prev + nd);  // this query's Gamma~ per surrogate
  int *eid = reinterpret_cast<int *>(xbar_prev + nd + (d.Nc + 1) / 2);  // surrogate of each entry
  {
    const float *src = gtq ? gtq + (size_t)blockIdx.x * d.Nc : d.gt0;
    for (int t = tid; t < d.Nc; t += kRunThreads) gt[t] = src[t];
    for (int e = tid; e < nnz; e += kRunThreads) eid[e] = d.eid[e];
  }
  for (int m = tid; m < kMaxM + 32; m += kRunThreads) xh[m] = m < M ? xhat[m] : 0.0;
  __syncthreads();

  // positions at xhat in FP64: the sampled rows (p < nd) and the surrogates
  // (Algorithm "HyperPair" preamble), one thread per coordinate
  // With stash, the sampled rows' basis (Phibar) also goes to the first M
  // columns of the FP32 [C | rbar] matrix, where C is then formed in place.
  auto positions = [&](int np, bool stash) {
    constexpr int kB = 32;  // loads in flight per thread
    for (int p = tid; p < np; p += kRunThreads) {
      const double *col = d.pt + p;
      double x0 = d.p0[p], x1 = 0.0;
      for (int m0 = 0; m0 < M; m0 += kB) {
        double v[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) v[u] = m0 + u < M ? col[(size_t)(m0 + u) * d.P] : 0.0;
#pragma unroll
        for (int u = 0; u < kB; u += 2) {
          x0 = fma(v[u], xh[m0 + u], x0);
          x1 = fma(v[u + 1], xh[m0 + u + 1], x1);
        }
        if (stash && p < nd)
#pragma unroll
          for (int u = 0; u < kB; ++u)
            if (m0 + u < M) Cf[(size_t)p * ldcf + m0 + u] = (float)v[u];
      }
      pos[p] = x0 + x1;
    }
  };

  // HyperPair of the paper: each target's list is taken by a group of 8
  // lanes; the separations are formed in FP64 and the pair terms evaluated
  // in FP32, summed in FP64.  With res == false only fbar_out and the
  // sampled rows (xbar_out) are kept.
  auto hyperpair = [&](bool res, double *xbar_out, double *fbar_out) {
    positions(d.P, res);
    __syncthreads();
    for (int t0 = 0; t0 < ns; t0 += kRunThreads / 8) {
      const int t = t0 + (tid >> 3), part = tid & 7;
      if (t < ns) {  // whole groups of 8 lanes are in or out
        const double tx = pos[t], ty = pos[ns + t];
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
        const int e1 = d.off[t + 1];
        for (int e = d.off[t] + part; e < e1; e += 8) {
          const int c = eid[e];
          const float rx = (float)(tx - pos[nd + 2 * c]);
          const float ry = (float)(ty - pos[nd + 2 * c + 1]);
          const float qq = fmaf(rx, rx, fmaf(ry, ry, d.d2));
          const float r = qq > 0.f ? 1.0f / qq : 0.f;  // zero separation adds nothing
          const float g = gt[c] * r, g2 = g * r;
          const float a2 = (rx + rx) * ry, dd = fmaf(ry, ry, -rx * rx);
          s0 += -ry * g;
          s1 += rx * g;
          s2 += g2 * a2;
          s3 += g2 * (dd - d.d2);
          s4 += g2 * (dd + d.d2);
        }
        s0 = sum8(s0);
        s1 = sum8(s1);
        s2 = sum8(s2);
        s3 = sum8(s3);
        s4 = sum8(s4);
        if (part == 0) {
          const double Fx = s0 * kInv2PiD + d.ubar[t], Fy = s1 * kInv2PiD + d.ubar[ns + t];
          fbar_out[t] = Fx;
          fbar_out[ns + t] = Fy;
          if (res) {
            const double r0 = (tx - xbar_prev[t]) - hdt * (Fx + fbar_prev[t]);
            const double r1 = (ty - xbar_prev[ns + t]) - hdt * (Fy + fbar_prev[ns + t]);
            const float h0 = (float)r0, h1 = (float)r1;
            Cf[(size_t)t * ldcf + M] = h0;
            Cf[(size_t)t * ldcf + M + 1] = (float)(r0 - (double)h0);
            Cf[(size_t)(ns + t) * ldcf + M] = h1;
            Cf[(size_t)(ns + t) * ldcf + M + 1] = (float)(r1 - (double)h1);
            bt[3 * t] = s2 * kInv2PiD;
            bt[3 * t + 1] = s3 * kInv2PiD;
            bt[3 * t + 2] = s4 * kInv2PiD;
          }
        }
      }
    }
    if (xbar_out)
      for (int q = tid; q < nd; q += kRunThreads) xbar_out[q] = pos[q];
    __syncthreads();
  };

  hyperpair(false, xbar_prev, fbar_prev);  // previous-step terms for the first step

  const int tcn = M1p / 16, ntile = tcn * (tcn + 1) / 2;
  for (int step = 0; step < nsteps; ++step) {
    int k = 1;
    for (;;) {
      hyperpair(true, nullptr, fbar);
      // C = Phibar - dt/2 B Phibar
      // (in place over the stashed Phibar: one thread per target and mode
      // takes both of the target's rows)
      for (int q = tid; q < ns * M; q += kRunThreads) {
        const int t = q / M, m = q - t * M;
        const double px = Cf[(size_t)t * ldcf + m], py = Cf[(size_t)(ns + t) * ldcf + m];
        const double B00 = bt[3 * t], B01 = bt[3 * t + 1], B10 = bt[3 * t + 2];
        Cf[(size_t)t * ldcf + m] = (float)(px - hdt * (B00 * px + B01 * py));
        Cf[(size_t)(ns + t) * ldcf + m] = (float)(py - hdt * (B10 * px - B00 * py));
      }
      // zero padding: columns past M, rows past nd (and their low parts)
      for (int q = tid; q < nd * (M1p - M - 2); q += kRunThreads) {
        const int row = q / (M1p - M - 2);
        Cf[(size_t)row * ldcf + M + 2 + (q - row * (M1p - M - 2))] = 0.0f;
      }
      for (int q = tid; q < (ndp - nd) * ldcf; q += kRunThreads) Cf[(size_t)nd * ldcf + q] = 0.0f;
      // N' = G'^T G' over 16-row blocks of A (the gather's LDS is free now)
      dbl4 acc[kMaxTiles];
#pragma unroll
      for (int u = 0; u < kMaxTiles; ++u) acc[u] = dbl4{0.0, 0.0, 0.0, 0.0};
      // A's 16-row blocks: the first kPf elements of each thread's share are
      // fetched into registers one block ahead, so their loads run under the
      // previous block's products
      double pf[kPf];
      auto fetch = [&](int rb) {
#pragma unroll
        for (int u = 0; u < kPf; ++u) {
          const int t = tid + u * kRunThreads, r = t / ndp, q = t - r * ndp;
          pf[u] = t < 16 * ndp && rb + r < Mr && q < nd ? d.A[(size_t)(rb + r) * nd + q] : 0.0;
        }
      };
      fetch(0);
      __syncthreads();  // C complete; the gather's terms in region 2 are dead
      for (int rb = 0; rb < Mr; rb += 16) {
        // the previous block's G' has been read (barrier after its N' inputs)
#pragma unroll
        for (int u = 0; u < kPf; ++u) {
          const int t = tid + u * kRunThreads;
          if (t < 16 * ndp) Ab[t + t / ndp] = pf[u];  // row r at r * lda
        }
        for (int t = tid + kPf * kRunThreads; t < 16 * ndp; t += kRunThreads) {
          const int r = t / ndp, q = t - r * ndp;
          Ab[(size_t)r * lda + q] = rb + r < Mr && q < nd ? d.A[(size_t)(rb + r) * nd + q] : 0.0;
        }
        __syncthreads();
        if (rb + 16 < Mr) fetch(rb + 16);
        for (int tj = wave; tj < tcn; tj += nwaves) {
          // G'_blk tile = A_blk [C | rbar] (K = ndp, no guards: both operands
          // are zero padded); four k-steps' operands are loaded before their
          // products issue
          const int j0 = tj * 16, r = lane & 15, kq = lane >> 4;
          const double *ap = Ab + (size_t)r * lda + kq;
          const float *cp = Cf + (size_t)kq * ldcf + j0 + r;
          dbl4 g = dbl4{0.0, 0.0, 0.0, 0.0}, g1 = g, g2 = g, g3 = g;  // independent chains
          int k0 = 0;
          for (; k0 + 16 <= ndp; k0 += 16) {
            double a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              a[u] = ap[k0 + 4 * u];
              b[u] = (double)cp[(size_t)(k0 + 4 * u) * ldcf];
            }
            g = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], g, 0, 0, 0);
            g1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1], b[1], g1, 0, 0, 0);
            g2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[2], b[2], g2, 0, 0, 0);
            g3 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[3], b[3], g3, 0, 0, 0);
          }
          for (; k0 < ndp; k0 += 4) {
            const double a = ap[k0];
            const double b = (double)cp[(size_t)k0 * ldcf];
            g = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, g, 0, 0, 0);
          }
          g = (g + g1) + (g2 + g3);
#pragma unroll
          for (int q = 0; q < 4; ++q) Gb[(4 * q + kq) * M1p + j0 + r] = g[q];
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kMaxTiles; ++u) {
          const int tile = wave + u * nwaves;
          if (tile < ntile) {
            int ti = 0;
            while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
            const int tj = tile - ti * (ti + 1) / 2;
            acc[u] = mfma_tile(16, lane, [&](int i, int q) { return Gb[q * M1p + ti * 16 + i]; },
                               [&](int q, int j) { return Gb[q * M1p + tj * 16 + j]; }, acc[u]);
          }
        }
      }
      __syncthreads();  // C and rbar are dead: N takes region 1
      // N = G^T G into the padded tableau T (Mp x Mp, row stride ldT; the
      // padding is the identity), g = G^T b into gb
      for (int t = tid; t < Mp * Mp; t += kRunThreads) {
        const int i = t / Mp, j = t - i * Mp;
        if (i >= M || j >= M) T[(size_t)i * ldT + j] = i == j ? 1.0 : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kMaxTiles; ++u) {
        const int tile = wave + u * nwaves;
        if (tile < ntile) {
          int ti = 0;
          while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
          const int tj = tile - ti * (ti + 1) / 2;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = ti * 16 + 4 * r + (lane >> 4), col = tj * 16 + (lane & 15);
            const double v = acc[u][r];
            if (row < M && col <= row) {  // lower triangle only: one writer per entry
              T[(size_t)row * ldT + col] = v;
              T[(size_t)col * ldT + row] = v;
            } else if (row == M && col < M) {
              gb[col] = v;  // g = G^T b, b from rbar_hi
            } else if (row == M + 1 && col < M) {
              gb2[col] = v;  // and from rbar_lo
            }
          }
        }
      }
      __syncthreads();
      if (wave == 0) {
        double sq = 0.0;
        for (int i = lane; i < M; i += 64) {
          gb[i] += gb2[i];
          sq += gb[i] * gb[i];
        }
        const double gn = sqrt(wsumd(sq));
        if (lane == 0) s_gn = gn;
      }
      // ---- blocked Gauss-Jordan inversion of T in place (16 x 16 blocks),
      // on the lower block triangle only.  With the swept blocks S (those
      // before K) and the unswept ones U, T holds [[N_SS^-1, N_SS^-1 N_SU],
      // [-N_US N_SS^-1, N_UU - N_US N_SS^-1 N_SU]], so an upper block is the
      // transpose of its mirror, negated when it joins S to U.  For pivot
      // block K: P = T_KK is inverted by one wave (a non-positive pivot leaves
      // its direction out); with P_J = T_KJ (J < K) and Q_I = T_IK (I > K) the
      // panels R_J = P^-1 P_J and C_I = -Q_I P^-1 and the lower trailing
      // blocks (I >= J, I, J != K)
      //   I, J > K:   T_IJ += C_I Q_J^T
      //   I > K > J:  T_IJ += C_I P_J
      //   K > I >= J: T_IJ += P_I^T R_J
      // run on the matrix cores; then T_KK = P^-1, T_KJ = R_J, T_IK = C_I.
      const int nb = Mp / 16;
      for (int kb = 0; kb < nb; ++kb) {
        const int k0 = kb * 16;
        if (wave == 0) {
          // lane (g, j) = 16 g + j holds column j of rows 4 g .. 4 g + 3; per
          // pivot k, row k reaches every lane and column k every row group by
          // lane permutes, and all 64 lanes update their four elements
          const int j = lane & 15, g = lane >> 4;
          double a[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) a[r] = T[(size_t)(k0 + 4 * g + r) * ldT + k0 + j];
#pragma unroll
          for (int k = 0; k < 16; ++k) {
            const int kg = k >> 2, kr = k & 3;
            const double piv = lane_d(a[kr], 16 * kg + k);
            double ip = 0.0;
            if (piv > 0.0) {
              ip = __builtin_amdgcn_rcp(piv);
              ip = fma(ip, fma(-piv, ip, 1.0), ip);
              ip = fma(ip, fma(-piv, ip, 1.0), ip);
            }
            const double rk = __shfl(a[kr], 16 * kg + j);  // a_kj
            double ck[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) ck[r] = __shfl(a[r], 16 * g + k);  // a_ik, i = 4 g + r
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const bool row = 4 * g + r == k, col = j == k;
              const double gen = fma(-ck[r] * ip, rk, a[r]);
              a[r] = row ? (col ? ip : rk * ip) : (col ? -ck[r] * ip : gen);
            }
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) Pinv[(4 * g + r) * 17 + j] = a[r];
        }
        __syncthreads();
        // panels: R_J for J < K (into Rp, 16 x Mp) and C_I for I > K (into Cpn, Mp x 16)
        for (int tb = wave; tb < nb - 1; tb += nwaves) {
          const int bb = tb < kb ? tb : tb + 1, b0 = bb * 16;
          if (bb < kb) {
            const dbl4 r4 = mfma_tile(16, lane, [&](int i, int q) { return Pinv[i * 17 + q]; },
                                      [&](int q, int j) { return T[(size_t)(k0 + q) * ldT + b0 + j]; });
#pragma unroll
            for (int r = 0; r < 4; ++r) Rp[(4 * r + (lane >> 4)) * Mp + b0 + (lane & 15)] = r4[r];
          } else {
            const dbl4 c4 = mfma_tile(16, lane, [&](int i, int q) { return T[(size_t)(b0 + i) * ldT + k0 + q]; },
                                      [&](int q, int j) { return Pinv[q * 17 + j]; });
#pragma unroll
            for (int r = 0; r < 4; ++r) Cpn[(b0 + 4 * r + (lane >> 4)) * 16 + (lane & 15)] = -c4[r];
          }
        }
        __syncthreads();
        // lower trailing blocks; they read row K and column K before the
        // write-back below replaces them
        const int nr = nb - 1, ntri = nr * (nr + 1) / 2;
        for (int tile = wave; tile < ntri; tile += nwaves) {
          int ti = 0;
          while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
          const int tj = tile - ti * (ti + 1) / 2;
          const int bi = ti < kb ? ti : ti + 1, bj = tj < kb ? tj : tj + 1;
          const int i0 = bi * 16, j0 = bj * 16;
          dbl4 t4;
#pragma unroll
          for (int r = 0; r < 4; ++r) t4[r] = T[(size_t)(i0 + 4 * r + (lane >> 4)) * ldT + j0 + (lane & 15)];
          dbl4 u4;
          if (bj > kb)
            u4 = mfma_tile(16, lane, [&](int i, int q) { return Cpn[(i0 + i) * 16 + q]; },
                           [&](int q, int j) { return T[(size_t)(j0 + j) * ldT + k0 + q]; }, t4);
          else if (bi > kb)
            u4 = mfma_tile(16, lane, [&](int i, int q) { return Cpn[(i0 + i) * 16 + q]; },
                           [&](int q, int j) { return T[(size_t)(k0 + q) * ldT + j0 + j]; }, t4);
          else
            u4 = mfma_tile(16, lane, [&](int i, int q) { return T[(size_t)(k0 + q) * ldT + i0 + i]; },
                           [&](int q, int j) { return Rp[q * Mp + j0 + j]; }, t4);
#pragma unroll
          for (int r = 0; r < 4; ++r) T[(size_t)(i0 + 4 * r + (lane >> 4)) * ldT + j0 + (lane & 15)] = u4[r];
        }
        __syncthreads();
        // write back the lower parts of row K and column K and the block inverse
        for (int t = tid; t < 16 * Mp; t += kRunThreads) {
          const int r = t / Mp, c = t - r * Mp;
          if (c < k0) T[(size_t)(k0 + r) * ldT + c] = Rp[r * Mp + c];
          else if (c < k0 + 16) T[(size_t)(k0 + r) * ldT + c] = Pinv[r * 17 + (c - k0)];
          const int i = t >> 4, q = t & 15;  // column panel: row i, column k0 + q
          if (i >= k0 + 16) T[(size_t)i * ldT + k0 + q] = Cpn[i * 16 + q];
        }
        __syncthreads();
      }
      // x = N^-1 g (8 lanes per row)
      for (int o = tid >> 3; o < M; o += kRunThreads / 8) {
        const int part = tid & 7;
        double sx = 0.0;
        for (int j = part; j < M; j += 8) {
          // N^-1 is symmetric and only its lower block triangle (and the
          // diagonal blocks) is held
          const double tv = (j >> 4) <= (o >> 4) ? T[(size_t)o * ldT + j] : T[(size_t)j * ldT + o];
          sx = fma(tv, gb[j], sx);
        }
        sx = sum8(sx);
        if (part == 0) xs[o] = sx;
      }
      __syncthreads();
      if (tid < M) xh[tid] -= d.alpha * xs[tid];
      if (tid == 0) {
        const double gn = s_gn;
        if (k == 1) s_g1 = gn;
        const double g1 = k == 1 ? gn : s_g1;
        s_eps = g1 > 0.0 ? gn / g1 : 0.0;
      }
      __syncthreads();
      ++k;
      if (!(s_eps > d.tol) || k > d.max_iter) break;
      __syncthreads();
    }
    if (tid < M && hist) hist[(size_t)step * M + tid] = xh[tid];
    if (tid == 0 && iters) iters[step] = k - 1;
    // previous-step terms: sampled rows at the accepted xhat, velocity of the
    // last HyperPair evaluation
    __syncthreads();  // the last solve's reads of region 2 are done
    positions(nd, false);
    __syncthreads();
    for (int q = tid; q < nd; q += kRunThreads) {
      xbar_prev[q] = pos[q];
      fbar_prev[q] = fbar[q];
    }
    __syncthreads();
  }
  if (tid < M) xhat[tid] = xh[tid];
}

// dynamic LDS of the run kernel: G' and the tableaux always; the copies of
// the arrays in the LDS-copy variant; the per-entry terms only in the entry-parallel
// gather
// the basis bound of the small kernel that runs a basis of M modes
int mb_of(int M) { return M <= 8 ? 8 : M <= 16 ? 16 : M <= 24 ? 24 : kSmallM; }

size_t solve_lds_bytes(int M, int Mr) {
  return sizeof(double) * ((size_t)Mr * (M + 1) + (size_t)mb_of(M) * 64);
}

// the small run kernel for a basis of M modes
template <int MB>
const void *run_kernel_mb(bool exact, bool ldsa, bool split) {
  if (split) return reinterpret_cast<const void *>(rom_run_kernel<false, true, true, MB>);
  if (exact)
    return ldsa ? reinterpret_cast<const void *>(rom_run_kernel<true, true, false, MB>)
                : reinterpret_cast<const void *>(rom_run_kernel<true, false, false, MB>);
  return ldsa ? reinterpret_cast<const void *>(rom_run_kernel<false, true, false, MB>)
              : reinterpret_cast<const void *>(rom_run_kernel<false, false, false, MB>);
}
const void *run_kernel(int M, bool exact, bool ldsa, bool split) {
  switch (mb_of(M)) {
    case 8: return run_kernel_mb<8>(exact, ldsa, split);
    case 16: return run_kernel_mb<16>(exact, ldsa, split);
    case 24: return run_kernel_mb<24>(exact, ldsa, split);
    default: return run_kernel_mb<kSmallM>(exact, ldsa, split);
  }
}

size_t run_lds_bytes(int M, int Mr, int nd, int ns, int ldc, int64_t nnz, bool entry_par, int64_t nc_table) {
  return solve_lds_bytes(M, Mr) +
         sizeof(double) * ((size_t)Mr * (nd + 1) + (size_t)nd * ldc + 5 * (size_t)nd + 3 * (size_t)ns) +
         sizeof(float) * ((size_t)nd * (M + 1) + (entry_par ? 5 * (size_t)nnz : 0) + (size_t)nc_table);
}
// split runs: the same copies without the whole table's terms, plus the
// slice's terms (5 L floats), its rows (ew / 4 float4 chunks per entry,
// 16-byte aligned), the summed slices (5 ns doubles), each list's slice span
// and local range (4 ns ints) and the waves' sums (5 nt floats per wave)
size_t split_lds_bytes(const RomDev &d, int L, int nt, int64_t nc_table) {
  return run_lds_bytes(d.M, d.Mr, d.nd, d.ns, d.ldc, d.nnz, false, nc_table) + sizeof(double) * 7 * (size_t)d.ns +
         sizeof(float) * 5 * ((size_t)L + (kRunThreads / 64) * (size_t)nt) + 16 + sizeof(float) * (size_t)d.ew * L;
}

// the most targets whose lists meet one slice of L entries
int slice_targets(const std::vector<int> &off, int64_t nnz, int L) {
  int best = 0;
  const int ns = int(off.size()) - 1;
  for (int64_t e0 = 0; e0 < nnz; e0 += L) {
    const int64_t e1 = std::min<int64_t>(nnz, e0 + L);
    // targets t with off[t] < e1 and off[t + 1] > e0
    const int ta = int(std::upper_bound(off.begin() + 1, off.end(), int(e0)) - (off.begin() + 1));
    const int tb = int(std::lower_bound(off.begin(), off.end() - 1, int(e1)) - off.begin()) - 1;
    best = std::max(best, std::min(tb, ns - 1) - ta + 1);
  }
  return best;
}

// Gamma~ of every surrogate for every query: the sum of its members' Gamma
// (FP64 accumulation, members in increasing id order).
__global__ void reassign_kernel(int nq, int64_t n, int Nc, const int *__restrict__ mem_off,
                                const int *__restrict__ mem_ids, const float *__restrict__ gamma_q,
                                float *__restrict__ gt_q) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nq * Nc) return;
  const int q = int(t / Nc), c = int(t - (int64_t)q * Nc);
  const float *g = gamma_q + (size_t)q * n;
  double s = 0.0;
  for (int k = mem_off[c]; k < mem_off[c + 1]; ++k) s += (double)g[mem_ids[k]];
  gt_q[t] = (float)s;
}

}  // namespace

struct ptrom_rom {
  ptrom_ctx *ctx = nullptr;
  RomDev d{};
  void *buf = nullptr;
  int *members = nullptr;  // device: mem_off [Nc+1] then mem_ids
  int64_t n_bodies = 0;
  size_t max_dyn_lds = 0;      // dynamic LDS the run kernel may take on this device
  size_t max_dyn_lds_big = 0;  // same for the larger-basis kernel
  int coop = 0;                // the device takes cooperative launches
  int split = 0;               // workgroups per query of split runs: 0 automatic, 1 never
  unsigned split_polls = 0;    // failed barrier checks before a split run aborts (0: kSplitPolls)
  std::vector<int> off;        // host copy of the list offsets [ns + 1]
};

extern "C" int ptrom_rom_create(ptrom_ctx *ctx, const ptrom_rom_desc *desc, ptrom_rom **out) {
  if (!ctx) return PTROM_EINVAL;
  ctx->err.clear();
  if (!desc || !out) return ctx->fail(PTROM_EINVAL, "NULL argument");
  const ptrom_rom_desc &s = *desc;
  if (s.M < 1 || s.M > kMaxM || s.Mr < s.M || s.Mr > kMaxMr || s.ns < 1 || s.ns > (1 << 20))
    return ctx->fail(PTROM_EINVAL, "need 1 <= M <= 112, M <= Mr <= 256, 1 <= ns <= 2^20");
  if (s.jac_mode == PTROM_JAC_EXACT && (s.M > kSmallM || s.Mr > kSmallMr))
    return ctx->fail(PTROM_EINVAL, "the exact Jacobian needs M <= 32 and Mr <= 64");
  const int nd = 2 * s.ns;
  if (s.Nc < 0 || s.nnz < 0 || s.Nc > kMaxN || s.nnz > (int64_t(1) << 31) - 1 ||
      nd + 2 * s.Nc > (int64_t(1) << 31) - 1)
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
  // entry rows: r0 = xbar0_i - xqt0_c, Gamma~_c, D = Phibar_i - Phit_c
  // (differences in FP64); component k of entry e at ((k / 4) nnz + e) 4 +
  // k % 4 (chunk-major, paper Jacobian) or e ew + k (row-major, exact)
  const size_t ne = size_t(s.nnz > 0 ? s.nnz : 1);
  const bool cm = s.jac_mode != PTROM_JAC_EXACT;
  std::vector<float> ent(ne * ew, 0.0f);
  auto at = [&](int64_t e, int k) -> float & {
    return cm ? ent[(size_t(k / 4) * ne + size_t(e)) * 4 + size_t(k % 4)] : ent[size_t(e) * ew + size_t(k)];
  };
  for (int i = 0; i < s.ns; ++i)
    for (int64_t e = s.off[i]; e < s.off[i + 1]; ++e) {
      const int64_t c = s.ids[e];
      at(e, 0) = float(s.xbar0[i] - s.xqt0[2 * c]);
      at(e, 1) = float(s.xbar0[s.ns + i] - s.xqt0[2 * c + 1]);
      at(e, 2) = float(s.Gt[c]);
      const int32_t cid = int32_t(c);
      std::memcpy(&at(e, 3), &cid, sizeof(cid));
      for (int m = 0; m < M; ++m) {
        at(e, 4 + 2 * m) = float(s.Phibar[(size_t)i * M + m] - s.Phit[(size_t)(2 * c) * M + m]);
        at(e, 5 + 2 * m) = float(s.Phibar[(size_t)(s.ns + i) * M + m] - s.Phit[(size_t)(2 * c + 1) * M + m]);
      }
    }

  // point form: sampled rows then surrogate coordinates, mode-major FP64
  const int64_t P = nd + 2 * s.Nc;
  std::vector<double> pt(size_t(M) * P), p0(P);
  for (int q = 0; q < nd; ++q) {
    p0[q] = s.xbar0[q];
    for (int m = 0; m < M; ++m) pt[(size_t)m * P + q] = s.Phibar[(size_t)q * M + m];
  }
  for (int64_t c = 0; c < s.Nc; ++c)
    for (int k = 0; k < 2; ++k) {
      p0[nd + 2 * c + k] = s.xqt0[2 * c + k];
      for (int m = 0; m < M; ++m) pt[(size_t)m * P + nd + 2 * c + k] = s.Phit[(size_t)(2 * c + k) * M + m];
    }
  std::vector<int> etg(size_t(s.nnz > 0 ? s.nnz : 1), 0), eid(etg.size(), 0);
  for (int i = 0; i < s.ns; ++i)
    for (int64_t e = s.off[i]; e < s.off[i + 1]; ++e) {
      etg[e] = i;
      eid[e] = int(s.ids[e]);
    }
  // Morton order (16 bits per axis over the points' bounding box) of n
  // points x[i * stride], x[i * stride + off2]: order[r] = the r-th point
  auto morton_order = [](int64_t n, const double *x, int64_t stride, int64_t off2) {
    auto spread = [](uint32_t v) {
      uint64_t u = v & 0xFFFFu;
      u = (u | (u << 8)) & 0x00FF00FFull;
      u = (u | (u << 4)) & 0x0F0F0F0Full;
      u = (u | (u << 2)) & 0x33333333ull;
      u = (u | (u << 1)) & 0x55555555ull;
      return u;
    };
    double lo[2] = {x[0], x[off2]}, hi[2] = {x[0], x[off2]};
    for (int64_t i = 0; i < n; ++i)
      for (int k = 0; k < 2; ++k) {
        const double v = x[i * stride + k * off2];
        lo[k] = std::min(lo[k], v);
        hi[k] = std::max(hi[k], v);
      }
    std::vector<std::pair<uint64_t, int>> key(static_cast<size_t>(n));
    for (int64_t i = 0; i < n; ++i) {
      uint32_t g[2];
      for (int k = 0; k < 2; ++k) {
        const double w = hi[k] > lo[k] ? (x[i * stride + k * off2] - lo[k]) / (hi[k] - lo[k]) : 0.0;
        g[k] = uint32_t(std::min(65535.0, std::max(0.0, std::floor(w * 65536.0))));
      }
      key[i] = {spread(g[0]) | (spread(g[1]) << 1), int(i)};
    }
    std::sort(key.begin(), key.end());
    std::vector<int> order(static_cast<size_t>(n));
    for (int64_t r = 0; r < n; ++r) order[r] = key[r].second;
    return order;
  };
  // the hook's target order: lexicographic in each list's eight largest
  // surrogate ids, so targets whose lists share their far-field clusters sit
  // together and neighbouring waves read the same records
  std::vector<int> tord(size_t(s.ns));
  {
    constexpr int kKey = 8;
    std::vector<std::array<int64_t, kKey>> key(size_t(s.ns));
    for (int i = 0; i < s.ns; ++i) {
      std::vector<int64_t> l(s.ids + s.off[i], s.ids + s.off[i + 1]);
      const size_t k = std::min<size_t>(kKey, l.size());
      std::partial_sort(l.begin(), l.begin() + k, l.end(), std::greater<int64_t>());
      key[i].fill(-1);
      for (size_t j = 0; j < k; ++j) key[i][j] = l[j];
      tord[i] = i;
    }
    std::stable_sort(tord.begin(), tord.end(), [&](int a, int b) { return key[a] > key[b]; });
  }
  // record order of the hook's surrogate table: Morton order of the
  // surrogates' reference positions
  std::vector<int> rec(size_t(s.Nc > 0 ? s.Nc : 1), 0), erec(etg.size(), 0);
  if (s.Nc > 0) {
    const std::vector<int> order = morton_order(s.Nc, s.xqt0, 2, 1);
    for (int64_t r = 0; r < s.Nc; ++r) rec[order[r]] = int(r);
    // each target's entries in record order: neighbouring lanes read
    // neighbouring records (the hook's sums run in this order)
    for (int i = 0; i < s.ns; ++i) {
      for (int64_t e = s.off[i]; e < s.off[i + 1]; ++e) erec[e] = rec[s.ids[e]];
      std::sort(erec.begin() + s.off[i], erec.begin() + s.off[i + 1]);
    }
  }
  // the hook's target groups: consecutive targets of tord, at most
  // kGroupTargets, closed early when the union of their records would pass
  // kUnionCap (a target whose own list passes it forms a group alone and
  // reads the global table)
  std::vector<int> gstart{0}, ustart{0}, urec;
  std::vector<unsigned short> eloc(erec.size(), 0);
  {
    std::vector<int> stamp(size_t(s.Nc > 0 ? s.Nc : 1), -1), loc(size_t(s.Nc > 0 ? s.Nc : 1), 0);
    int r = 0;
    while (r < s.ns) {
      const int g = int(gstart.size()) - 1;
      std::vector<int> u;
      int r1 = r;
      while (r1 < s.ns && r1 - r < kGroupTargets) {
        const int t = tord[r1];
        size_t add = 0;
        for (int64_t e = s.off[t]; e < s.off[t + 1]; ++e) add += stamp[erec[e]] != g;
        if (r1 > r && u.size() + add > size_t(kUnionCap)) break;
        for (int64_t e = s.off[t]; e < s.off[t + 1]; ++e)
          if (stamp[erec[e]] != g) {
            stamp[erec[e]] = g;
            u.push_back(erec[e]);
          }
        ++r1;
      }
      std::sort(u.begin(), u.end());
      if (u.size() <= size_t(kUnionCap)) {
        for (size_t k = 0; k < u.size(); ++k) loc[u[k]] = int(k);
        for (int q = r; q < r1; ++q)
          for (int64_t e = s.off[tord[q]]; e < s.off[tord[q] + 1]; ++e) eloc[e] = (unsigned short)loc[erec[e]];
      }
      urec.insert(urec.end(), u.begin(), u.end());
      gstart.push_back(r1);
      ustart.push_back(int(urec.size()));
      r = r1;
    }
    if (urec.empty()) urec.push_back(0);
  }
  // the hook's entries in target order tord: toff[r] .. toff[r + 1) are
  // those of target tord[r]
  std::vector<int> toff(size_t(s.ns) + 1, 0);
  {
    std::vector<int> erec_t(erec.size(), 0);
    std::vector<unsigned short> eloc_t(eloc.size(), 0);
    for (int q = 0; q < s.ns; ++q) {
      const int t = tord[q];
      int64_t k = toff[q];
      for (int64_t e = s.off[t]; e < s.off[t + 1]; ++e, ++k) {
        erec_t[k] = erec[e];
        eloc_t[k] = eloc[e];
      }
      toff[q + 1] = int(k);
    }
    erec.swap(erec_t);
    eloc.swap(eloc_t);
  }
  std::vector<double> ubar(nd, 0.0);
  if (s.ubar)
    for (int q = 0; q < nd; ++q) ubar[q] = s.ubar[q];
  std::vector<float> gt0(size_t(s.Nc > 0 ? s.Nc : 1), 0.0f);
  for (int64_t c = 0; c < s.Nc; ++c) gt0[c] = float(s.Gt[c]);

  auto rom = new ptrom_rom();
  rom->ctx = ctx;
  rom->off = off32;
  {
    // dynamic LDS the run kernel may request: the device's per-workgroup
    // limit minus the kernel's static LDS
    int maxsh = 0;
    if (hipDeviceGetAttribute(&maxsh, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device) != hipSuccess)
      maxsh = 64 * 1024;
    size_t stat = 0;
    std::vector<const void *> kernels;
    for (int Mq : {8, 16, 24, kSmallM})
      for (int v = 0; v < 5; ++v) kernels.push_back(run_kernel(Mq, v & 1, v & 2, v == 4));
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
    hipFuncAttributes fb{};
    const void *bigs[3] = {reinterpret_cast<const void *>(rom_run_large_kernel<0>),
                           reinterpret_cast<const void *>(rom_run_large_kernel<1>),
                           reinterpret_cast<const void *>(rom_run_large_kernel<2>)};
    size_t sb = 0;
    for (const void *k : bigs)
      if (hipFuncGetAttributes(&fb, k) == hipSuccess) sb = std::max(sb, fb.sharedSizeBytes);
    size_t dynb = size_t(maxsh) > sb ? size_t(maxsh) - sb : 0;
    for (const void *k : bigs)
      if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, int(dynb)) != hipSuccess) {
        dynb = 64 * 1024 > sb ? 64 * 1024 - sb : 0;
        (void)hipGetLastError();
        break;
      }
    rom->max_dyn_lds_big = dynb;
    rom->max_dyn_lds = dyn;
    if (hipDeviceGetAttribute(&rom->coop, hipDeviceAttributeCooperativeLaunch, ctx->device) != hipSuccess)
      rom->coop = 0;
  }
  RomDev &d = rom->d;
  d.M = M; d.Mr = s.Mr; d.ns = s.ns; d.nd = nd; d.jac_mode = s.jac_mode; d.max_iter = s.max_iter;
  d.ew = ew; d.nnz = s.nnz; d.Nc = int(s.Nc);
  d.ldc = (M + 1 + 3) / 4 * 4;
  {
    // run-kernel gather: groups of G lanes per target, chosen to minimise
    // (rounds of the workgroup's waves over the targets) x (entry passes of the
    // longest list)
    int64_t maxlen = 0;
    for (int i = 0; i < s.ns; ++i) maxlen = std::max<int64_t>(maxlen, s.off[i + 1] - s.off[i]);
    d.maxlen = int(std::min<int64_t>(maxlen, int64_t(1) << 30));
    int64_t best = -1;
    for (int G : {16, 32, 64}) {
      const int64_t per_round = int64_t(kRunThreads / 64) * (64 / G);
      const int64_t cost = (s.ns + per_round - 1) / per_round * std::max<int64_t>(1, (maxlen + G - 1) / G);
      if (best < 0 || cost < best) {
        best = cost;
        d.glanes = G;
      }
    }
  }
  d.d2 = float(s.delta) * float(s.delta);
  d.dt = float(s.dt);
  d.tol = s.tol; d.alpha = s.alpha;

  const size_t bytes[] = {align256(phibar.size() * 4), align256(xbar0.size() * 4), align256(ent.size() * 4),
                          align256(off32.size() * 4), align256(size_t(s.Mr) * nd * 8),
                          align256(nd * 8), align256(nd * 8), align256(nd * 8),
                          align256(size_t(nd) * ((M + 4) / 4 * 4) * 8), align256(pt.size() * 8),
                          align256(p0.size() * 8), align256(etg.size() * 4), align256(eid.size() * 4),
                          align256(gt0.size() * 4), align256(ubar.size() * 8), align256(size_t(P) * 8),
                          align256(size_t(s.Nc > 0 ? s.Nc : 1) * 32), align256(rec.size() * 4),
                          align256(erec.size() * 4), align256(tord.size() * 4), align256(gstart.size() * 4),
                          align256(ustart.size() * 4), align256(urec.size() * 4), align256(eloc.size() * 2),
                          align256(toff.size() * 4)};
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
  d.P = int(P); d.pt = (double *)ptrs[9]; d.p0 = (double *)ptrs[10]; d.etg = (int *)ptrs[11];
  d.eid = (int *)ptrs[12]; d.gt0 = (float *)ptrs[13]; d.ubar = (double *)ptrs[14]; d.pos = (double *)ptrs[15];
  d.spk = (double *)ptrs[16];
  d.rec = (int *)ptrs[17];
  d.erec = (int *)ptrs[18];
  d.tord = (int *)ptrs[19];
  d.ngroups = int(gstart.size()) - 1;
  d.umax = 1;
  for (int g = 0; g < d.ngroups; ++g)
    if (ustart[g + 1] - ustart[g] <= kUnionCap) d.umax = std::max(d.umax, ustart[g + 1] - ustart[g]);
  d.gstart = (int *)ptrs[20];
  d.ustart = (int *)ptrs[21];
  d.urec = (int *)ptrs[22];
  d.eloc = (unsigned short *)ptrs[23];
  d.toff = (int *)ptrs[24];
  hipError_t e = hipMemcpy(ptrs[0], phibar.data(), phibar.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ptrs[1], xbar0.data(), xbar0.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ptrs[2], ent.data(), ent.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ptrs[3], off32.data(), off32.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ptrs[4], s.A, size_t(s.Mr) * nd * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ptrs[9], pt.data(), pt.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ptrs[10], p0.data(), p0.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ptrs[11], etg.data(), etg.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ptrs[12], eid.data(), eid.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ptrs[13], gt0.data(), gt0.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ptrs[14], ubar.data(), ubar.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ptrs[17], rec.data(), rec.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ptrs[18], erec.data(), erec.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ptrs[19], tord.data(), tord.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ptrs[20], gstart.data(), gstart.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ptrs[21], ustart.data(), ustart.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ptrs[22], urec.data(), urec.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess && !eloc.empty()) e = hipMemcpy(ptrs[23], eloc.data(), eloc.size() * 2, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ptrs[24], toff.data(), toff.size() * 4, hipMemcpyHostToDevice);
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
  if (rom->members) hipFree(rom->members);
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
  if (d.jac_mode == PTROM_JAC_EXACT) {
    hipLaunchKernelGGL(gather_kernel<true>, dim3(gg), dim3(256), 0, st, d, xhat, xbar_prev, fbar_prev, xbar, fbar,
                       rbar, C);
  } else {
    // point form: positions once per surrogate, 4 bytes per list entry
    hipLaunchKernelGGL(point_positions_kernel, dim3((unsigned)((d.P + 255) / 256)), dim3(256), 0, st, d, xhat,
                       d.pos);
    hipLaunchKernelGGL(gather_point_kernel, dim3((unsigned)d.ngroups), dim3(64 * kGroupTargets),
                       d.umax * sizeof(dbl4), st, d, d.pos, xbar_prev, fbar_prev, xbar, fbar, rbar, C);
  }
  PTROM_CHECK_HIP(ctx, hipGetLastError());
  return PTROM_OK;
}

namespace {

__global__ void split_zero_kernel(unsigned *p, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// Workgroups per query of a split run (paper Jacobian, small basis, arrays in
// LDS): about kSplitEntries entries per slice, at most kSplitMaxW, widened
// until the slice fits next to the other LDS copies; 1 (no split) when the
// automatic choice meets fewer than kSplitMinEntries entries (below that
// the exchange costs more than the slices save), the device takes no
// cooperative launch, the grid would not be resident at once, or the
// barrier count would pass 2^32.  *lds: the split launch's dynamic LDS.
constexpr int64_t kSplitEntries = 1024;
constexpr int64_t kSplitMinEntries = 4096;  // automatic splits start here
constexpr int kSplitMaxW = 64;
int split_width(ptrom_rom *rom, int nq, int nsteps, int64_t table, int *W_out, size_t *lds) {
  const RomDev &d = rom->d;
  *W_out = 1;
  if (rom->split == 1 || !rom->coop || d.nnz < 1 || d.jac_mode != PTROM_JAC_PAPER || d.M > kSmallM ||
      d.Mr > kSmallMr || nq < 1)
    return PTROM_OK;
  if (rom->split == 0 && d.nnz < kSplitMinEntries) return PTROM_OK;
  int W = rom->split >= 2 ? rom->split : int(std::min<int64_t>(16, (d.nnz + kSplitEntries - 1) / kSplitEntries));
  if (W < 2) return PTROM_OK;
  auto L = [&](int w) { return int((d.nnz + w - 1) / w); };
  auto bytes_at = [&](int w) { return split_lds_bytes(d, L(w), slice_targets(rom->off, d.nnz, L(w)), table); };
  while (W <= kSplitMaxW && bytes_at(W) > rom->max_dyn_lds) ++W;
  if (W > kSplitMaxW) return PTROM_OK;
  const int64_t barriers = 1 + int64_t(nsteps) * d.max_iter;
  if (int64_t(W) * barriers >= (int64_t(1) << 32) - 1) return PTROM_OK;
  const size_t bytes = bytes_at(W);
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, run_kernel(d.M, false, true, true),
                                                   kRunThreads, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return PTROM_OK;
  }
  if (int64_t(W) * nq > int64_t(per_cu) * rom->ctx->num_cus) return PTROM_OK;
  *W_out = W;
  *lds = bytes;
  return PTROM_OK;
}

// One launch of the device-resident loop over nq queries (one workgroup
// each, or W per query in split runs); gtq NULL means the training
// circulations of the entries.
int launch_run(ptrom_rom *rom, int nq, const float *gtq, int nsteps, double *xhat, double *xhat_hist,
               int32_t *iters, hipStream_t st) {
  ptrom_ctx *ctx = rom->ctx;
  const RomDev &d = rom->d;
  if (d.M > kSmallM || d.Mr > kSmallMr) {
    // the query's arrays in LDS when they fit; otherwise [C | rbar] and N
    // (the largest) in global memory, or, if the rest still does not fit,
    // every array there
    const BigLayout L = big_layout(d.M, d.Mr, d.nd, d.ns, d.nnz, d.Nc);
    size_t lds = L.total * sizeof(double), glob = 0;
    int mode = 0;
    if (lds > rom->max_dyn_lds_big) {
      mode = (L.total - L.r1) * sizeof(double) <= rom->max_dyn_lds_big ? 1 : 2;
      glob = size_t(nq) * (mode == 1 ? L.r1 : L.total) * sizeof(double);
      lds = mode == 1 ? (L.total - L.r1) * sizeof(double) : 0;
      if (int rc = ctx->reserve(glob + 256)) return rc;
    }
    double *sp = mode ? static_cast<double *>(ctx->ws) : nullptr;
    if (mode == 0)
      hipLaunchKernelGGL(rom_run_large_kernel<0>, dim3(nq), dim3(kRunThreads), lds, st, d, nsteps, gtq, xhat,
                         xhat_hist, iters, sp);
    else if (mode == 1)
      hipLaunchKernelGGL(rom_run_large_kernel<1>, dim3(nq), dim3(kRunThreads), lds, st, d, nsteps, gtq, xhat,
                         xhat_hist, iters, sp);
    else
      hipLaunchKernelGGL(rom_run_large_kernel<2>, dim3(nq), dim3(kRunThreads), lds, st, d, nsteps, gtq, xhat,
                         xhat_hist, iters, sp);
    PTROM_CHECK_HIP(ctx, hipGetLastError());
    return PTROM_OK;
  }
  const int64_t table = gtq ? d.Nc : 0;
  // entry-parallel gather (paper Jacobian) when its per-entry terms fit in LDS
  // next to the other copies; otherwise the grouped gather
  int entry_par = d.jac_mode == PTROM_JAC_PAPER &&
                  run_lds_bytes(d.M, d.Mr, d.nd, d.ns, d.ldc, d.nnz, true, table) <= rom->max_dyn_lds;
  const size_t lds = run_lds_bytes(d.M, d.Mr, d.nd, d.ns, d.ldc, d.nnz, entry_par != 0, table);
  const int use_lds = lds <= rom->max_dyn_lds;
  if (!use_lds) {
    entry_par = 0;
    // the global-memory fallback has one scratch set: a single query only
    if (nq != 1 || gtq)
      return ctx->fail(PTROM_EINVAL, "batched queries need the run arrays to fit in LDS (sample set too large)");
  }
  const bool ex = d.jac_mode == PTROM_JAC_EXACT;
  if (!ex && use_lds) {
    int W = 1;
    size_t slds = 0;
    if (int rc = split_width(rom, nq, nsteps, table, &W, &slds)) return rc;
    if (W > 1) {
      // tagged slice sums (two parities) and the abort flag in the
      // workspace, zeroed before the launch (tags start at 1)
      SplitArgs sp;
      sp.W = W;
      sp.L = int((d.nnz + W - 1) / W);
      sp.nt = slice_targets(rom->off, d.nnz, sp.L);
      const size_t npart = 2 * size_t(nq) * W * 5 * size_t(d.ns);
      const size_t words = 2 * npart + 1;  // 32-bit words, abort flag last
      if (int rc = ctx->reserve(words * sizeof(unsigned) + 256)) return rc;
      unsigned *w32 = static_cast<unsigned *>(ctx->ws);
      sp.part = reinterpret_cast<unsigned long long *>(w32);
      sp.abort = w32 + 2 * npart;
      sp.max_polls = rom->split_polls ? rom->split_polls : kSplitPolls;
      const int zb = int(std::min<size_t>(1024, (words + 255) / 256));
      hipLaunchKernelGGL(split_zero_kernel, dim3(zb), dim3(256), 0, st, w32, (long long)words);
      PTROM_CHECK_HIP(ctx, hipGetLastError());
      int ep = 0;
      void *args[] = {const_cast<RomDev *>(&d), &nsteps, &ep, &gtq, &xhat, &xhat_hist, &iters, &sp};
      PTROM_CHECK_HIP(ctx, hipLaunchCooperativeKernel(run_kernel(d.M, false, true, true),
                                                      dim3(unsigned(nq) * W), dim3(kRunThreads), args,
                                                      unsigned(slds), st));
      return PTROM_OK;
    }
  }
  const size_t shmem = use_lds ? lds : solve_lds_bytes(d.M, d.Mr);
  const int ep = ex ? 0 : entry_par;
  SplitArgs one;
  int epv = ep;
  void *args[] = {const_cast<RomDev *>(&d), &nsteps, &epv, &gtq, &xhat, &xhat_hist, &iters, &one};
  PTROM_CHECK_HIP(ctx, hipLaunchKernel(run_kernel(d.M, ex, use_lds != 0, false), dim3(nq), dim3(kRunThreads), args,
                                       shmem, st));
  return PTROM_OK;
}

}  // namespace

extern "C" int ptrom_rom_run(ptrom_rom *rom, int nsteps, double *xhat, double *xhat_hist,
                             int32_t *iters, ptrom_stream stream) {
  if (!rom) return PTROM_EINVAL;
  ptrom_ctx *ctx = rom->ctx;
  ctx->err.clear();
  if (!xhat || nsteps < 0) return ctx->fail(PTROM_EINVAL, "xhat required and nsteps >= 0");
  if (hipSetDevice(ctx->device) != hipSuccess) return ctx->fail(PTROM_EHIP, "hipSetDevice");
  return launch_run(rom, 1, nullptr, nsteps, xhat, xhat_hist, iters, (hipStream_t)stream);
}

extern "C" int ptrom_rom_set_split(ptrom_rom *rom, int workgroups, uint32_t max_polls) {
  if (!rom) return PTROM_EINVAL;
  rom->ctx->err.clear();
  if (workgroups < 0 || workgroups > kSplitMaxW)
    return rom->ctx->fail(PTROM_EINVAL, "workgroups per query must be 0 (automatic) .. 64");
  rom->split = workgroups;
  rom->split_polls = max_polls;
  return PTROM_OK;
}

extern "C" int ptrom_rom_split_plan(ptrom_rom *rom, int batched_nq, int nsteps, int32_t *workgroups) {
  if (!rom) return PTROM_EINVAL;
  ptrom_ctx *ctx = rom->ctx;
  ctx->err.clear();
  if (!workgroups || batched_nq < 0 || nsteps < 0) return ctx->fail(PTROM_EINVAL, "workgroups required, nq and nsteps >= 0");
  int W = 1;
  size_t lds = 0;
  const int nq = batched_nq > 0 ? batched_nq : 1;
  if (int rc = split_width(rom, nq, nsteps, batched_nq > 0 ? rom->d.Nc : 0, &W, &lds)) return rc;
  *workgroups = W;
  return PTROM_OK;
}

extern "C" int ptrom_rom_members(ptrom_rom *rom, int64_t n, const int64_t *mem_off, const int64_t *mem_ids) {
  if (!rom) return PTROM_EINVAL;
  ptrom_ctx *ctx = rom->ctx;
  ctx->err.clear();
  const int Nc = rom->d.Nc;
  if (n < 1 || n > kMaxN || !mem_off || (Nc > 0 && !mem_ids)) return ctx->fail(PTROM_EINVAL, "bad membership");
  if (mem_off[0] != 0) return ctx->fail(PTROM_EINVAL, "mem_off must start at 0");
  for (int c = 0; c < Nc; ++c)
    if (mem_off[c + 1] <= mem_off[c]) return ctx->fail(PTROM_EINVAL, "every surrogate needs at least one member");
  const int64_t nmem = mem_off[Nc];
  if (nmem > (int64_t(1) << 31) - 1) return ctx->fail(PTROM_EINVAL, "too many members");
  std::vector<int> host(size_t(Nc) + 1 + size_t(nmem));
  for (int c = 0; c <= Nc; ++c) host[c] = int(mem_off[c]);
  for (int64_t k = 0; k < nmem; ++k) {
    if (mem_ids[k] < 0 || mem_ids[k] >= n) return ctx->fail(PTROM_EINVAL, "member id out of [0, n)");
    host[size_t(Nc) + 1 + size_t(k)] = int(mem_ids[k]);
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return ctx->fail(PTROM_EHIP, "hipSetDevice");
  if (rom->members) {
    PTROM_CHECK_HIP(ctx, hipDeviceSynchronize());
    PTROM_CHECK_HIP(ctx, hipFree(rom->members));
    rom->members = nullptr;
  }
  if (hipMalloc(&rom->members, host.size() * sizeof(int)) != hipSuccess)
    return ctx->fail(PTROM_ENOMEM, "membership allocation");
  PTROM_CHECK_HIP(ctx, hipMemcpy(rom->members, host.data(), host.size() * sizeof(int), hipMemcpyHostToDevice));
  rom->n_bodies = n;
  return PTROM_OK;
}

extern "C" int ptrom_rom_reassign(ptrom_rom *rom, int nq, const float *gamma_q, float *gt_q, ptrom_stream stream) {
  if (!rom) return PTROM_EINVAL;
  ptrom_ctx *ctx = rom->ctx;
  ctx->err.clear();
  if (!rom->members) return ctx->fail(PTROM_EINVAL, "membership not set (ptrom_rom_members)");
  if (nq < 1 || !gamma_q || !gt_q) return ctx->fail(PTROM_EINVAL, "nq >= 1 and both arrays required");
  if (hipSetDevice(ctx->device) != hipSuccess) return ctx->fail(PTROM_EHIP, "hipSetDevice");
  const int Nc = rom->d.Nc;
  const int64_t total = int64_t(nq) * Nc;
  if (total == 0) return PTROM_OK;
  const int *mem_off = rom->members, *mem_ids = rom->members + Nc + 1;
  hipLaunchKernelGGL(reassign_kernel, dim3(unsigned((total + 255) / 256)), dim3(256), 0, (hipStream_t)stream, nq,
                     rom->n_bodies, Nc, mem_off, mem_ids, gamma_q, gt_q);
  PTROM_CHECK_HIP(ctx, hipGetLastError());
  return PTROM_OK;
}

extern "C" int ptrom_rom_run_batched(ptrom_rom *rom, int nq, const float *gt_q, int nsteps, double *xhat,
                                     double *xhat_hist, int32_t *iters, ptrom_stream stream) {
  if (!rom) return PTROM_EINVAL;
  ptrom_ctx *ctx = rom->ctx;
  ctx->err.clear();
  if (nq < 1 || nq > 65535 || !gt_q || !xhat || nsteps < 0)
    return ctx->fail(PTROM_EINVAL, "1 <= nq <= 65535, gt_q and xhat required, nsteps >= 0");
  if (hipSetDevice(ctx->device) != hipSuccess) return ctx->fail(PTROM_EHIP, "hipSetDevice");
  return launch_run(rom, nq, gt_q, nsteps, xhat, xhat_hist, iters, (hipStream_t)stream);
}
