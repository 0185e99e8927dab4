// Device-side building blocks of the all-pairs Biot-Savart kernels, shared
// by the single-system grid kernels and the batched persistent kernel.
#pragma once

#include "internal.h"

namespace ptrom {

// The work-item's index in its workgroup and the workgroup's index, read
// from their hardware registers.  The each-pair-once kernels are built with
// IEEE mode off, and the device library's id functions (threadIdx,
// blockIdx) are then not inlined into them.
__device__ __forceinline__ int local_id() { return (int)__builtin_amdgcn_workitem_id_x(); }
__device__ __forceinline__ int group_id() { return (int)__builtin_amdgcn_workgroup_id_x(); }

constexpr float kInv2Pi = 0.159154943091895335768883763372514362f;

template <int OP> struct Traits;
template <> struct Traits<OP_VEL> { static constexpr int NSRC = 3, NTGT = 2, NACC = 2; };
template <> struct Traits<OP_BJAC> { static constexpr int NSRC = 3, NTGT = 2, NACC = 3; };
template <> struct Traits<OP_JVP> { static constexpr int NSRC = 5, NTGT = 4, NACC = 2; };
template <> struct Traits<OP_VJP> { static constexpr int NSRC = 5, NTGT = 5, NACC = 3; };
template <> struct Traits<OP_PSI> { static constexpr int NSRC = 3, NTGT = 2, NACC = 1; };
// velocity and the self block in one pass: fx, fy, then the block's B00, B01, B10
template <> struct Traits<OP_VBJ> { static constexpr int NSRC = 3, NTGT = 2, NACC = 5; };

// accumulators of an operation (host side)
inline int nacc(int op) {
  switch (op) {
    case OP_VEL: return Traits<OP_VEL>::NACC;
    case OP_BJAC: return Traits<OP_BJAC>::NACC;
    case OP_JVP: return Traits<OP_JVP>::NACC;
    case OP_PSI: return Traits<OP_PSI>::NACC;
    case OP_VBJ: return Traits<OP_VBJ>::NACC;
    default: return Traits<OP_VJP>::NACC;
  }
}

// -ln(2)/(4 pi): the stream-function sum is accumulated with log2
constexpr float kPsiScale = -0.0551589363396979447f;

__device__ __forceinline__ void kahan_add(float &s, float &c, float x) {
  const float y = x - c;
  const float t = s + y;
  c = (t - s) - y;
  s = t;
}

// One target-source interaction.  t: target data (x, y, extras), s: source
// data (x, y, Gamma, extras), d2 = delta^2.  `self` marks the self pair,
// whose contribution is forced to zero (only used when MASK).
template <int OP, bool MASK>
__device__ __forceinline__ void interact(const float *t, const float *s, float d2, float *acc,
                                         bool self) {
  const float dx = t[0] - s[0];
  const float dy = t[1] - s[1];
  const float q = fmaf(dx, dx, fmaf(dy, dy, d2));
  if constexpr (OP == OP_PSI) {
    // Gamma_j log2(|r|^2 + delta^2) (stream function of the regularized flow)
    float L = __builtin_amdgcn_logf(q);
    if (MASK) L = self ? 0.0f : L;
    acc[0] = fmaf(s[2], L, acc[0]);
    return;
  }
  float r = __builtin_amdgcn_rcpf(q);
  if (MASK) r = self ? 0.0f : r;
  if constexpr (OP == OP_VEL) {
    const float g = s[2] * r;
    acc[0] = fmaf(-dy, g, acc[0]);
    acc[1] = fmaf(dx, g, acc[1]);
  } else if constexpr (OP == OP_BJAC) {
    const float g2 = s[2] * r * r;
    const float a2 = (dx + dx) * dy;
    const float dd = fmaf(dy, dy, -dx * dx);
    acc[0] = fmaf(g2, a2, acc[0]);
    acc[1] = fmaf(g2, dd - d2, acc[1]);
    acc[2] = fmaf(g2, dd + d2, acc[2]);
  } else if constexpr (OP == OP_VBJ) {
    const float g = s[2] * r;
    acc[0] = fmaf(-dy, g, acc[0]);
    acc[1] = fmaf(dx, g, acc[1]);
    const float g2 = g * r;
    const float a2 = (dx + dx) * dy;
    const float dd = fmaf(dy, dy, -dx * dx);
    acc[2] = fmaf(g2, a2, acc[2]);
    acc[3] = fmaf(g2, dd - d2, acc[3]);
    acc[4] = fmaf(g2, dd + d2, acc[4]);
  } else if constexpr (OP == OP_JVP) {
    // du/dr = R (I - 2 r r^T / q) / q with R the rotation by +90 degrees, so
    // H e = R (e - c r) / q,  c = 2 (r . e) / q,  e = v_i - v_j.
    const float ex = t[2] - s[3];
    const float ey = t[3] - s[4];
    const float c = fmaf(dx, ex, dy * ey) * (r + r);
    const float wx = fmaf(-c, dx, ex);
    const float wy = fmaf(-c, dy, ey);
    const float g = s[2] * r;
    acc[0] = fmaf(-g, wy, acc[0]);
    acc[1] = fmaf(g, wx, acc[1]);
  } else {
    // H^T q = (I - 2 r r^T / q) R^T q / q with q = Gamma_j w_k - Gamma_k w_j,
    // R^T q = (q_y, -q_x); and the circulation partial -w_j . R r / q.
    const float qx = fmaf(s[2], t[2], -t[4] * s[3]);
    const float qy = fmaf(s[2], t[3], -t[4] * s[4]);
    const float c = fmaf(dx, qy, -dy * qx) * (r + r);
    const float wx = fmaf(-c, dx, qy);
    const float wy = fmaf(-c, dy, -qx);
    acc[0] = fmaf(r, wx, acc[0]);
    acc[1] = fmaf(r, wy, acc[1]);
    acc[2] = fmaf(r, fmaf(s[3], dy, -s[4] * dx), acc[2]);
  }
}

template <int OP>
__device__ __forceinline__ void load_source(int n, int j, const float *__restrict__ xy,
                                            const float *__restrict__ gam,
                                            const float *__restrict__ aux, float *s) {
  s[0] = xy[j];
  s[1] = xy[n + j];
  s[2] = gam[j];
  if constexpr (Traits<OP>::NSRC == 5) {
    s[3] = aux[j];
    s[4] = aux[n + j];
  }
}

// Final layout of the scaled accumulators of one target.
template <int OP>
__device__ __forceinline__ void store_final(int n, int i, const float *v, float *__restrict__ out,
                                            float *__restrict__ out2) {
  if constexpr (OP == OP_VEL || OP == OP_JVP) {
    out[i] = v[0] * kInv2Pi;
    out[n + i] = v[1] * kInv2Pi;
  } else if constexpr (OP == OP_BJAC) {
    out[i] = v[0] * kInv2Pi;
    out[n + i] = v[1] * kInv2Pi;
    out[2 * n + i] = v[2] * kInv2Pi;
    out[3 * n + i] = -v[0] * kInv2Pi;
  } else if constexpr (OP == OP_PSI) {
    out[i] = v[0] * kPsiScale;
  } else if constexpr (OP == OP_VBJ) {
    out[i] = v[0] * kInv2Pi;
    out[n + i] = v[1] * kInv2Pi;
    out2[i] = v[2] * kInv2Pi;
    out2[n + i] = v[3] * kInv2Pi;
    out2[2 * n + i] = v[4] * kInv2Pi;
    out2[3 * n + i] = -v[2] * kInv2Pi;
  } else {
    out[i] = v[0] * kInv2Pi;
    out[n + i] = v[1] * kInv2Pi;
    out2[i] = v[2] * kInv2Pi;
  }
}


// Compensated sums over sources [sb, se) for the K targets of this lane
// (targets tgt0 + k*kBlock + threadIdx.x).  Called by all threads of a
// workgroup with uniform arguments (LDS staging synchronises the block).
template <int OP, int K, int STAGING>
__device__ __forceinline__ void pair_block(int n, const float *__restrict__ xy,
                                           const float *__restrict__ gam,
                                           const float *__restrict__ aux, float d2, int tgt0,
                                           int sb, int se, float *lds,
                                           float (&res)[K][Traits<OP>::NACC]) {
  using T = Traits<OP>;
  constexpr int NS = T::NSRC, NT = T::NTGT, NA = T::NACC;
  const int tid = local_id();
  float tg[K][NT];
  int ti[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = tgt0 + k * kBlock + tid;
    ti[k] = i;
    const int ic = i < n ? i : n - 1;
    tg[k][0] = xy[ic];
    tg[k][1] = xy[n + ic];
    if constexpr (OP == OP_JVP || OP == OP_VJP) {
      tg[k][2] = aux[ic];
      tg[k][3] = aux[n + ic];
    }
    if constexpr (OP == OP_VJP) tg[k][4] = gam[ic];
  }
  float sum[K][NA], cmp[K][NA];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int a = 0; a < NA; ++a) sum[k][a] = cmp[k][a] = 0.0f;
  const int tgt_end = tgt0 + kBlock * K;

  for (int ts = sb; ts < se; ts += kTile) {
    const int cnt = min(kTile, se - ts);
    if constexpr (STAGING == STAGE_LDS) {
      __syncthreads();
      if (tid < cnt) {
        float s[NS];
        load_source<OP>(n, ts + tid, xy, gam, aux, s);
#pragma unroll
        for (int q = 0; q < NS; ++q) lds[q * kTile + tid] = s[q];
      }
      __syncthreads();
    }
    float part[K][NA];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int a = 0; a < NA; ++a) part[k][a] = 0.0f;

    const bool diag = (ts < tgt_end) && (tgt0 < ts + cnt);
    if (cnt == kTile && !diag) {
#pragma unroll 4
      for (int jj = 0; jj < kTile; ++jj) {
        float s[NS];
        if constexpr (STAGING == STAGE_LDS) {
#pragma unroll
          for (int q = 0; q < NS; ++q) s[q] = lds[q * kTile + jj];
        } else {
          load_source<OP>(n, ts + jj, xy, gam, aux, s);
        }
#pragma unroll
        for (int k = 0; k < K; ++k) interact<OP, false>(tg[k], s, d2, part[k], false);
      }
    } else {
      for (int jj = 0; jj < cnt; ++jj) {
        float s[NS];
        if constexpr (STAGING == STAGE_LDS) {
#pragma unroll
          for (int q = 0; q < NS; ++q) s[q] = lds[q * kTile + jj];
        } else {
          load_source<OP>(n, ts + jj, xy, gam, aux, s);
        }
        const int j = ts + jj;
#pragma unroll
        for (int k = 0; k < K; ++k) interact<OP, true>(tg[k], s, d2, part[k], j == ti[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int a = 0; a < NA; ++a) kahan_add(sum[k][a], cmp[k][a], part[k][a]);
  }
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int a = 0; a < NA; ++a) res[k][a] = sum[k][a] - cmp[k][a];
}

}  // namespace ptrom
