// Each-unordered-pair-once evaluation of one block pair, shared by the
// single-system kernels and the batched parametric kernel.
//
// The pair terms are antisymmetric (velocity, Jacobian product, adjoint) or
// symmetric (the Jacobian's self blocks, the stream function) under exchange
// of target and source, so one evaluation of a pair gives both bodies'
// terms.  A
// workgroup takes targets [tgt0, tgt0 + 256 K) and sources
// [src0, src0 + 256 K) (disjoint ranges), stages 64 sources at a time in LDS
// and sweeps them in 64 steps, lane l taking source (l + t) mod 64 at step t.
// The reaction accumulators travel with their sources: every step rotates
// them one lane to the left inside the add (v_add_f32 with the DPP
// wave_rol:1 modifier), so after the sweep lane l holds the complete
// reaction on source (l - 1) mod 64 and no per-step shared-memory traffic is
// needed.
#pragma once

#include "pair_core.h"

namespace ptrom {

constexpr float kFar = 1.0e15f;  // position of padding bodies (never coincides with a real one)

// Forward and reaction terms of one pair; t: target data, s: source data.
// Factors of 2 and 1/2 are written as scalings of one operation's result
// (2 * (a * b), 0.5f * (a * b)).  Where a translation unit is built with
// FP32 denormals flushed and IEEE mode off (the single-system kernels), the
// compiler folds such a scaling into the instruction's output modifier at no
// cost.  Scaling by a power of two is exact, so the values are those of the
// plain expressions.
template <int OP>
__device__ __forceinline__ void interact_sym(const float *t, const float *s, float d2, float *acc,
                                             float *react) {
  const float dx = t[0] - s[0];
  const float dy = t[1] - s[1];
  const float q = fmaf(dx, dx, fmaf(dy, dy, d2));
  if constexpr (OP == OP_PSI) {
    // the log is even in r: both bodies gain the other's Gamma times it
    const float L = __builtin_amdgcn_logf(q);
    acc[0] = fmaf(s[2], L, acc[0]);
    react[0] = fmaf(t[4], L, react[0]);
    return;
  }
  const float r = __builtin_amdgcn_rcpf(q);
  if constexpr (OP == OP_VEL) {
    const float gj = s[2] * r, gi = t[4] * r;
    acc[0] = fmaf(-dy, gj, acc[0]);
    acc[1] = fmaf(dx, gj, acc[1]);
    react[0] = fmaf(dy, gi, react[0]);
    react[1] = fmaf(-dx, gi, react[1]);
  } else if constexpr (OP == OP_JVP) {
    const float ex = t[2] - s[3];
    const float ey = t[3] - s[4];
    const float r2 = 2.0f * r;  // 2 / q
    const float c = fmaf(dx, ex, dy * ey) * r2;
    const float wx = fmaf(-c, dx, ex);
    const float wy = fmaf(-c, dy, ey);
    const float gj = 0.5f * (s[2] * r2), gi = 0.5f * (t[4] * r2);
    acc[0] = fmaf(-gj, wy, acc[0]);
    acc[1] = fmaf(gj, wx, acc[1]);
    react[0] = fmaf(gi, wy, react[0]);
    react[1] = fmaf(-gi, wx, react[1]);
  } else if constexpr (OP == OP_BJAC) {
    // entries 0..2 of q^-2 [2 rx ry, ry^2 - rx^2 - d^2; ry^2 - rx^2 + d^2, -2 rx ry]
    // (Gamma r) r as in the one-sided kernel, which keeps Gamma / q^2 finite
    // wherever that one is
    const float h0 = 2.0f * (dx * dy);
    const float m = fmaf(dy, dy, -dx * dx);
    const float h1 = m - d2, h2 = m + d2;
    const float gj = (s[2] * r) * r, gi = (t[4] * r) * r;
    acc[0] = fmaf(gj, h0, acc[0]);
    acc[1] = fmaf(gj, h1, acc[1]);
    acc[2] = fmaf(gj, h2, acc[2]);
    react[0] = fmaf(gi, h0, react[0]);
    react[1] = fmaf(gi, h1, react[1]);
    react[2] = fmaf(gi, h2, react[2]);
  } else if constexpr (OP == OP_VBJ) {
    // velocity (antisymmetric reaction) and self block (symmetric reaction)
    const float gj = s[2] * r, gi = t[4] * r;
    acc[0] = fmaf(-dy, gj, acc[0]);
    acc[1] = fmaf(dx, gj, acc[1]);
    react[0] = fmaf(dy, gi, react[0]);
    react[1] = fmaf(-dx, gi, react[1]);
    const float h0 = 2.0f * (dx * dy);
    const float m = fmaf(dy, dy, -dx * dx);
    const float h1 = m - d2, h2 = m + d2;
    const float gj2 = gj * r, gi2 = gi * r;
    acc[2] = fmaf(gj2, h0, acc[2]);
    acc[3] = fmaf(gj2, h1, acc[3]);
    acc[4] = fmaf(gj2, h2, acc[4]);
    react[2] = fmaf(gi2, h0, react[2]);
    react[3] = fmaf(gi2, h1, react[3]);
    react[4] = fmaf(gi2, h2, react[4]);
  } else {
    const float qx = fmaf(s[2], t[2], -t[4] * s[3]);
    const float qy = fmaf(s[2], t[3], -t[4] * s[4]);
    const float c = fmaf(dx, qy, -dy * qx) * (r + r);
    const float tx = r * fmaf(-c, dx, qy);
    const float ty = r * fmaf(-c, dy, -qx);
    acc[0] += tx;
    acc[1] += ty;
    react[0] -= tx;
    react[1] -= ty;
    acc[2] = fmaf(r, fmaf(s[3], dy, -s[4] * dx), acc[2]);
    react[2] = fmaf(r, fmaf(t[3], dx, -t[2] * dy), react[2]);
  }
}

// lane l receives lane (l + 1) mod 64's value, added to `add`
__device__ __forceinline__ float rotate_add(float v, float add) {
  const int r = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x134 /* wave_rol:1 */, 0xF, 0xF, false);
  return __builtin_bit_cast(float, r) + add;
}

// One off-diagonal block pair of a system of n bodies.  Targets (block I)
// start at tgt0, sources (block J) at src0.  The targets' forward sums go to
// Fo[a n + i], the reactions on the sources to Ro[a n + j] (a = accumulator;
// the caller points Fo and Ro at the block pair's slots).  s_src and
// racc_lds are the workgroup's LDS staging; all threads call this with
// uniform arguments.
template <int OP, int K>
__device__ __forceinline__ void sym_block_pair(int n, const float *__restrict__ xy, const float *__restrict__ gam,
                                               const float *__restrict__ aux, float d2, int tgt0, int src0,
                                               float4 (*s_src)[2], float (*racc_lds)[Traits<OP>::NACC][64],
                                               float *__restrict__ Fo, float *__restrict__ Ro) {
  using T = Traits<OP>;
  constexpr int NA = T::NACC, NS = T::NSRC;
  constexpr int TB = kBlock * K;
  const int tid = local_id(), lane = tid & 63, wave = tid >> 6;
  // targets of block I: x, y, aux0, aux1, Gamma (padding: far away, no strength)
  float tg[K][5];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = tgt0 + k * kBlock + tid;
    const bool ok = i < n;
    tg[k][0] = ok ? xy[i] : 2.0f * kFar;
    tg[k][1] = ok ? xy[n + i] : 2.0f * kFar;
    if constexpr (NS == 5) {
      tg[k][2] = ok ? aux[i] : 0.0f;
      tg[k][3] = ok ? aux[n + i] : 0.0f;
    } else {
      tg[k][2] = tg[k][3] = 0.0f;
    }
    tg[k][4] = ok ? gam[i] : 0.0f;
  }
  // forward partials: plain FP32 over a 256-source tile, then added to the
  // compensated sums
  float sum[K][NA], cmp[K][NA], part[K][NA];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int a = 0; a < NA; ++a) sum[k][a] = cmp[k][a] = part[k][a] = 0.0f;

  for (int u = 0; u < TB; u += 64) {
    const int j0 = src0 + u;
    if (j0 >= n) break;
    __syncthreads();
    if (tid < 64) {
      const int j = j0 + tid;
      const bool ok = j < n;
      const float4 a = make_float4(ok ? xy[j] : kFar, ok ? xy[n + j] : kFar, ok ? gam[j] : 0.0f,
                                   (NS == 5 && ok) ? aux[j] : 0.0f);
      const float4 b = make_float4((NS == 5 && ok) ? aux[n + j] : 0.0f, 0.0f, 0.0f, 0.0f);
      s_src[tid][0] = a;
      s_src[tid][1] = b;
      s_src[tid + 64][0] = a;
      s_src[tid + 64][1] = b;
    }
    __syncthreads();
    float racc[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) racc[a] = 0.0f;
    const float4(*src)[2] = s_src + lane;
#pragma unroll 8
    for (int t = 0; t < 64; ++t) {
      const float4 A = src[t][0];
      float s[5] = {A.x, A.y, A.z, A.w, NS == 5 ? src[t][1].x : 0.0f};
      float react[NA];
#pragma unroll
      for (int a = 0; a < NA; ++a) react[a] = 0.0f;
#pragma unroll
      for (int k = 0; k < K; ++k) interact_sym<OP>(tg[k], s, d2, part[k], react);
#pragma unroll
      for (int a = 0; a < NA; ++a) racc[a] = rotate_add(racc[a], react[a]);
    }
    // lane l now holds the reaction on source (l - 1) mod 64
#pragma unroll
    for (int a = 0; a < NA; ++a) racc_lds[wave][a][(lane + 63) & 63] = racc[a];
    if ((u & (kTile - 64)) == kTile - 64 || u + 64 >= TB || j0 + 64 >= n) {
#pragma unroll
      for (int k = 0; k < K; ++k)
#pragma unroll
        for (int a = 0; a < NA; ++a) {
          kahan_add(sum[k][a], cmp[k][a], part[k][a]);
          part[k][a] = 0.0f;
        }
    }
    __syncthreads();
    if (tid < 64 && j0 + tid < n) {
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        float s = 0.0f, c = 0.0f;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) kahan_add(s, c, racc_lds[w][a][tid]);
        Ro[(size_t)a * n + j0 + tid] = s - c;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = tgt0 + k * kBlock + tid;
    if (i < n)
#pragma unroll
      for (int a = 0; a < NA; ++a) Fo[(size_t)a * n + i] = sum[k][a] - cmp[k][a];
  }
}

}  // namespace ptrom

