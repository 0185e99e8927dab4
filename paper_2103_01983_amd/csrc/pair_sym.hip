// All-pairs kernels that evaluate every unordered pair once.
//
// The Biot-Savart pair terms are antisymmetric: with r = x_i - x_j the term
// body j receives from body i is the term body i receives from j with
// Gamma_j replaced by Gamma_i and the sign flipped (velocity: u(-r) = -u(r);
// Jacobian product: H(-r) = H(r) and v_j - v_i = -(v_i - v_j); adjoint:
// q_ji = -q_ij).  The self blocks of the Jacobian are symmetric instead:
// H(-r) = H(r), so body j's block gains Gamma_i H(r) with the same sign.  The body index range is cut into blocks of 256*K; block
// pairs (I, J) with J > I are evaluated once, each interaction adding the
// forward term to the target (registers) and the reaction term to the
// source; diagonal blocks (I, I) use the ordinary one-sided tile.
//
// Inside an off-diagonal item a workgroup stages 64 sources of block J in
// LDS and each wave sweeps them in 64 steps, lane l taking source
// (l + t) mod 64 at step t.  The reaction accumulators travel with their
// sources: every step rotates them one lane to the left inside the add
// (v_add_f32 with the DPP wave_rol:1 modifier), so after the sweep lane l
// holds the complete reaction on source (l - 1) mod 64 and no per-step
// shared-memory traffic is needed.  Workgroups pop items from a device
// counter (persistent launch).  Forward sums land in F[J][.][N], reactions
// in R[I][.][N]; a final kernel adds, per body, its forward slots
// J >= block(b) and reaction slots I < block(b) in a fixed order (Kahan
// compensated sums over 8 contiguous slot ranges, combined in range order), so
// results are bitwise reproducible.
#include "pair_core.h"

namespace ptrom {
namespace {

constexpr float kFar = 1.0e15f;  // position of padding bodies (never coincides with a real one)

// Forward and reaction terms of one pair; t: target data, s: source data.
template <int OP>
__device__ __forceinline__ void interact_sym(const float *t, const float *s, float d2, float *acc,
                                             float *react) {
  const float dx = t[0] - s[0];
  const float dy = t[1] - s[1];
  const float q = fmaf(dx, dx, fmaf(dy, dy, d2));
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
    const float c = fmaf(dx, ex, dy * ey) * (r + r);
    const float wx = fmaf(-c, dx, ex);
    const float wy = fmaf(-c, dy, ey);
    const float gj = s[2] * r, gi = t[4] * r;
    acc[0] = fmaf(-gj, wy, acc[0]);
    acc[1] = fmaf(gj, wx, acc[1]);
    react[0] = fmaf(gi, wy, react[0]);
    react[1] = fmaf(-gi, wx, react[1]);
  } else if constexpr (OP == OP_BJAC) {
    // entries 0..2 of q^-2 [2 rx ry, ry^2 - rx^2 - d^2; ry^2 - rx^2 + d^2, -2 rx ry]
    // (Gamma r) r as in the one-sided kernel, which keeps Gamma / q^2 finite
    // wherever that one is
    const float h0 = (dx + dx) * dy;
    const float m = fmaf(dy, dy, -dx * dx);
    const float h1 = m - d2, h2 = m + d2;
    const float gj = (s[2] * r) * r, gi = (t[4] * r) * r;
    acc[0] = fmaf(gj, h0, acc[0]);
    acc[1] = fmaf(gj, h1, acc[1]);
    acc[2] = fmaf(gj, h2, acc[2]);
    react[0] = fmaf(gi, h0, react[0]);
    react[1] = fmaf(gi, h1, react[1]);
    react[2] = fmaf(gi, h2, react[2]);
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

__global__ void sym_reset_kernel(int *__restrict__ counter) {
  if (threadIdx.x == 0) counter[0] = 0;
}

template <int OP, int K>
__global__ void __launch_bounds__(kBlock)
    pair_sym_kernel(int n, const float *__restrict__ xy, const float *__restrict__ gam,
                    const float *__restrict__ aux, float d2, int nb, int *__restrict__ counter,
                    float *__restrict__ F, float *__restrict__ R) {
  using T = Traits<OP>;
  constexpr int NA = T::NACC, NS = T::NSRC;
  constexpr int TB = kBlock * K;
  // the 64 staged sources, stored twice in a row (entries l and l + 64 are the
  // same source), so lane l reads entry l + t at step t with no wrap-around:
  // one address per lane and constant offsets per step
  __shared__ float4 s_src[128][2];
  __shared__ float racc_lds[kBlock / 64][NA][64];
  __shared__ float lds_diag[NS * kTile];
  __shared__ int item_s;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  for (;;) {
    if (tid == 0) item_s = atomicAdd(counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(item_s);
    __syncthreads();
    if (it >= nb * nb) break;
    const int I = it / nb, J = it % nb;
    if (J < I) continue;
    const int tgt0 = I * TB;
    if (J == I) {
      float res[K][NA];
      pair_block<OP, K, STAGE_LDS>(n, xy, gam, aux, d2, tgt0, tgt0, min(n, tgt0 + TB), lds_diag, res);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int i = tgt0 + k * kBlock + tid;
        if (i < n)
#pragma unroll
          for (int a = 0; a < NA; ++a) F[(size_t)(J * NA + a) * n + i] = res[k][a];
      }
      continue;
    }
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
    float sum[K][NA], cmp[K][NA];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int a = 0; a < NA; ++a) sum[k][a] = cmp[k][a] = 0.0f;

    const int src0 = J * TB;
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
      float part[K][NA], racc[NA];
#pragma unroll
      for (int k = 0; k < K; ++k)
#pragma unroll
        for (int a = 0; a < NA; ++a) part[k][a] = 0.0f;
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
#pragma unroll
      for (int k = 0; k < K; ++k)
#pragma unroll
        for (int a = 0; a < NA; ++a) kahan_add(sum[k][a], cmp[k][a], part[k][a]);
      __syncthreads();
      if (tid < 64 && j0 + tid < n) {
#pragma unroll
        for (int a = 0; a < NA; ++a) {
          float s = 0.0f, c = 0.0f;
#pragma unroll
          for (int w = 0; w < kBlock / 64; ++w) kahan_add(s, c, racc_lds[w][a][tid]);
          R[(size_t)(I * NA + a) * n + j0 + tid] = s - c;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = tgt0 + k * kBlock + tid;
      if (i < n)
#pragma unroll
        for (int a = 0; a < NA; ++a) F[(size_t)(J * NA + a) * n + i] = sum[k][a] - cmp[k][a];
    }
  }
}

// Per body b (in block B = b / tb) the slots to add are, in this order, its
// forward slots J = B .. nb-1 and its reaction slots I = 0 .. B-1.  A
// workgroup takes 64 consecutive bodies (tb is a multiple of 64, so one wave
// shares B) and kSlices contiguous ranges of that slot list; each range is
// added with Kahan compensation, then the ranges are combined in slice order.
constexpr int kSlices = 8;

template <int OP>
__global__ void __launch_bounds__(64 * kSlices)
    sym_reduce_kernel(int n, int tb, int nb, const float *__restrict__ F, const float *__restrict__ R,
                      float *__restrict__ out, float *__restrict__ out2) {
  constexpr int NA = Traits<OP>::NACC;
  __shared__ float part[NA][kSlices][64];
  const int lane = threadIdx.x & 63, slice = threadIdx.x >> 6;
  const int b = blockIdx.x * 64 + lane;
  const bool ok = b < n;
  const int B = (blockIdx.x * 64) / tb;
  const int nf = nb - B;  // forward slots come first
  const int q0 = (slice * nb) / kSlices, q1 = ((slice + 1) * nb) / kSlices;
#pragma unroll
  for (int a = 0; a < NA; ++a) {
    float s = 0.0f, c = 0.0f;
    if (ok) {
      for (int q = q0; q < q1; ++q) {
        const float v = q < nf ? F[(size_t)((B + q) * NA + a) * n + b] : R[(size_t)((q - nf) * NA + a) * n + b];
        kahan_add(s, c, v);
      }
    }
    part[a][slice][lane] = s - c;
  }
  __syncthreads();
  if (slice == 0 && ok) {
    float v[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      float s = 0.0f, c = 0.0f;
#pragma unroll
      for (int w = 0; w < kSlices; ++w) kahan_add(s, c, part[a][w][lane]);
      v[a] = s - c;
    }
    store_final<OP>(n, b, v, out, out2);
  }
}

template <int OP, int K>
hipError_t launch_sym_t(int n, const float *xy, const float *gam, const float *aux, float d2,
                        int grid, float *ws, float *out, float *out2, hipStream_t st) {
  constexpr int NA = Traits<OP>::NACC;
  const int tb = kBlock * K;
  const int nb = (n + tb - 1) / tb;
  float *F = ws;
  float *R = ws + (size_t)nb * NA * n;
  int *counter = reinterpret_cast<int *>(R + (size_t)nb * NA * n);
  hipLaunchKernelGGL(sym_reset_kernel, dim3(1), dim3(64), 0, st, counter);
  hipLaunchKernelGGL((pair_sym_kernel<OP, K>), dim3(grid), dim3(kBlock), 0, st, n, xy, gam, aux, d2, nb,
                     counter, F, R);
  hipLaunchKernelGGL(sym_reduce_kernel<OP>, dim3((n + 63) / 64), dim3(64 * kSlices), 0, st, n, tb, nb, F, R, out,
                     out2);
  return hipGetLastError();
}

template <int OP>
hipError_t launch_sym_op(int k, int n, const float *xy, const float *gam, const float *aux, float d2,
                         int grid, float *ws, float *out, float *out2, hipStream_t st) {
  if (k == 2) return launch_sym_t<OP, 2>(n, xy, gam, aux, d2, grid, ws, out, out2, st);
  if (k == 4) return launch_sym_t<OP, 4>(n, xy, gam, aux, d2, grid, ws, out, out2, st);
  return launch_sym_t<OP, 1>(n, xy, gam, aux, d2, grid, ws, out, out2, st);
}

}  // namespace

size_t pair_sym_ws_floats(int op, int k, int64_t n) {
  const int64_t tb = kBlock * int64_t(k);
  const int64_t nb = (n + tb - 1) / tb;
  const int na = (op == OP_VJP || op == OP_BJAC) ? 3 : 2;
  return size_t(2 * nb * na * n + 64);
}

hipError_t launch_pair_sym(int op, int k, int waves_per_simd, int num_cus, int64_t n64, const float *xy,
                           const float *gamma, const float *aux, float delta, float *out, float *out2,
                           float *ws, size_t ws_floats, hipStream_t stream) {
  if (ws_floats < pair_sym_ws_floats(op, k, n64)) return hipErrorInvalidValue;
  const int n = int(n64);
  const float d2 = delta * delta;
  const int grid = num_cus * (waves_per_simd < 1 ? 1 : waves_per_simd);
  switch (op) {
    case OP_VEL: return launch_sym_op<OP_VEL>(k, n, xy, gamma, aux, d2, grid, ws, out, out2, stream);
    case OP_JVP: return launch_sym_op<OP_JVP>(k, n, xy, gamma, aux, d2, grid, ws, out, out2, stream);
    case OP_VJP: return launch_sym_op<OP_VJP>(k, n, xy, gamma, aux, d2, grid, ws, out, out2, stream);
    case OP_BJAC: return launch_sym_op<OP_BJAC>(k, n, xy, gamma, aux, d2, grid, ws, out, out2, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ptrom
