// All-pairs kernels that evaluate every unordered pair once.
//
// The Biot-Savart pair terms are antisymmetric: with r = x_i - x_j the term
// body j receives from body i is the term body i receives from j with
// Gamma_j replaced by Gamma_i and the sign flipped (velocity: u(-r) = -u(r);
// Jacobian product: H(-r) = H(r) and v_j - v_i = -(v_i - v_j); adjoint:
// q_ji = -q_ij).  The self blocks of the Jacobian are symmetric instead:
// H(-r) = H(r), so body j's block gains Gamma_i H(r) with the same sign; so
// is the stream function's log(|r|^2 + delta^2).
// The body index range is cut into blocks of 256*K; block pairs (I, J) with
// J > I are evaluated once, each interaction adding the forward term to the
// target (registers) and the reaction term to the source; diagonal blocks
// (I, I) use the ordinary one-sided tile.
// Workgroups pop items from a device counter (persistent launch).  Item q
// of the nb (nb - 1) / 2 off-diagonal block pairs is decoded arithmetically:
// the items run by decreasing block distance d = J - I.  The diagonal blocks
// come last, each cut into K slices of 256 targets, so that the small
// slices fill the launch's tail.  Forward sums land in
// F[J][.][N], reactions in R[I][.][N]; a final kernel adds, per body, its
// forward slots J >= block(b) and reaction slots I < block(b) in a fixed
// order (Kahan compensated sums over 8 contiguous slot ranges, combined in
// range order), so results are bitwise reproducible.
#include "pair_sym_core.h"

namespace ptrom {
namespace {

__global__ void sym_reset_kernel(unsigned long long *__restrict__ counter) {
  if (local_id() == 0) counter[0] = 0;
}

// Block pair of item q: with e = floor((sqrt(8 q + 1) - 1) / 2) the items
// e (e + 1) / 2 .. e (e + 1) / 2 + e share the distance d = nb - 1 - e, and
// I runs from 0 in that group.
__device__ __forceinline__ void tri_item(long long q, int nb, int &I, int &J) {
  long long e = (long long)((__builtin_sqrt(8.0 * double(q) + 1.0) - 1.0) * 0.5);
  while (e * (e + 1) / 2 > q) --e;
  while ((e + 1) * (e + 2) / 2 <= q) ++e;
  I = int(q - e * (e + 1) / 2);
  J = I + (nb - 1 - int(e));
}

template <int OP, int K>
__global__ void __launch_bounds__(kBlock)
    pair_sym_kernel(int n, const float *__restrict__ xy, const float *__restrict__ gam,
                    const float *__restrict__ aux, float d2, int nb, unsigned long long *__restrict__ counter,
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
  __shared__ unsigned long long item_s;
  const int tid = local_id();
  // the off-diagonal block pairs come first (the items of distance >= 1),
  // then every diagonal block in K slices of 256 targets
  const long long offd = (long long)nb * (nb - 1) / 2;
  const long long items = offd + (long long)nb * K;

  for (;;) {
    if (tid == 0) item_s = atomicAdd(counter, 1ull);
    __syncthreads();
    const long long it = (long long)item_s;
    __syncthreads();
    if (it >= items) break;
    if (it >= offd) {
      // diagonal block I, target slice h (one target per lane) against the
      // block's sources: the one-sided tile, the self pair masked.  The
      // slices write disjoint targets of the block's forward slot.
      const int I = int((it - offd) / K), h = int((it - offd) % K);
      const int tgt0 = I * TB + h * kBlock;
      if (tgt0 >= n) continue;  // uniform: a slice past the last body
      float res[1][NA];
      pair_block<OP, 1, STAGE_LDS>(n, xy, gam, aux, d2, tgt0, I * TB, min(n, I * TB + TB), lds_diag, res);
      const int i = tgt0 + tid;
      if (i < n)
#pragma unroll
        for (int a = 0; a < NA; ++a) F[(size_t)(I * NA + a) * n + i] = res[0][a];
      continue;
    }
    int I, J;
    tri_item(it, nb, I, J);  // J > I
    sym_block_pair<OP, K>(n, xy, gam, aux, d2, I * TB, J * TB, s_src, racc_lds, F + (size_t)J * NA * n,
                          R + (size_t)I * NA * n);
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
  const int lane = local_id() & 63, slice = local_id() >> 6;
  const int b = group_id() * 64 + lane;
  const bool ok = b < n;
  const int B = (group_id() * 64) / tb;
  const int nf = nb - B;  // forward slots come first
  const int q0 = (slice * nb) / kSlices, q1 = ((slice + 1) * nb) / kSlices;
#pragma unroll
  for (int a = 0; a < NA; ++a) {
    float s = 0.0f, c = 0.0f;
    if (ok) {
      // eight slots' loads in flight, then their compensated sum in slot order
      for (int q = q0; q < q1; q += 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int qq = q + u;
          v[u] = qq >= q1   ? 0.0f
                 : qq < nf ? F[(size_t)((B + qq) * NA + a) * n + b]
                           : R[(size_t)((qq - nf) * NA + a) * n + b];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (q + u < q1) kahan_add(s, c, v[u]);
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
  auto *counter = reinterpret_cast<unsigned long long *>(R + (size_t)nb * NA * n);
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
  return size_t(2 * nb * nacc(op) * n + 64);
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
    case OP_VBJ: return launch_sym_op<OP_VBJ>(k, n, xy, gamma, aux, d2, grid, ws, out, out2, stream);
    case OP_PSI: return launch_sym_op<OP_PSI>(k, n, xy, gamma, aux, d2, grid, ws, out, out2, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ptrom
