// Many independent parametric instances (own N_b, own core delta_b) in one
// persistent launch per velocity evaluation, every unordered pair of an
// instance evaluated once.  The host cuts every instance into blocks of 256 K
// bodies (K targets per lane and the workgroups per CU come from the tuning
// table, keyed by the pair-weighted mean instance size sum N_b^2 / sum N_b)
// and lists its block pairs (instance, I, J), J >= I, sorted by pair
// count (largest first), once per instance set; every workgroup then pops
// items from a device counter until the list is exhausted, so large and
// small instances share the chip without a tail.  Off-diagonal items run
// the each-pair-once sweep (forward sums to the targets, rotated reactions
// to the sources); diagonal items the one-sided tile.  Instance b keeps one
// slot per block, P_b[slot][2][N_b]: a body of block B receives forward
// sums in slots J >= B and reactions in slots I < B, each written once.  A
// second kernel adds each body's slots in a fixed order (bitwise
// reproducible).
#include <algorithm>
#include <cstring>
#include <memory>
#include <numeric>

#include "pair_sym_core.h"

namespace ptrom {
namespace {

constexpr int64_t kMaxBatchItems = int64_t(1) << 24;
constexpr int kNA = Traits<OP_VEL>::NACC;

__global__ void reset_counter_kernel(int *__restrict__ counter) {
  if (threadIdx.x == 0) counter[0] = 0;
}

// K targets per lane: blocks of 256 K bodies.  K <= 2 keeps the kernel at 64
// VGPRs or fewer (eight waves per SIMD), as the single-system kernel reaches
// without the bound.
template <int K>
__global__ void __launch_bounds__(kBlock, K <= 2 ? 8 : 1)
    batched_sym_kernel(const int4 *__restrict__ items, int n_items, int *__restrict__ counter,
                       const int *__restrict__ off, const float *__restrict__ d2s,
                       const int64_t *__restrict__ slot_off, const float *__restrict__ xy,
                       const float *__restrict__ gam, float *__restrict__ P) {
  constexpr int NS = Traits<OP_VEL>::NSRC;
  constexpr int TB = kBlock * K;
  __shared__ float4 s_src[128][2];
  __shared__ float racc_lds[kBlock / 64][kNA][64];
  __shared__ float lds_diag[NS * kTile];
  __shared__ int item_s;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) item_s = atomicAdd(counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(item_s);
    __syncthreads();  // everyone has read item_s before it is overwritten
    if (it >= n_items) break;
    const int4 w = items[it];
    const int b = w.x, I = w.y, J = w.z;
    const int o = off[b];
    const int n = off[b + 1] - o;
    const float *xb = xy + 2 * (size_t)o;
    const float *gb = gam + o;
    float *Pb = P + slot_off[b];
    const float d2 = d2s[b];
    const int tgt0 = I * TB;
    if (I == J) {
      float res[K][kNA];
      pair_block<OP_VEL, K, STAGE_LDS>(n, xb, gb, nullptr, d2, tgt0, tgt0, min(n, tgt0 + TB), lds_diag, res);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int i = tgt0 + k * kBlock + tid;
        if (i < n)
#pragma unroll
          for (int a = 0; a < kNA; ++a) Pb[(size_t)(I * kNA + a) * n + i] = res[k][a];
      }
      continue;
    }
    sym_block_pair<OP_VEL, K>(n, xb, gb, nullptr, d2, tgt0, J * TB, s_src, racc_lds, Pb + (size_t)J * kNA * n,
                              Pb + (size_t)I * kNA * n);
  }
}

// Per body: its forward slots B .. nbk-1, then its reaction slots 0 .. B-1,
// Kahan-compensated, loads issued eight slots at a time.
__global__ void __launch_bounds__(256)
    batched_sym_reduce_kernel(int total, int tb, const int *__restrict__ inst, const int *__restrict__ off,
                              const int64_t *__restrict__ slot_off, const float *__restrict__ P,
                              float *__restrict__ out) {
  constexpr int kB = 8;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int b = inst[g];
  const int o = off[b];
  const int n = off[b + 1] - o;
  const int i = g - o;
  const int B = i / tb, nbk = (n + tb - 1) / tb;
  const float *Pb = P + slot_off[b];
  float s[kNA] = {}, c[kNA] = {};
  for (int q0 = 0; q0 < nbk; q0 += kB) {
    const int cnt = min(kB, nbk - q0);
    float t[kB][kNA];
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const int q = q0 + u;
      const int slot = q < nbk - B ? B + q : q - (nbk - B);
#pragma unroll
      for (int a = 0; a < kNA; ++a) t[u][a] = u < cnt ? Pb[(size_t)(slot * kNA + a) * n + i] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < kB; ++u)
      if (u < cnt) {
#pragma unroll
        for (int a = 0; a < kNA; ++a) kahan_add(s[a], c[a], t[u][a]);
      }
  }
#pragma unroll
  for (int a = 0; a < kNA; ++a) out[2 * (size_t)o + (size_t)a * n + i] = (s[a] - c[a]) * kInv2Pi;
}

}  // namespace

// Device-side description of one instance set.
struct BatchPlan {
  std::vector<int64_t> offsets;
  std::vector<float> delta;
  int k = 2, blocks_per_cu = 8;  // targets per lane (blocks of 256 k bodies), workgroups per CU
  int nb = 0, total = 0, n_items = 0;
  size_t slot_floats = 0;  // per-block slots of all instances, sum of nbk_b * 2 * N_b
  void *buf = nullptr;     // items | off | d2 | slot_off | inst | counter
  int4 *items = nullptr;
  int *off = nullptr, *inst = nullptr, *counter = nullptr;
  int64_t *slot_off = nullptr;
  float *d2 = nullptr;
  ~BatchPlan() {
    if (buf) hipFree(buf);
  }
};

}  // namespace ptrom

using namespace ptrom;

static int get_plan(ptrom_ctx *ctx, int nb, const int64_t *offsets, const float *delta,
                    std::shared_ptr<BatchPlan> &out) {
  if (nb < 1 || !offsets || !delta) return ctx->fail(PTROM_EINVAL, "nb >= 1 and host offsets/delta required");
  if (offsets[0] != 0) return ctx->fail(PTROM_EINVAL, "offsets[0] must be 0");
  for (int b = 0; b < nb; ++b) {
    if (offsets[b + 1] <= offsets[b]) return ctx->fail(PTROM_EINVAL, "every instance needs >= 1 body");
    if (!(delta[b] >= 0.0f) || !std::isfinite(delta[b])) return ctx->fail(PTROM_EINVAL, "delta must be >= 0");
  }
  if (offsets[nb] > kMaxN) return ctx->fail(PTROM_EINVAL, "total bodies must be <= 2^30");
  const PairCfg cfg = ctx->tune.get_batched(batched_size(nb, offsets));
  const int kb = cfg.k, bpc = cfg.waves_per_simd;
  const int64_t tbk = int64_t(kBlock) * kb;
  const auto &cur = ctx->batch_plan;
  if (cur && cur->nb == nb && cur->k == kb && cur->blocks_per_cu == bpc &&
      std::equal(offsets, offsets + nb + 1, cur->offsets.begin()) && std::equal(delta, delta + nb, cur->delta.begin())) {
    out = cur;
    return PTROM_OK;
  }
  auto p = std::make_shared<BatchPlan>();
  p->offsets.assign(offsets, offsets + nb + 1);
  p->delta.assign(delta, delta + nb);
  p->k = kb;
  p->blocks_per_cu = bpc;
  p->nb = nb;
  p->total = int(offsets[nb]);
  struct It {
    int4 v;
    int64_t cost;
  };
  std::vector<It> items;
  std::vector<int> off32(nb + 1), inst(p->total);
  std::vector<int64_t> slot_off(nb);
  std::vector<float> d2(nb);
  int64_t n_items = 0;
  uint64_t slot_bytes = 0;
  for (int b = 0; b < nb; ++b) {
    const int64_t n = offsets[b + 1] - offsets[b];
    const int64_t nbk = (n + tbk - 1) / tbk;
    n_items += nbk * (nbk + 1) / 2;
    slot_bytes += uint64_t(nbk) * kNA * uint64_t(n) * sizeof(float);
  }
  if (n_items > kMaxBatchItems)
    return ctx->fail(PTROM_EINVAL, "instances too large for one batched launch (block pairs > 2^24)");
  if (slot_bytes > ctx->tune.ws_cap_bytes)
    return ctx->fail(PTROM_EINVAL, "instances too large for one batched launch (block slots of " +
                                       std::to_string(slot_bytes) + " bytes beyond 1/32 of the device memory)");
  items.reserve(size_t(n_items));
  size_t slots = 0;
  for (int b = 0; b < nb; ++b) {
    const int n = int(offsets[b + 1] - offsets[b]);
    const int nbk = int((n + tbk - 1) / tbk);
    slot_off[b] = int64_t(slots);
    slots += size_t(nbk) * kNA * size_t(n);
    off32[b] = int(offsets[b]);
    d2[b] = delta[b] * delta[b];
    for (int i = int(offsets[b]); i < int(offsets[b + 1]); ++i) inst[i] = b;
    for (int I = 0; I < nbk; ++I)
      for (int J = I; J < nbk; ++J) {
        const int64_t nt = std::min<int64_t>(tbk, n - I * tbk);
        const int64_t ns = std::min<int64_t>(tbk, n - J * tbk);
        // one-sided diagonal tile: nt^2 ordered pairs; off-diagonal: nt ns
        // unordered pairs at about 1.5 times the one-sided cost per pair
        items.push_back({make_int4(b, I, J, 0), I == J ? nt * nt : 3 * nt * ns / 2});
      }
  }
  p->slot_floats = slots;
  off32[nb] = p->total;
  std::stable_sort(items.begin(), items.end(), [](const It &a, const It &b) { return a.cost > b.cost; });
  p->n_items = int(items.size());
  std::vector<int4> iv(items.size());
  for (size_t q = 0; q < items.size(); ++q) iv[q] = items[q].v;
  const size_t b_items = align256(iv.size() * sizeof(int4)), b_off = align256((nb + 1) * sizeof(int)),
               b_d2 = align256(nb * sizeof(float)), b_so = align256(nb * sizeof(int64_t)),
               b_inst = align256(size_t(p->total) * sizeof(int)), b_cnt = 256;
  hipError_t e = hipMalloc(&p->buf, b_items + b_off + b_d2 + b_so + b_inst + b_cnt);
  if (e != hipSuccess) {
    p->buf = nullptr;
    return ctx->fail(PTROM_ENOMEM, "batched plan allocation");
  }
  char *q = static_cast<char *>(p->buf);
  p->items = reinterpret_cast<int4 *>(q); q += b_items;
  p->off = reinterpret_cast<int *>(q); q += b_off;
  p->d2 = reinterpret_cast<float *>(q); q += b_d2;
  p->slot_off = reinterpret_cast<int64_t *>(q); q += b_so;
  p->inst = reinterpret_cast<int *>(q); q += b_inst;
  p->counter = reinterpret_cast<int *>(q);
  e = hipMemcpy(p->items, iv.data(), iv.size() * sizeof(int4), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->off, off32.data(), (nb + 1) * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d2, d2.data(), nb * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->slot_off, slot_off.data(), nb * sizeof(int64_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->inst, inst.data(), size_t(p->total) * sizeof(int), hipMemcpyHostToDevice);
  if (e != hipSuccess) return ctx->hip_fail(e, "batched plan upload");
  // graphs captured for an earlier instance set reference its buffers
  for (auto &g : ctx->graphs) hipGraphExecDestroy(g.exec);
  ctx->graphs.clear();
  ctx->batch_plan = p;
  out = p;
  return PTROM_OK;
}

// counter reset + persistent pass + slot reduction, all stream-ordered
static hipError_t launch_batched_velocity(ptrom_ctx *ctx, const BatchPlan &p, const float *xy,
                                          const float *gamma, float *f, float *slots, hipStream_t st) {
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, st, p.counter);
  const dim3 grid(ctx->num_cus * p.blocks_per_cu);
  if (p.k == 4)
    hipLaunchKernelGGL(batched_sym_kernel<4>, grid, dim3(kBlock), 0, st, p.items, p.n_items, p.counter, p.off, p.d2,
                       p.slot_off, xy, gamma, slots);
  else if (p.k == 1)
    hipLaunchKernelGGL(batched_sym_kernel<1>, grid, dim3(kBlock), 0, st, p.items, p.n_items, p.counter, p.off, p.d2,
                       p.slot_off, xy, gamma, slots);
  else
    hipLaunchKernelGGL(batched_sym_kernel<2>, grid, dim3(kBlock), 0, st, p.items, p.n_items, p.counter, p.off, p.d2,
                       p.slot_off, xy, gamma, slots);
  hipLaunchKernelGGL(batched_sym_reduce_kernel, dim3((p.total + 255) / 256), dim3(256), 0, st, p.total,
                     kBlock * p.k, p.inst, p.off, p.slot_off, slots, f);
  return hipGetLastError();
}

extern "C" int ptrom_velocity_batched(ptrom_ctx *ctx, int nb, const int64_t *offsets,
                                      const float *xy, const float *gamma, const float *delta,
                                      float *f, ptrom_stream stream) {
  if (!ctx) return PTROM_EINVAL;
  ctx->err.clear();
  if (!xy || !gamma || !f) return ctx->fail(PTROM_EINVAL, "NULL array");
  if (hipSetDevice(ctx->device) != hipSuccess) return ctx->fail(PTROM_EHIP, "hipSetDevice");
  std::shared_ptr<BatchPlan> p;
  if (int rc = get_plan(ctx, nb, offsets, delta, p)) return rc;
  const size_t partf = p->slot_floats;
  if (int rc = ctx->reserve(partf * sizeof(float))) return rc;
  hipError_t e = launch_batched_velocity(ctx, *p, xy, gamma, f, static_cast<float *>(ctx->ws),
                                         (hipStream_t)stream);
  if (e != hipSuccess) return ctx->hip_fail(e, "batched velocity");
  return PTROM_OK;
}

extern "C" int ptrom_rk4_batched(ptrom_ctx *ctx, int nb, const int64_t *offsets, float *xy,
                                 const float *gamma, const float *delta, float dt, int nsteps,
                                 int use_graph, ptrom_stream stream) {
  if (!ctx) return PTROM_EINVAL;
  ctx->err.clear();
  if (!xy || !gamma) return ctx->fail(PTROM_EINVAL, "NULL array");
  if (!(dt > 0.0f) || nsteps < 0) return ctx->fail(PTROM_EINVAL, "dt must be > 0 and nsteps >= 0");
  if (hipSetDevice(ctx->device) != hipSuccess) return ctx->fail(PTROM_EHIP, "hipSetDevice");
  std::shared_ptr<BatchPlan> p;
  if (int rc = get_plan(ctx, nb, offsets, delta, p)) return rc;
  if (nsteps == 0) return PTROM_OK;
  const int64_t m = 2 * int64_t(p->total);
  const size_t partf = p->slot_floats;
  if (int rc = ctx->reserve(5 * align256(m * sizeof(float)) + align256(partf * sizeof(float)) + 256)) return rc;
  Carver cv{static_cast<char *>(ctx->ws), ctx->ws_bytes};
  float *k[4];
  for (int q = 0; q < 4; ++q) k[q] = cv.take<float>(m);
  float *s = cv.take<float>(m);
  float *part = cv.take<float>(partf);
  if (!k[3] || !s || !part) return ctx->fail(PTROM_ENOMEM, "workspace carve");
  hipStream_t st = (hipStream_t)stream;

  auto record = [&](hipStream_t rs) -> int {
    const float *in = xy;
    for (int q = 0; q < 4; ++q) {
      hipError_t e = launch_batched_velocity(ctx, *p, in, gamma, k[q], part, rs);
      if (e != hipSuccess) return ctx->hip_fail(e, "batched velocity");
      if (q < 3) {
        e = launch_axpy(m, s, xy, (q < 2 ? 0.5f : 1.0f) * dt, k[q], rs);
        if (e != hipSuccess) return ctx->hip_fail(e, "batched stage");
        in = s;
      }
    }
    hipError_t e = launch_rk4_combine(m, xy, k[0], k[1], k[2], k[3], dt, rs);
    if (e != hipSuccess) return ctx->hip_fail(e, "batched combine");
    return PTROM_OK;
  };

  if (!use_graph) {
    for (int t = 0; t < nsteps; ++t)
      if (int rc = record(st)) return rc;
    return PTROM_OK;
  }
  char keybuf[256];
  std::snprintf(keybuf, sizeof keybuf, "rk4b:%p:%p:%p:%a:%p", (void *)p.get(), (void *)xy,
                (const void *)gamma, (double)dt, ctx->ws);
  hipGraphExec_t ex = nullptr;
  if (int rc = ctx->graph_for(keybuf, record, &ex)) return rc;
  for (int t = 0; t < nsteps; ++t) PTROM_CHECK_HIP(ctx, hipGraphLaunch(ex, st));
  return PTROM_OK;
}
