// Many independent parametric instances (own N_b, own core delta_b) in one
// persistent launch per velocity evaluation.  The host cuts every instance
// into work items (instance, block of 512 targets, chunk of 4096 sources),
// sorts them by pair count (largest first) and uploads the list once per
// instance set; every workgroup then pops items from a device counter until
// the list is exhausted, so large and small instances share the chip without
// a tail.  Items write compensated partial sums per source chunk; a second
// kernel adds each body's chunks in chunk order (bitwise reproducible).
#include <algorithm>
#include <cstring>
#include <memory>
#include <numeric>

#include "pair_core.h"

namespace ptrom {
namespace {

constexpr int kBatchK = 2;                      // targets per lane
constexpr int kBatchTargets = kBlock * kBatchK;  // targets per item
constexpr int kChunk = 16 * kTile;              // sources per item
constexpr int kBlocksPerCU = 8;

__global__ void reset_counter_kernel(int *__restrict__ counter) {
  if (threadIdx.x == 0) counter[0] = 0;
}

template <int STAGING>
__global__ void __launch_bounds__(kBlock)
    batched_velocity_kernel(const int4 *__restrict__ items, int n_items, int *__restrict__ counter,
                            const int *__restrict__ off, const float *__restrict__ d2s,
                            const float *__restrict__ xy, const float *__restrict__ gam, int total,
                            float *__restrict__ part) {
  __shared__ float lds[STAGING == STAGE_LDS ? 3 * kTile : 1];
  __shared__ int item_s;
  for (;;) {
    if (threadIdx.x == 0) item_s = atomicAdd(counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(item_s);
    __syncthreads();  // everyone has read item_s before it is overwritten
    if (it >= n_items) break;
    const int4 w = items[it];
    const int b = w.x;
    const int o = off[b];
    const int nb = off[b + 1] - o;
    const int tgt0 = w.y * kBatchTargets;
    const int sb = w.z * kChunk;
    const int se = min(nb, sb + kChunk);
    float res[kBatchK][2];
    pair_block<OP_VEL, kBatchK, STAGING>(nb, xy + 2 * (size_t)o, gam + o, nullptr, d2s[b], tgt0, sb,
                                         se, lds, res);
#pragma unroll
    for (int k = 0; k < kBatchK; ++k) {
      const int i = tgt0 + k * kBlock + threadIdx.x;
      if (i < nb) {
        part[(size_t)(w.z * 2) * total + o + i] = res[k][0];
        part[(size_t)(w.z * 2 + 1) * total + o + i] = res[k][1];
      }
    }
  }
}

__global__ void __launch_bounds__(256)
    batched_reduce_kernel(int total, const int *__restrict__ inst, const int *__restrict__ off,
                          const int *__restrict__ nsplit, const float *__restrict__ part,
                          float *__restrict__ out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int b = inst[g];
  const int o = off[b];
  const int nb = off[b + 1] - o;
  const int S = nsplit[b];
  for (int q = 0; q < 2; ++q) {
    float s = 0.0f, c = 0.0f;
    for (int p = 0; p < S; ++p) kahan_add(s, c, part[(size_t)(p * 2 + q) * total + g]);
    out[2 * (size_t)o + (size_t)q * nb + (g - o)] = (s - c) * kInv2Pi;
  }
}

}  // namespace

// Device-side description of one instance set.
struct BatchPlan {
  std::vector<int64_t> offsets;
  std::vector<float> delta;
  int nb = 0, total = 0, n_items = 0, max_split = 0, staging = STAGE_SCALAR;
  void *buf = nullptr;  // items | off | d2 | nsplit | inst | counter
  int4 *items = nullptr;
  int *off = nullptr, *nsplit = nullptr, *inst = nullptr, *counter = nullptr;
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
  const auto &cur = ctx->batch_plan;
  if (cur && cur->nb == nb && std::equal(offsets, offsets + nb + 1, cur->offsets.begin()) &&
      std::equal(delta, delta + nb, cur->delta.begin())) {
    out = cur;
    return PTROM_OK;
  }
  auto p = std::make_shared<BatchPlan>();
  p->offsets.assign(offsets, offsets + nb + 1);
  p->delta.assign(delta, delta + nb);
  p->nb = nb;
  p->total = int(offsets[nb]);
  p->staging = ctx->tune.get(OP_VEL, 8192).staging;
  struct It {
    int4 v;
    int64_t cost;
  };
  std::vector<It> items;
  std::vector<int> nsplit(nb), off32(nb + 1), inst(p->total);
  std::vector<float> d2(nb);
  for (int b = 0; b < nb; ++b) {
    const int n = int(offsets[b + 1] - offsets[b]);
    const int T = (n + kBatchTargets - 1) / kBatchTargets;
    const int S = (n + kChunk - 1) / kChunk;
    nsplit[b] = S;
    p->max_split = std::max(p->max_split, S);
    off32[b] = int(offsets[b]);
    d2[b] = delta[b] * delta[b];
    for (int i = int(offsets[b]); i < int(offsets[b + 1]); ++i) inst[i] = b;
    for (int t = 0; t < T; ++t)
      for (int s = 0; s < S; ++s) {
        const int64_t nt = std::min(kBatchTargets, n - t * kBatchTargets);
        const int64_t ns = std::min(kChunk, n - s * kChunk);
        items.push_back({make_int4(b, t, s, 0), nt * ns});
      }
  }
  off32[nb] = p->total;
  std::stable_sort(items.begin(), items.end(), [](const It &a, const It &b) { return a.cost > b.cost; });
  p->n_items = int(items.size());
  std::vector<int4> iv(items.size());
  for (size_t q = 0; q < items.size(); ++q) iv[q] = items[q].v;
  const size_t b_items = align256(iv.size() * sizeof(int4)), b_off = align256((nb + 1) * sizeof(int)),
               b_d2 = align256(nb * sizeof(float)), b_ns = align256(nb * sizeof(int)),
               b_inst = align256(size_t(p->total) * sizeof(int)), b_cnt = 256;
  hipError_t e = hipMalloc(&p->buf, b_items + b_off + b_d2 + b_ns + b_inst + b_cnt);
  if (e != hipSuccess) {
    p->buf = nullptr;
    return ctx->fail(PTROM_ENOMEM, "batched plan allocation");
  }
  char *q = static_cast<char *>(p->buf);
  p->items = reinterpret_cast<int4 *>(q); q += b_items;
  p->off = reinterpret_cast<int *>(q); q += b_off;
  p->d2 = reinterpret_cast<float *>(q); q += b_d2;
  p->nsplit = reinterpret_cast<int *>(q); q += b_ns;
  p->inst = reinterpret_cast<int *>(q); q += b_inst;
  p->counter = reinterpret_cast<int *>(q);
  e = hipMemcpy(p->items, iv.data(), iv.size() * sizeof(int4), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->off, off32.data(), (nb + 1) * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d2, d2.data(), nb * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->nsplit, nsplit.data(), nb * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->inst, inst.data(), size_t(p->total) * sizeof(int), hipMemcpyHostToDevice);
  if (e != hipSuccess) return ctx->hip_fail(e, "batched plan upload");
  // graphs captured for an earlier instance set reference its buffers
  for (auto &g : ctx->graphs) hipGraphExecDestroy(g.exec);
  ctx->graphs.clear();
  ctx->batch_plan = p;
  out = p;
  return PTROM_OK;
}

// counter reset + persistent pass + chunk reduction, all stream-ordered
static hipError_t launch_batched_velocity(ptrom_ctx *ctx, const BatchPlan &p, const float *xy,
                                          const float *gamma, float *f, float *part, hipStream_t st) {
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, st, p.counter);
  const dim3 grid(ctx->num_cus * kBlocksPerCU);
  if (p.staging == STAGE_LDS)
    hipLaunchKernelGGL(batched_velocity_kernel<STAGE_LDS>, grid, dim3(kBlock), 0, st, p.items, p.n_items,
                       p.counter, p.off, p.d2, xy, gamma, p.total, part);
  else
    hipLaunchKernelGGL(batched_velocity_kernel<STAGE_SCALAR>, grid, dim3(kBlock), 0, st, p.items,
                       p.n_items, p.counter, p.off, p.d2, xy, gamma, p.total, part);
  hipLaunchKernelGGL(batched_reduce_kernel, dim3((p.total + 255) / 256), dim3(256), 0, st, p.total,
                     p.inst, p.off, p.nsplit, part, f);
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
  const size_t partf = size_t(p->max_split) * 2 * p->total;
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
  const size_t partf = size_t(p->max_split) * 2 * p->total;
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
