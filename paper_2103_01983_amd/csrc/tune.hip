// Launch-parameter autotuner for the pair kernels: times every candidate
// (source staging x targets per lane x occupancy target) on this device at a
// ladder of sizes and keeps the fastest per (operation, size class).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <vector>

#include "internal.h"

using namespace ptrom;

static const char *kOpNames[OP_COUNT] = {"velocity", "block_jacobian", "jvp", "vjp", "stream_function",
                                         "velocity_block_jacobian"};
static const char *kBatchName = "batched_velocity";

// Reads a tuning file into t; returns the number of entries loaded (-1 if the
// file cannot be opened).
static int read_tuning(const char *path, Tuning &t) {
  std::ifstream in(path);
  if (!in) return -1;
  std::string line;
  int loaded = 0;
  while (std::getline(in, line)) {
    if (line.empty() || line[0] == '#') continue;
    std::istringstream ss(line);
    std::string name;
    int cls, staging, k, waves, sym = 0;
    if (!(ss >> name >> cls >> staging >> k >> waves)) continue;
    std::string tok;
    if (ss >> tok && tok[0] != '#') sym = std::atoi(tok.c_str());
    int op = -1;
    for (int q = 0; q < OP_COUNT; ++q)
      if (name == kOpNames[q]) op = q;
    if (name == kBatchName) op = OP_BATCH;
    if (op < 0 || (k != 1 && k != 2 && k != 4) || (staging != STAGE_LDS && staging != STAGE_SCALAR) ||
        waves < 1 || waves > 64)
      continue;
    if (sym != 0 && sym != 1) continue;
    PairCfg c;
    c.staging = staging;
    c.k = k;
    c.waves_per_simd = waves;
    c.sym = sym;
    t.table[{op, cls}] = c;
    ++loaded;
  }
  return loaded;
}

extern "C" int ptrom_load_tuning(ptrom_ctx *ctx, const char *path) {
  if (!ctx || !path) return PTROM_EINVAL;
  const int loaded = read_tuning(path, ctx->tune);
  if (loaded < 0) return ctx->fail(PTROM_EINVAL, std::string("cannot open ") + path);
  return loaded ? PTROM_OK : ctx->fail(PTROM_EINVAL, "no tuning entries");
}

// Batched velocity launch: targets per lane (blocks of 256 K bodies) and
// workgroups per CU, timed on instance sets of equal sizes 2048, 8192 and
// 32768 (262144 bodies each) and on 24 instances log-spaced from 2048 to
// 32768 bodies, keyed by the class of the pair-weighted mean size.
static int tune_batched(ptrom_ctx *ctx, std::ostringstream &report) {
  std::vector<std::vector<int64_t>> sets;
  for (int64_t m : {int64_t(2048), int64_t(8192), int64_t(32768)}) sets.push_back(std::vector<int64_t>(262144 / m, m));
  {
    std::vector<int64_t> mix;
    for (int q = 0; q < 24; ++q) mix.push_back(int64_t(std::llround(2048.0 * std::pow(16.0, q / 23.0))));
    sets.push_back(mix);
  }
  int64_t total = 0;
  for (auto &v : sets) {
    int64_t t = 0;
    for (int64_t m : v) t += m;
    total = std::max(total, t);
  }
  std::vector<float> h(3 * total);
  float *d = nullptr, *f = nullptr;
  PTROM_CHECK_HIP(ctx, hipMalloc(&d, 3 * total * sizeof(float)));
  hipError_t e = hipMalloc(&f, 2 * total * sizeof(float));
  hipEvent_t a = nullptr, b = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  int rc = PTROM_OK;
  for (const auto &sizes : sets) {
    if (e != hipSuccess || rc) break;
    const int nb = int(sizes.size());
    std::vector<int64_t> off(nb + 1, 0);
    std::vector<float> delta(nb);
    for (int q = 0; q < nb; ++q) off[q + 1] = off[q] + sizes[q];
    const int64_t tot = off[nb];
    for (int q = 0; q < nb; ++q) {
      const int64_t m = sizes[q];
      delta[q] = 0.005f + 0.045f * float(q) / float(nb);
      for (int64_t i = 0; i < m; ++i) {
        // golden-angle spiral per instance (x block, y block, then Gamma)
        const double t = 2.399963229728653 * double(i) + 0.7 * q;
        const double rr = 0.25 * std::sqrt((i + 0.5) / double(m));
        h[2 * off[q] + i] = float(rr * std::cos(t));
        h[2 * off[q] + m + i] = float(rr * std::sin(t));
        h[2 * tot + off[q] + i] = float(1.0 / double(m));
      }
    }
    e = hipMemcpy(d, h.data(), 3 * tot * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) break;
    const int64_t nb_size = batched_size(nb, off.data());
    const int cls = size_class(nb_size);
    float best = 1e30f;
    PairCfg bestc;
    for (int k : {1, 2, 4})
      for (int bpc : {4, 8, 16}) {
        PairCfg c;
        c.staging = STAGE_LDS;
        c.k = k;
        c.waves_per_simd = bpc;
        c.sym = 1;
        ctx->tune.table[{OP_BATCH, cls}] = c;
        for (int rep = 0; rep < 2 && !rc; ++rep)
          rc = ptrom_velocity_batched(ctx, nb, off.data(), d, d + 2 * tot, delta.data(), f, nullptr);
        if (rc) break;
        const int reps = 3;
        float ms = 1e30f;
        for (int trial = 0; trial < 3 && !rc && e == hipSuccess; ++trial) {
          e = hipEventRecord(a, nullptr);
          for (int rep = 0; rep < reps && !rc && e == hipSuccess; ++rep)
            rc = ptrom_velocity_batched(ctx, nb, off.data(), d, d + 2 * tot, delta.data(), f, nullptr);
          if (e == hipSuccess) e = hipEventRecord(b, nullptr);
          if (e == hipSuccess) e = hipEventSynchronize(b);
          float t = 0.0f;
          if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
          if (e == hipSuccess) ms = std::min(ms, t / reps);
        }
        if (e != hipSuccess || rc) break;
        if (ms < best) {
          best = ms;
          bestc = c;
        }
      }
    if (e != hipSuccess || rc) break;
    ctx->tune.table[{OP_BATCH, cls}] = bestc;
    report << kBatchName << " " << cls << " " << bestc.staging << " " << bestc.k << " " << bestc.waves_per_simd
           << " " << bestc.sym << "   # " << best << " ms at " << nb << " instances, pair-weighted mean size "
           << nb_size << "\n";
  }
  if (a) hipEventDestroy(a);
  if (b) hipEventDestroy(b);
  hipFree(d);
  hipFree(f);
  ctx->batch_plan.reset();
  if (rc) return rc;
  if (e != hipSuccess) return ctx->hip_fail(e, "autotune (batched)");
  return PTROM_OK;
}

extern "C" int ptrom_autotune(ptrom_ctx *ctx, const char *cache_path) {
  if (!ctx) return PTROM_EINVAL;
  ctx->err.clear();
  if (hipSetDevice(ctx->device) != hipSuccess) return ctx->fail(PTROM_EHIP, "hipSetDevice");
  const int64_t sizes[] = {2048, 8192, 32768, 65536, 131072};
  const int64_t nmax = 131072;
  // synthetic Gaussian-like cloud: deterministic, no RNG state needed
  std::vector<float> h(5 * nmax);
  for (int64_t i = 0; i < nmax; ++i) {
    const double a = 2.399963229728653 * double(i);  // golden-angle spiral
    const double rr = 0.5 * std::sqrt((i + 0.5) / double(nmax));
    h[i] = float(rr * std::cos(a));
    h[nmax + i] = float(rr * std::sin(a));
    h[2 * nmax + i] = float(1.0 / nmax);
    h[3 * nmax + i] = float(std::sin(0.37 * i));
    h[4 * nmax + i] = float(std::cos(0.11 * i));
  }
  float *d = nullptr, *o = nullptr, *o2 = nullptr, *wsb = nullptr;
  PTROM_CHECK_HIP(ctx, hipMalloc(&d, 5 * nmax * sizeof(float)));
  hipError_t e = hipMalloc(&o, 4 * nmax * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&o2, 4 * nmax * sizeof(float));
  const size_t wsf = std::max(size_t(64) * 5 * nmax, pair_sym_ws_floats(OP_VBJ, 2, nmax));  // split / pair-block partials
  if (e == hipSuccess) e = hipMalloc(&wsb, wsf * sizeof(float));
  if (e == hipSuccess) e = hipMemcpy(d, h.data(), 5 * nmax * sizeof(float), hipMemcpyHostToDevice);
  hipEvent_t a = nullptr, b = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  std::ostringstream report;
  report << "# op size_class staging k waves_per_simd sym   (ms)\n";
  for (int op = 0; op < OP_COUNT && e == hipSuccess; ++op) {
    for (int64_t n : sizes) {
      // gather the packed copies for this n
      std::vector<float> hp(5 * n);
      for (int c = 0; c < 5; ++c)
        for (int64_t i = 0; i < n; ++i) hp[c * n + i] = h[c * nmax + (i * (nmax / n))];
      e = hipMemcpy(d, hp.data(), 5 * n * sizeof(float), hipMemcpyHostToDevice);
      if (e != hipSuccess) break;
      const float *xy = d, *gam = d + 2 * n, *aux = d + 3 * n;
      float best = 1e30f;
      PairCfg bestc;
      std::vector<PairCfg> cands;
      for (int staging : {STAGE_LDS, STAGE_SCALAR})
        for (int k : {1, 2, 4})
          for (int waves : {4, 8, 16}) {
            PairCfg c;
            c.staging = staging;
            c.k = k;
            c.waves_per_simd = waves;
            cands.push_back(c);
          }
      for (int k : {2, 4})
        for (int waves : {2, 4, 8}) {
          PairCfg c;
          c.staging = STAGE_LDS;
          c.k = k;
          c.waves_per_simd = waves;
          c.sym = 1;
          cands.push_back(c);
        }
      for (const PairCfg &c : cands) {
            if (pair_ws_floats(op, c, ctx->num_cus, n) > wsf) continue;
            for (int rep = 0; rep < 2 && e == hipSuccess; ++rep)
              e = launch_pair(op, c, ctx->num_cus, n, xy, gam, aux, 0.01f, o, o2, wsb, wsf, nullptr);
            // the best of three timed runs of back-to-back launches: the
            // candidates differ by a few percent, about the drift of one run
            const int reps = n <= 8192 ? 20 : 8;
            float ms = 1e30f;
            for (int trial = 0; trial < 3 && e == hipSuccess; ++trial) {
              e = hipEventRecord(a, nullptr);
              for (int rep = 0; rep < reps && e == hipSuccess; ++rep)
                e = launch_pair(op, c, ctx->num_cus, n, xy, gam, aux, 0.01f, o, o2, wsb, wsf, nullptr);
              if (e == hipSuccess) e = hipEventRecord(b, nullptr);
              if (e == hipSuccess) e = hipEventSynchronize(b);
              float t = 0.0f;
              if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
              if (e == hipSuccess) ms = std::min(ms, t / reps);
            }
            if (e != hipSuccess) break;
            if (ms < best) {
              best = ms;
              bestc = c;
            }
          }
      if (e != hipSuccess) break;
      const int cls = size_class(n);
      ctx->tune.table[{op, cls}] = bestc;
      report << kOpNames[op] << " " << cls << " " << bestc.staging << " " << bestc.k << " "
             << bestc.waves_per_simd << " " << bestc.sym << "   # " << best << " ms at n=" << n << "\n";
    }
  }
  if (a) hipEventDestroy(a);
  if (b) hipEventDestroy(b);
  hipFree(d);
  hipFree(o);
  hipFree(o2);
  hipFree(wsb);
  if (e != hipSuccess) return ctx->hip_fail(e, "autotune");
  if (int rc = tune_batched(ctx, report)) return rc;
  if (cache_path) {
    std::ofstream out(cache_path);
    if (!out) return ctx->fail(PTROM_EINVAL, std::string("cannot write ") + cache_path);
    out << report.str();
  }
  return PTROM_OK;
}

static void describe(const PairCfg &c, int op, int num_cus, int64_t n, int32_t *out) {
  const bool sym = c.sym != 0;
  out[0] = c.staging;
  out[1] = c.k;
  out[2] = c.waves_per_simd;
  out[3] = sym ? 1 : 0;
  out[4] = sym ? 0 : pair_splits(op, c, num_cus, n);
}

extern "C" int ptrom_pair_config(ptrom_ctx *ctx, int op, int64_t n, int32_t *out) {
  if (!ctx || !out || op < 0 || op > OP_BATCH || n < 1 || n > kMaxN) return PTROM_EINVAL;
  if (op == OP_BATCH) {
    const PairCfg c = ctx->tune.get_batched(n);
    out[0] = c.staging;
    out[1] = c.k;
    out[2] = c.waves_per_simd;
    out[3] = 1;
    out[4] = 0;
    return PTROM_OK;
  }
  describe(ctx->tune.get(op, n), op, ctx->num_cus, n, out);
  return PTROM_OK;
}

extern "C" int ptrom_pair_plan(const char *tuning_path, int num_cus, uint64_t device_bytes, int op, int64_t n,
                               int32_t *out, uint64_t *ws_bytes) {
  if (!out || op < 0 || op >= OP_COUNT || n < 1 || n > kMaxN || num_cus < 1 || device_bytes == 0)
    return PTROM_EINVAL;
  Tuning t;
  t.ws_cap_bytes = device_bytes / kWsCapDivisor;
  if (tuning_path && read_tuning(tuning_path, t) <= 0) return PTROM_EINVAL;
  const PairCfg c = t.get(op, n);
  describe(c, op, num_cus, n, out);
  if (ws_bytes) *ws_bytes = uint64_t(pair_ws_floats(op, c, num_cus, n)) * sizeof(float);
  return PTROM_OK;
}
