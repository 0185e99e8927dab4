// Library-internal declarations shared by the HIP translation units of libptrom.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "ptrom.h"

namespace ptrom {

constexpr int kBlock = 256;   // threads per workgroup of the pair kernels (4 wave64)
constexpr int kTile = 256;    // sources staged per LDS tile
constexpr int64_t kMaxN = int64_t(1) << 30;

enum PairOp { OP_VEL = 0, OP_BJAC = 1, OP_JVP = 2, OP_VJP = 3, OP_PSI = 4, OP_VBJ = 5, OP_COUNT = 6 };


// Source staging of the pair kernels.
//  LDS:    the workgroup stages a tile of sources in LDS; every lane reads it
//          back with broadcast reads.
//  SCALAR: the wave reads sources straight from memory at wave-uniform
//          addresses, which the compiler turns into scalar-cache loads whose
//          values feed the vector ALUs as SGPR operands.
enum Staging { STAGE_LDS = 0, STAGE_SCALAR = 1 };

struct PairCfg {
  int staging = STAGE_SCALAR;
  int k = 2;               // targets per lane
  int waves_per_simd = 8;  // occupancy target used to choose the source split
  int sym = 0;             // 1: evaluate each unordered pair once (pair_sym.hip)
  int max_splits = 0;      // one-sided form: at most this many source chunks (0 = no limit)
};

// One tuned entry per operation and size class (log2 of N, clamped).
// The each-pair-once form keeps one partial-sum slot per body and block
// (2 nb NA N floats, growing as N^2); where that would pass ws_cap_bytes
// the one-sided form (workspace O(N)) is used instead.
struct Tuning {
  std::map<std::pair<int, int>, PairCfg> table;
  uint64_t ws_cap_bytes = uint64_t(8) << 30;  // set per device: its memory / kWsCapDivisor
  PairCfg get(int op, int64_t n) const;
  PairCfg get_table(int op, int64_t n) const;  // the table's entry, without the cap
  // batched velocity launch (k = targets per lane, waves_per_simd = workgroups
  // per CU) for instance sets of pair-weighted mean size nbar
  PairCfg get_batched(int64_t nbar) const;
};

// tuning-table key of the batched velocity launch ("batched_velocity")
constexpr int OP_BATCH = OP_COUNT;
// pair-weighted mean instance size sum N_b^2 / sum N_b (at least 1)
int64_t batched_size(int nb, const int64_t *offsets);

constexpr uint64_t kWsCapDivisor = 32;

// One-sided launch used where the each-pair-once workspace would be too large.
PairCfg large_n_cfg();

int size_class(int64_t n);

// Launch one pair-sum operation (all N targets x all N sources).
// out/out2 layouts as in the public calls.  ws must hold pair_ws_floats(...).
hipError_t launch_pair(int op, const PairCfg &cfg, int num_cus, int64_t n, const float *xy,
                       const float *gamma, const float *aux, float delta, float *out, float *out2,
                       float *ws, size_t ws_floats, hipStream_t stream);
size_t pair_ws_floats(int op, const PairCfg &cfg, int num_cus, int64_t n);
int pair_splits(int op, const PairCfg &cfg, int num_cus, int64_t n);

// Each-unordered-pair-once variant (velocity, JVP, VJP only).
size_t pair_sym_ws_floats(int op, int k, int64_t n);
hipError_t launch_pair_sym(int op, int k, int waves_per_simd, int num_cus, int64_t n, const float *xy,
                           const float *gamma, const float *aux, float delta, float *out, float *out2,
                           float *ws, size_t ws_floats, hipStream_t stream);

// velocity at nt arbitrary points p [2][nt] from all n bodies (no exclusion)
int points_splits(int num_cus, int64_t nt, int64_t n);
size_t points_ws_floats(int num_cus, int64_t nt, int64_t n);
hipError_t launch_velocity_points(int64_t nt, const float *p, int64_t n, const float *xy, const float *gamma,
                                  float delta, float *out, float *ws, size_t ws_floats, int num_cus,
                                  hipStream_t stream);

hipError_t launch_velocity_f64(int64_t n, const double *xy, const double *gamma, double delta,
                               double *f, hipStream_t stream);

// elementwise helpers (stream-ordered)
hipError_t launch_axpy(int64_t m, float *out, const float *x, float a, const float *y, hipStream_t s);
hipError_t launch_rk4_combine(int64_t m, float *x, const float *k1, const float *k2,
                              const float *k3, const float *k4, float h, hipStream_t s);
hipError_t launch_axpy_f64(int64_t m, double *out, const double *x, double a, const double *y,
                           hipStream_t s);
hipError_t launch_rk4_combine_f64(int64_t m, double *x, const double *k1, const double *k2,
                                  const double *k3, const double *k4, double h, hipStream_t s);

struct BatchPlan;

// Looks up, once per device, the device address of the allocation-free
// velocity call's scratch array (noalloc.hip); device must be current.
hipError_t noalloc_init(int device);

}  // namespace ptrom

struct GraphCacheEntry {
  std::string key;
  hipGraphExec_t exec = nullptr;
};

struct ptrom_ctx {
  int device = 0;
  int num_cus = 256;
  std::string err;
  void *ws = nullptr;
  size_t ws_bytes = 0;
  ptrom::Tuning tune;
  hipStream_t capture_stream = nullptr;
  std::vector<GraphCacheEntry> graphs;
  std::shared_ptr<ptrom::BatchPlan> batch_plan;
  double *pinned = nullptr;  // pinned host scratch for small device-to-host reads
  size_t pinned_count = 0;

  // at least count pinned doubles (kept until the context is destroyed)
  double *pinned_doubles(size_t count) {
    if (count <= pinned_count) return pinned;
    if (pinned) (void)hipHostFree(pinned);
    pinned = nullptr;
    pinned_count = 0;
    void *p = nullptr;
    if (hipHostMalloc(&p, count * sizeof(double), hipHostMallocDefault) != hipSuccess) return nullptr;
    pinned = static_cast<double *>(p);
    pinned_count = count;
    return pinned;
  }

  hipGraphExec_t find_graph(const std::string &key) const {
    for (auto &g : graphs)
      if (g.key == key) return g.exec;
    return nullptr;
  }
  void keep_graph(const std::string &key, hipGraphExec_t ex) {
    if (graphs.size() >= 16) {
      (void)hipGraphExecDestroy(graphs.front().exec);
      graphs.erase(graphs.begin());
    }
    graphs.push_back({key, ex});
  }
  // Capture `record(stream)` once into an executable graph cached under key.
  template <class F>
  int graph_for(const std::string &key, F &&record, hipGraphExec_t *out) {
    *out = find_graph(key);
    if (*out) return PTROM_OK;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    int rc = record(capture_stream);
    hipError_t e2 = hipStreamEndCapture(capture_stream, &g);
    if (rc) {
      if (g) hipGraphDestroy(g);
      return rc;
    }
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    hipGraphExec_t ex = nullptr;
    hipError_t e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e3 != hipSuccess) return hip_fail(e3, "hipGraphInstantiate");
    keep_graph(key, ex);
    *out = ex;
    return PTROM_OK;
  }

  int fail(int code, const std::string &msg) {
    err = msg;
    return code;
  }
  int hip_fail(hipError_t e, const char *what) {
    err = std::string(what) + ": " + hipGetErrorString(e);
    return PTROM_EHIP;
  }
  // Make sure the workspace holds `bytes`; returns PTROM_OK or an error code.
  int reserve(size_t bytes);
};

#define PTROM_CHECK_HIP(ctx, expr)                         \
  do {                                                     \
    hipError_t _e = (expr);                                \
    if (_e != hipSuccess) return (ctx)->hip_fail(_e, #expr); \
  } while (0)

// carve 256-byte aligned sub-buffers out of a workspace
struct Carver {
  char *p;
  size_t left;
  template <class T>
  T *take(size_t count) {
    size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    if (bytes > left) return nullptr;
    T *r = reinterpret_cast<T *>(p);
    p += bytes;
    left -= bytes;
    return r;
  }
};

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
