// Offline PTROM building blocks (training stages 2-3):
//  * host C++ quadtree over the weighted POD space W_phi = Phi Sigma_hat, the
//    per-node weighted means (Algorithm "ClusterPOD", WeightedMean), the
//    per-target neighbour-search traversal (FindClusters / Traverse with
//    Algorithm "checkPrune") and UniqueSearch into a CSR interaction list;
//  * FP64 GPU kernels for the POD by the method of snapshots: the Gram matrix
//    X X^T of a snapshot block and the combination Y = T^T X used to form and
//    re-orthogonalise the basis (CholeskyQR).
//
// Cluster conventions (the readings of the passages the paper leaves open):
// root cell = tight bounding box of the points; a cell splits at its midpoint
// while it holds more than one body and its level is below max_level;
// membership is half-open [lo, mid) / [mid, hi]; width = longer side;
// weighted means use |Gamma| (plain mean when all weights vanish) and the
// surrogate strength is the sum of Gamma; a source cell is pruned when it
// does not overlap the target leaf grown by pc times its width on every side
// (strict inequalities) and does not hold the target; a cell whose weighted
// mean initial position coincides with the target's (within 1e-9 of the
// target's distance from the origin, plus 1e-9) is never pruned either; an
// unpruned leaf is expanded into its bodies without the target; a pruned
// cell holding one body is that body.  Unique surrogates are ordered bodies first (by index)
// then cells (by level, row, column); each list is sorted by surrogate id.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

using namespace ptrom;

namespace {

struct QNode {
  double lo[2], hi[2];
  int level, ix, iy;
  int first, count;  // range in the member permutation
  int child[4];
  int nchild;
};

struct QTree {
  std::vector<QNode> nodes;
  std::vector<int> perm;     // members of node k are perm[first .. first+count)
  std::vector<int> leaf_of;  // body -> leaf node
  const double *P = nullptr;
  int max_level = 6;

  void build(int64_t n, const double *pts, int levels) {
    P = pts;
    max_level = levels;
    perm.resize(n);
    for (int64_t i = 0; i < n; ++i) perm[i] = int(i);
    leaf_of.assign(n, -1);
    double lo[2] = {pts[0], pts[1]}, hi[2] = {pts[0], pts[1]};
    for (int64_t i = 1; i < n; ++i)
      for (int d = 0; d < 2; ++d) {
        lo[d] = std::min(lo[d], pts[2 * i + d]);
        hi[d] = std::max(hi[d], pts[2 * i + d]);
      }
    nodes.reserve(4 * n / 3 + 16);
    make(lo, hi, 0, 0, 0, 0, int(n));
  }

  int make(const double lo[2], const double hi[2], int level, int ix, int iy, int first, int count) {
    const int id = int(nodes.size());
    QNode q;
    q.lo[0] = lo[0]; q.lo[1] = lo[1]; q.hi[0] = hi[0]; q.hi[1] = hi[1];
    q.level = level; q.ix = ix; q.iy = iy; q.first = first; q.count = count; q.nchild = 0;
    nodes.push_back(q);
    if (count > 1 && level < max_level) {
      const double mid[2] = {0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1])};
      // stable partition of the member range into the four quadrants
      std::vector<int> buckets[4];
      for (int t = first; t < first + count; ++t) {
        const int j = perm[t];
        const int qx = P[2 * j] >= mid[0] ? 1 : 0, qy = P[2 * j + 1] >= mid[1] ? 1 : 0;
        buckets[qx + 2 * qy].push_back(j);
      }
      int pos = first;
      int starts[4];
      for (int b = 0; b < 4; ++b) {
        starts[b] = pos;
        for (int j : buckets[b]) perm[pos++] = j;
      }
      for (int b = 0; b < 4; ++b) {
        if (buckets[b].empty()) continue;
        const int qx = b & 1, qy = b >> 1;
        const double clo[2] = {qx ? mid[0] : lo[0], qy ? mid[1] : lo[1]};
        const double chi[2] = {qx ? hi[0] : mid[0], qy ? hi[1] : mid[1]};
        const int c = make(clo, chi, level + 1, 2 * ix + qx, 2 * iy + qy, starts[b], int(buckets[b].size()));
        nodes[id].child[nodes[id].nchild++] = c;
      }
    } else {
      for (int t = first; t < first + count; ++t) leaf_of[perm[t]] = id;
    }
    return id;
  }
};

constexpr int64_t kNodeTag = int64_t(1) << 60;

inline int64_t node_key(const QNode &q) {
  return kNodeTag | (int64_t(q.level) << 40) | (int64_t(q.iy) << 20) | int64_t(q.ix);
}

struct PruneRule {
  int criterion;          // 0 neighbour search, 1 Barnes-Hut
  double theta;
  double hlo[2], hhi[2];  // neighbourhood of the target leaf
  double si[2];           // target point
  double xi[2], tol;      // target's initial physical position, coincidence radius
  const std::vector<double> *mean;  // per node weighted mean point [2]
  const std::vector<double> *phys;  // per node weighted mean initial position [2]
};

// A surrogate whose position at x^0 is the target's own (to rounding) would
// make the pair singular at delta = 0; such a cell is opened instead.
constexpr double kCoincide = 1e-9;

void traverse(const QTree &T, int node, int target, const PruneRule &pr, const QNode &leaf,
              std::vector<int64_t> &out) {
  const QNode &q = T.nodes[node];
  bool ov;
  if (pr.criterion == 0) {
    ov = pr.hhi[0] > q.lo[0] && pr.hlo[0] < q.hi[0] && pr.hhi[1] > q.lo[1] && pr.hlo[1] < q.hi[1];
  } else {
    const double dx = (*pr.mean)[2 * node] - pr.si[0], dy = (*pr.mean)[2 * node + 1] - pr.si[1];
    const double dist = std::sqrt(dx * dx + dy * dy);
    const double w = std::max(q.hi[0] - q.lo[0], q.hi[1] - q.lo[1]);
    ov = !(dist > 0.0 && w / dist <= pr.theta);
  }
  const int sh = leaf.level - q.level;
  if (sh >= 0 && (leaf.ix >> sh) == q.ix && (leaf.iy >> sh) == q.iy) ov = true;  // holds the target
  if (!ov && q.count > 1) {
    const double dx = (*pr.phys)[2 * node] - pr.xi[0], dy = (*pr.phys)[2 * node + 1] - pr.xi[1];
    if (std::sqrt(dx * dx + dy * dy) <= pr.tol) ov = true;
  }
  if (!ov) {
    out.push_back(q.count == 1 ? int64_t(T.perm[q.first]) : node_key(q));
    return;
  }
  if (q.nchild == 0) {
    for (int t = q.first; t < q.first + q.count; ++t)
      if (T.perm[t] != target) out.push_back(T.perm[t]);
    return;
  }
  for (int c = 0; c < q.nchild; ++c) traverse(T, q.child[c], target, pr, leaf, out);
}

}  // namespace

struct ptrom_clusters {
  int64_t nc = 0, nnz = 0;
  int M = 0;
  std::vector<double> xqt0, phit, gt;
  std::vector<int64_t> off, ids, keys;
  std::vector<int64_t> mem_off, mem_ids;  // bodies of each unique surrogate (CSR)
};

extern "C" int ptrom_cluster_build(int64_t n, const double *wpts, const double *xy0, const double *phi,
                                   int M, const double *gamma, int max_level, int criterion, double pc,
                                   double theta, int64_t nt, const int64_t *targets, ptrom_clusters **out) {
  if (!out || n < 1 || n > kMaxN || !wpts || !xy0 || !phi || !gamma || M < 1 || max_level < 0 ||
      max_level > 16 || !(pc >= 0.0) || !(theta >= 0.0) || (criterion != 0 && criterion != 1) || nt < 1 ||
      !targets)
    return PTROM_EINVAL;
  for (int64_t t = 0; t < nt; ++t)
    if (targets[t] < 0 || targets[t] >= n) return PTROM_EINVAL;
  QTree T;
  T.build(n, wpts, max_level);
  // per-node |Gamma|-weighted means: the point in W_phi (Barnes-Hut
  // surrogate position) and the initial physical position
  std::vector<double> mean(2 * T.nodes.size(), 0.0), phys(2 * T.nodes.size(), 0.0);
  for (size_t k = 0; k < T.nodes.size(); ++k) {
    const QNode &q = T.nodes[k];
    double ws = 0.0, mx = 0.0, my = 0.0, px = 0.0, py = 0.0;
    for (int t = q.first; t < q.first + q.count; ++t) ws += std::fabs(gamma[T.perm[t]]);
    for (int t = q.first; t < q.first + q.count; ++t) {
      const int j = T.perm[t];
      const double wj = ws == 0.0 ? 1.0 / q.count : std::fabs(gamma[j]) / ws;
      mx += wj * wpts[2 * j];
      my += wj * wpts[2 * j + 1];
      px += wj * xy0[j];
      py += wj * xy0[n + j];
    }
    mean[2 * k] = mx;
    mean[2 * k + 1] = my;
    phys[2 * k] = px;
    phys[2 * k + 1] = py;
  }
  // per-target lists of surrogate keys
  std::vector<std::vector<int64_t>> lists(nt);
  for (int64_t t = 0; t < nt; ++t) {
    const int i = int(targets[t]);
    const QNode &leaf = T.nodes[T.leaf_of[i]];
    const double w = std::max(leaf.hi[0] - leaf.lo[0], leaf.hi[1] - leaf.lo[1]);
    PruneRule pr;
    pr.criterion = criterion;
    pr.theta = theta;
    pr.hlo[0] = leaf.lo[0] - pc * w; pr.hlo[1] = leaf.lo[1] - pc * w;
    pr.hhi[0] = leaf.hi[0] + pc * w; pr.hhi[1] = leaf.hi[1] + pc * w;
    pr.si[0] = wpts[2 * i]; pr.si[1] = wpts[2 * i + 1];
    pr.xi[0] = xy0[i]; pr.xi[1] = xy0[n + i];
    pr.tol = kCoincide * (1.0 + std::sqrt(xy0[i] * xy0[i] + xy0[n + i] * xy0[n + i]));
    pr.mean = &mean;
    pr.phys = &phys;
    traverse(T, 0, i, pr, leaf, lists[t]);
  }
  // UniqueSearch
  std::vector<int64_t> keys;
  for (auto &L : lists) keys.insert(keys.end(), L.begin(), L.end());
  std::sort(keys.begin(), keys.end());
  keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
  auto *r = new ptrom_clusters();
  r->M = M;
  r->nc = int64_t(keys.size());
  r->keys = keys;
  r->xqt0.assign(2 * r->nc, 0.0);
  r->mem_off.assign(1, 0);
  r->phit.assign(2 * r->nc * M, 0.0);
  r->gt.assign(r->nc, 0.0);
  // node lookup by key
  std::vector<std::pair<int64_t, int>> nk;
  nk.reserve(T.nodes.size());
  for (size_t k = 0; k < T.nodes.size(); ++k) nk.push_back({node_key(T.nodes[k]), int(k)});
  std::sort(nk.begin(), nk.end());
  for (int64_t c = 0; c < r->nc; ++c) {
    const int64_t key = keys[c];
    if (key < kNodeTag) {
      const int64_t j = key;
      r->mem_ids.push_back(j);
      r->mem_off.push_back(int64_t(r->mem_ids.size()));
      r->xqt0[2 * c] = xy0[j];
      r->xqt0[2 * c + 1] = xy0[n + j];
      r->gt[c] = gamma[j];
      for (int m = 0; m < M; ++m) {
        r->phit[(2 * c) * M + m] = phi[j * M + m];
        r->phit[(2 * c + 1) * M + m] = phi[(n + j) * M + m];
      }
      continue;
    }
    auto it = std::lower_bound(nk.begin(), nk.end(), std::make_pair(key, -1));
    const QNode &q = T.nodes[it->second];
    const size_t m0 = r->mem_ids.size();
    for (int t = q.first; t < q.first + q.count; ++t) r->mem_ids.push_back(T.perm[t]);
    std::sort(r->mem_ids.begin() + m0, r->mem_ids.end());  // the subtree's ranges are grouped by quadrant
    r->mem_off.push_back(int64_t(r->mem_ids.size()));
    double wsum = 0.0, gsum = 0.0;
    for (int t = q.first; t < q.first + q.count; ++t) {
      wsum += std::fabs(gamma[T.perm[t]]);
      gsum += gamma[T.perm[t]];
    }
    const bool plain = (wsum == 0.0);
    const double norm = plain ? double(q.count) : wsum;
    double sx = 0.0, sy = 0.0;
    std::vector<double> px(M, 0.0), py(M, 0.0);
    for (int t = q.first; t < q.first + q.count; ++t) {
      const int64_t j = T.perm[t];
      const double wj = (plain ? 1.0 : std::fabs(gamma[j])) / norm;
      sx += wj * xy0[j];
      sy += wj * xy0[n + j];
      for (int m = 0; m < M; ++m) {
        px[m] += wj * phi[j * M + m];
        py[m] += wj * phi[(n + j) * M + m];
      }
    }
    r->xqt0[2 * c] = sx;
    r->xqt0[2 * c + 1] = sy;
    r->gt[c] = gsum;
    for (int m = 0; m < M; ++m) {
      r->phit[(2 * c) * M + m] = px[m];
      r->phit[(2 * c + 1) * M + m] = py[m];
    }
  }
  // CSR lists of surrogate ids, each sorted
  r->off.assign(nt + 1, 0);
  for (int64_t t = 0; t < nt; ++t) {
    std::vector<int64_t> ids;
    ids.reserve(lists[t].size());
    for (int64_t key : lists[t]) ids.push_back(std::lower_bound(keys.begin(), keys.end(), key) - keys.begin());
    std::sort(ids.begin(), ids.end());
    r->ids.insert(r->ids.end(), ids.begin(), ids.end());
    r->off[t + 1] = int64_t(r->ids.size());
  }
  r->nnz = int64_t(r->ids.size());
  *out = r;
  return PTROM_OK;
}

extern "C" int ptrom_cluster_sizes(const ptrom_clusters *c, int64_t *nc, int64_t *nnz) {
  if (!c || !nc || !nnz) return PTROM_EINVAL;
  *nc = c->nc;
  *nnz = c->nnz;
  return PTROM_OK;
}

extern "C" int ptrom_cluster_fetch(const ptrom_clusters *c, double *xqt0, double *phit, double *gt,
                                   int64_t *off, int64_t *ids, int64_t *keys) {
  if (!c) return PTROM_EINVAL;
  if (xqt0) std::memcpy(xqt0, c->xqt0.data(), c->xqt0.size() * sizeof(double));
  if (phit) std::memcpy(phit, c->phit.data(), c->phit.size() * sizeof(double));
  if (gt) std::memcpy(gt, c->gt.data(), c->gt.size() * sizeof(double));
  if (off) std::memcpy(off, c->off.data(), c->off.size() * sizeof(int64_t));
  if (ids) std::memcpy(ids, c->ids.data(), c->ids.size() * sizeof(int64_t));
  if (keys) std::memcpy(keys, c->keys.data(), c->keys.size() * sizeof(int64_t));
  return PTROM_OK;
}

extern "C" void ptrom_cluster_destroy(ptrom_clusters *c) { delete c; }

// ------------------------------------------------------------------ FP64 POD kernels

namespace {

constexpr int kGT = 16;   // Gram tile edge
constexpr int kGQ = 64;   // rows staged per step

// G = X X^T for X [k][nd] (row-major, one snapshot per row).  One workgroup per
// 16x16 tile of G; rows of X staged through LDS 64 columns at a time.
__global__ void __launch_bounds__(256)
    gram_f64_kernel(int64_t nd, int k, const double *__restrict__ X, double *__restrict__ G) {
  __shared__ double a[kGT][kGQ + 1], b[kGT][kGQ + 1];
  const int ta = threadIdx.x / kGT, tb = threadIdx.x % kGT;
  const int i0 = blockIdx.y * kGT, j0 = blockIdx.x * kGT;
  if (j0 > i0 + kGT - 1) return;  // upper triangle is mirrored
  double acc = 0.0;
  for (int64_t q0 = 0; q0 < nd; q0 += kGQ) {
    for (int t = threadIdx.x; t < kGT * kGQ; t += 256) {
      const int r = t / kGQ, c = t % kGQ;
      const int64_t q = q0 + c;
      a[r][c] = (i0 + r < k && q < nd) ? X[(size_t)(i0 + r) * nd + q] : 0.0;
      b[r][c] = (j0 + r < k && q < nd) ? X[(size_t)(j0 + r) * nd + q] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int c = 0; c < kGQ; ++c) acc += a[ta][c] * b[tb][c];
    __syncthreads();
  }
  const int i = i0 + ta, j = j0 + tb;
  if (i < k && j < k && j <= i) {
    G[(size_t)i * k + j] = acc;
    G[(size_t)j * k + i] = acc;
  }
}

// Y[m][q] = sum_a T[a][m] X[a][q]  (X [k][nd], T [k][M], Y [M][nd])
__global__ void __launch_bounds__(256)
    combine_f64_kernel(int64_t nd, int k, const double *__restrict__ X, int M,
                       const double *__restrict__ T, double *__restrict__ Y) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int m = blockIdx.y;
  if (q >= nd) return;
  double s = 0.0;
  for (int a = 0; a < k; ++a) s += T[(size_t)a * M + m] * X[(size_t)a * nd + q];
  Y[(size_t)m * nd + q] = s;
}

}  // namespace

extern "C" int ptrom_gram_f64(ptrom_ctx *ctx, int64_t nd, int k, const double *X, double *G,
                              ptrom_stream stream) {
  if (!ctx) return PTROM_EINVAL;
  ctx->err.clear();
  if (nd < 1 || k < 1 || k > 65535 || !X || !G) return ctx->fail(PTROM_EINVAL, "bad gram arguments");
  if (hipSetDevice(ctx->device) != hipSuccess) return ctx->fail(PTROM_EHIP, "hipSetDevice");
  const int tiles = (k + kGT - 1) / kGT;
  hipLaunchKernelGGL(gram_f64_kernel, dim3(tiles, tiles), dim3(256), 0, (hipStream_t)stream, nd, k, X, G);
  PTROM_CHECK_HIP(ctx, hipGetLastError());
  return PTROM_OK;
}

extern "C" int ptrom_combine_f64(ptrom_ctx *ctx, int64_t nd, int k, const double *X, int M,
                                 const double *T, double *Y, ptrom_stream stream) {
  if (!ctx) return PTROM_EINVAL;
  ctx->err.clear();
  if (nd < 1 || k < 1 || M < 1 || M > 65535 || !X || !T || !Y) return ctx->fail(PTROM_EINVAL, "bad combine arguments");
  if (hipSetDevice(ctx->device) != hipSuccess) return ctx->fail(PTROM_EHIP, "hipSetDevice");
  hipLaunchKernelGGL(combine_f64_kernel, dim3((unsigned)((nd + 255) / 256), M), dim3(256), 0,
                     (hipStream_t)stream, nd, k, X, M, T, Y);
  PTROM_CHECK_HIP(ctx, hipGetLastError());
  return PTROM_OK;
}

extern "C" int ptrom_cluster_members(const ptrom_clusters *c, int64_t *nmem, int64_t *mem_off, int64_t *mem_ids) {
  if (!c || !nmem) return PTROM_EINVAL;
  *nmem = int64_t(c->mem_ids.size());
  if (mem_off) std::memcpy(mem_off, c->mem_off.data(), c->mem_off.size() * sizeof(int64_t));
  if (mem_ids) std::memcpy(mem_ids, c->mem_ids.data(), c->mem_ids.size() * sizeof(int64_t));
  return PTROM_OK;
}
