// Scene construction: a binary BVH over the triangles, packed for the trace
// kernel and uploaded to the current device.
//
// The reordering method is agnostic to the acceleration structure
// (Section 1), so the builder is a free choice.  Two are provided:
//  * median split: split at the median centroid along the widest centroid
//    axis; balanced, depth ceil(log2(ceil(n/4))), fast to build;
//  * binned SAH: 256 bins per axis on centroids, surface-area cost, falling
//    back to the median split when a subtree could otherwise exceed the
//    trace kernel's stack depth.
// Leaves hold at most 3 triangles.  Nodes are emitted in depth-first order
// (a first child follows its parent) as a 4-wide tree, triangles in leaf
// order with their edges e1 = v1 - v0, e2 = v2 - v0 precomputed in binary32.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <future>
#include <memory>
#include <new>
#include <vector>

#include "common.hpp"

namespace rr {
namespace {

constexpr int kLeafMax = 3;  // measured best of 2..6 and SAH-terminated leaves of up to 7
constexpr int kBins = 256;

struct Box {
  float lo[3] = {INFINITY, INFINITY, INFINITY};
  float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  void grow(const float* p) {
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], p[k]);
      hi[k] = std::max(hi[k], p[k]);
    }
  }
  void grow(const Box& b) {
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], b.lo[k]);
      hi[k] = std::max(hi[k], b.hi[k]);
    }
  }
  double area() const {
    if (!(hi[0] >= lo[0])) return 0.0;
    const double x = hi[0] - lo[0], y = hi[1] - lo[1], z = hi[2] - lo[2];
    return 2.0 * (x * y + y * z + z * x);
  }
};

struct Prim {
  Box box;
  float c[3];
};

struct BNode {
  Box box;
  std::unique_ptr<BNode> kid[2];
  int32_t first = 0, count = 0;  // leaf range in the builder's index array
};

int median_depth(int64_t n) {
  int64_t leaves = (n + kLeafMax - 1) / kLeafMax;
  int d = 0;
  while ((int64_t(1) << d) < leaves) ++d;
  return d;
}

struct Builder {
  const std::vector<Prim>& prims;
  std::vector<int32_t>& order;
  int builder;
  int max_depth_seen = 0;

  Builder(const std::vector<Prim>& p, std::vector<int32_t>& o, int b) : prims(p), order(o), builder(b) {}

  // returns the split position in [b, e), or -1 for "use the median"
  int64_t sah_split(int64_t b, int64_t e, const Box& cb) {
    double best = INFINITY;
    int best_axis = -1, best_bin = -1;
    for (int axis = 0; axis < 3; ++axis) {
      const float ext = cb.hi[axis] - cb.lo[axis];
      if (!(ext > 0.0f)) continue;
      Box bb[kBins];
      int64_t cnt[kBins] = {0};
      const float scale = kBins / ext;
      for (int64_t i = b; i < e; ++i) {
        const Prim& p = prims[order[i]];
        int bin = (int)((p.c[axis] - cb.lo[axis]) * scale);
        bin = std::min(std::max(bin, 0), kBins - 1);
        cnt[bin]++;
        bb[bin].grow(p.box);
      }
      double right_area[kBins];
      int64_t right_cnt[kBins];
      Box acc;
      int64_t c = 0;
      for (int k = kBins - 1; k > 0; --k) {
        acc.grow(bb[k]);
        c += cnt[k];
        right_area[k] = acc.area();
        right_cnt[k] = c;
      }
      Box left;
      int64_t lc = 0;
      for (int k = 0; k < kBins - 1; ++k) {
        left.grow(bb[k]);
        lc += cnt[k];
        if (lc == 0 || right_cnt[k + 1] == 0) continue;
        const double cost = left.area() * (double)lc + right_area[k + 1] * (double)right_cnt[k + 1];
        if (cost < best) {
          best = cost;
          best_axis = axis;
          best_bin = k;
        }
      }
    }
    if (best_axis < 0) return -1;
    const float ext = cb.hi[best_axis] - cb.lo[best_axis];
    const float scale = kBins / ext;
    auto mid = std::partition(order.begin() + b, order.begin() + e, [&](int32_t id) {
      int bin = (int)((prims[id].c[best_axis] - cb.lo[best_axis]) * scale);
      bin = std::min(std::max(bin, 0), kBins - 1);
      return bin <= best_bin;
    });
    const int64_t m = mid - order.begin();
    if (m == b || m == e) return -1;
    return m;
  }

  int64_t median_split(int64_t b, int64_t e, const Box& cb) {
    int axis = 0;
    for (int k = 1; k < 3; ++k)
      if (cb.hi[k] - cb.lo[k] > cb.hi[axis] - cb.lo[axis]) axis = k;
    const int64_t m = b + (e - b) / 2;
    std::nth_element(order.begin() + b, order.begin() + m, order.begin() + e, [&](int32_t x, int32_t y) {
      const float cx = prims[x].c[axis], cy = prims[y].c[axis];
      return cx < cy || (cx == cy && x < y);
    });
    return m;
  }

  std::unique_ptr<BNode> build(int64_t b, int64_t e, int depth) {
    auto node = std::make_unique<BNode>();
    Box cb;
    for (int64_t i = b; i < e; ++i) {
      const Prim& p = prims[order[i]];
      node->box.grow(p.box);
      cb.grow(p.c);
    }
    const int64_t n = e - b;
    if (n <= kLeafMax) {
      node->first = (int32_t)b;
      node->count = (int32_t)n;
      return node;
    }
    int64_t m = -1;
    if (builder == 1 && depth + 1 + median_depth(n) + 2 < kMaxTreeDepth) m = sah_split(b, e, cb);
    if (m < 0) m = median_split(b, e, cb);
    if (depth < 4 && n > 65536) {
      auto fut = std::async(std::launch::async, [&, b, m, depth] { return build(b, m, depth + 1); });
      node->kid[1] = build(m, e, depth + 1);
      node->kid[0] = fut.get();
    } else {
      node->kid[0] = build(b, m, depth + 1);
      node->kid[1] = build(m, e, depth + 1);
    }
    return node;
  }
};

// Emits the 4-wide BVH: each binary inner node is widened by repeatedly
// replacing its largest-area inner child with that child's two children
// until it has four children or only leaves remain.
// 8-bit quantised child bounds (compressed 64-byte node): per axis an
// origin p (the node's lower bound) and a power-of-two step s with
// 255 * s >= extent; a child bound is stored as q, the plane at the exact
// real p + q * s.  q is rounded outward and then checked against that exact
// sum (see below), so the planes always contain the child's box.
void quantize_node(const Box* kids, int m, const int32_t* code, float4* out) {
  Box P;
  for (int j = 0; j < m; ++j) P.grow(kids[j]);
  float p[3], s[3];
  // The trace kernel places plane q at the exact real p + q * 2^e (it never
  // rounds that sum), so the checks below bound the exact sum: D = p + q * s
  // in double is within 2^-53 |D| of it, and a margin of 2^-52 |D| makes
  // each comparison hold for the exact value.
  auto below = [](double D, float x) { return D + std::fabs(D) * 0x1p-52 <= (double)x; };
  auto above = [](double D, float x) { return D - std::fabs(D) * 0x1p-52 >= (double)x; };
  for (int a = 0; a < 3; ++a) {
    p[a] = P.lo[a];
    const double ext = (double)P.hi[a] - (double)P.lo[a];
    int e = -100;
    if (ext > 0) {
      e = (int)std::ceil(std::log2(ext / 255.0));
      while (std::ldexp(255.0, e) < ext) ++e;
      while (e > -100 && std::ldexp(255.0, e - 1) >= ext) --e;
    }
    e = std::max(-100, e);
    while (!above((double)p[a] + std::ldexp(255.0, e), P.hi[a])) ++e;
    s[a] = std::ldexp(1.0f, e);  // e >= -100: a normal binary32 power of two
  }
  auto dec = [&](int a, uint32_t q) { return (double)p[a] + (double)q * (double)s[a]; };
  uint32_t lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int j = 0; j < m; ++j)
    for (int a = 0; a < 3; ++a) {
      double ql = std::floor(((double)kids[j].lo[a] - (double)p[a]) / (double)s[a]);
      double qh = std::ceil(((double)kids[j].hi[a] - (double)p[a]) / (double)s[a]);
      uint32_t l = (uint32_t)std::max(0.0, std::min(255.0, ql));
      uint32_t h = (uint32_t)std::max(0.0, std::min(255.0, qh));
      while (l > 0 && !below(dec(a, l), kids[j].lo[a])) --l;
      while (h < 255 && !above(dec(a, h), kids[j].hi[a])) ++h;
      lo[a] |= l << (8 * j);
      hi[a] |= h << (8 * j);
    }
  auto f = [](uint32_t v) {
    float x;
    std::memcpy(&x, &v, 4);
    return x;
  };
  auto fi = [](int32_t v) {
    float x;
    std::memcpy(&x, &v, 4);
    return x;
  };
  out[0] = make_float4(p[0], p[1], p[2], s[2]);
  out[1] = make_float4(f(lo[0]), f(hi[0]), f(lo[1]), f(hi[1]));
  out[2] = make_float4(f(lo[2]), f(hi[2]), s[0], s[1]);
  out[3] = make_float4(fi(code[0]), fi(code[1]), fi(code[2]), fi(code[3]));
}

struct Packer {
  const float* tris;
  const std::vector<int32_t>& order;
  std::vector<float4> nodes;
  std::vector<float4> gtris;
  int max_depth = 0;
  int stride = 8;  // float4 per node: 8 full-precision, 4 quantised

  int32_t leaf(const BNode* n) {
    const int32_t first = (int32_t)(gtris.size() / 3);
    for (int32_t k = 0; k < n->count; ++k) {
      const int32_t p = order[n->first + k];
      const float* v = tris + 9 * (int64_t)p;
      const float e1x = v[3] - v[0], e1y = v[4] - v[1], e1z = v[5] - v[2];
      const float e2x = v[6] - v[0], e2y = v[7] - v[1], e2z = v[8] - v[2];
      float pf;
      std::memcpy(&pf, &p, 4);
      gtris.push_back(make_float4(v[0], v[1], v[2], e1x));
      gtris.push_back(make_float4(e1y, e1z, e2x, e2y));
      gtris.push_back(make_float4(e2z, pf, 0.0f, 0.0f));
    }
    return ~((first << 3) | n->count);
  }

  int32_t pack(const BNode* n, int depth) {
    max_depth = std::max(max_depth, depth);
    if (!n->kid[0]) return leaf(n);
    const BNode* kids[4] = {n->kid[0].get(), n->kid[1].get(), nullptr, nullptr};
    int m = 2;
    while (m < 4) {
      int best = -1;
      double best_area = -1.0;
      for (int j = 0; j < m; ++j)
        if (kids[j]->kid[0] && kids[j]->box.area() > best_area) {
          best = j;
          best_area = kids[j]->box.area();
        }
      if (best < 0) break;
      const BNode* x = kids[best];
      kids[best] = x->kid[0].get();
      kids[m++] = x->kid[1].get();
    }
    const int32_t me = (int32_t)(nodes.size() / stride);
    nodes.resize(nodes.size() + stride);
    int32_t code[4] = {kEmptyChild, kEmptyChild, kEmptyChild, kEmptyChild};
    for (int j = 0; j < m; ++j) code[j] = pack(kids[j], depth + 1);
    if (stride == 4) {
      Box kb[4];
      for (int j = 0; j < m; ++j) kb[j] = kids[j]->box;
      quantize_node(kb, m, code, nodes.data() + 4 * (size_t)me);
      return me;
    }
    float lo[3][4], hi[3][4];
    for (int j = 0; j < 4; ++j)
      for (int k = 0; k < 3; ++k) {
        lo[k][j] = j < m ? kids[j]->box.lo[k] : 0.0f;
        hi[k][j] = j < m ? kids[j]->box.hi[k] : 0.0f;
      }
    float4* N = nodes.data() + 8 * (size_t)me;
    for (int k = 0; k < 3; ++k) {
      N[2 * k] = make_float4(lo[k][0], lo[k][1], lo[k][2], lo[k][3]);
      N[2 * k + 1] = make_float4(hi[k][0], hi[k][1], hi[k][2], hi[k][3]);
    }
    float c[4];
    std::memcpy(c, code, sizeof c);
    N[6] = make_float4(c[0], c[1], c[2], c[3]);
    N[7] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    return me;
  }
};

}  // namespace

rr_status build_scene(const float* tris, int64_t n, int builder, DeviceScene* out) {
  const bool quantised = (builder & RR_BUILD_FULL_NODES) == 0;
  builder &= 1;
  std::vector<Prim> prims((size_t)n);
  Box scene;
  for (int64_t i = 0; i < n; ++i) {
    const float* v = tris + 9 * i;
    Prim& p = prims[(size_t)i];
    for (int j = 0; j < 3; ++j) p.box.grow(v + 3 * j);
    for (int k = 0; k < 3; ++k) p.c[k] = (v[k] + v[3 + k] + v[6 + k]) * (1.0f / 3.0f);
    scene.grow(p.box);
  }
  std::vector<int32_t> order((size_t)n);
  for (int64_t i = 0; i < n; ++i) order[(size_t)i] = (int32_t)i;
  Builder B(prims, order, builder);
  std::unique_ptr<BNode> root = B.build(0, n, 0);
  Packer P{tris, order, {}, {}, 0, quantised ? 4 : 8};
  P.nodes.reserve((size_t)(n / 4 + 8) * P.stride);
  P.gtris.reserve((size_t)n * 3);
  const int32_t root_code = P.pack(root.get(), 0);
  if (P.max_depth > kMaxTreeDepth) return RR_ERR_UNSUPPORTED;

  DeviceScene d;
  d.root = root_code;
  d.n_nodes = (int64_t)(P.nodes.size() / P.stride);
  d.quantised = quantised ? 1 : 0;
  d.n_tris = n;
  d.depth = P.max_depth;
  for (int k = 0; k < 3; ++k) {
    d.lo[k] = scene.lo[k];
    d.hi[k] = scene.hi[k];
  }
  if (hipGetDevice(&d.device) != hipSuccess) return RR_ERR_DEVICE;
  const size_t nb = std::max<size_t>(P.nodes.size(), 8) * sizeof(float4);  // at least one node of either kind
  const size_t tb = P.gtris.size() * sizeof(float4);
  if (hipMalloc(&d.nodes, nb) != hipSuccess) return RR_ERR_OUT_OF_MEMORY;
  if (hipMalloc(&d.tris, tb) != hipSuccess) {
    (void)hipFree(d.nodes);
    return RR_ERR_OUT_OF_MEMORY;
  }
  d.bytes = nb + tb;
  if (!P.nodes.empty() && hipMemcpy(d.nodes, P.nodes.data(), P.nodes.size() * sizeof(float4),
                                    hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d.nodes);
    (void)hipFree(d.tris);
    return RR_ERR_DEVICE;
  }
  if (hipMemcpy(d.tris, P.gtris.data(), tb, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d.nodes);
    (void)hipFree(d.tris);
    return RR_ERR_DEVICE;
  }
  *out = d;
  return RR_OK;
}

}  // namespace rr
