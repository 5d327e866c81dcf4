/*
 * CPU oracle for ray reordering and closest-hit tracing.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header or constant with the HIP library; both follow the paper (Meister,
 * Boksansky, Guthe, Bittner, "On Ray Reordering Techniques for Faster GPU
 * Ray Tracing", I3D 2020) and the readings listed beside each function.
 *
 * Build: gcc -O2 -ffp-contract=off (no -ffast-math): every float expression
 * below rounds once per operation in IEEE binary32, in the written order.
 *
 * Ray record: 8 floats {org.x, org.y, org.z, tmin, dir.x, dir.y, dir.z, tmax}.
 * Triangle record: 9 floats {v0, v1, v2}.
 * Hit record: {float t; int32 prim; float u, v}; a miss is {+inf, -1, 0, 0}.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ==================================================================== keys
 * Section 3 (ray space, Morton curve) and Figure "codes" (bit layouts),
 * Section 3.1.2 (origin-direction, Reis et al.), Section 3.1.5 (Two Point)
 * and Section 3.1.6 (fixed-length termination estimate, 0.25 of the largest
 * scene extent).
 *
 * A key is a sequence of slots from the most significant bit down.  Each
 * slot names one (vector, component).  A component quantised with b bits
 * owns b slots; its first slot carries its most significant bit.  Runs of a
 * vector cycle x, y, z (figure caption).
 *
 * Readings (the paper is silent on these):
 *  - quantiser: u = (x - lo) * inv, clamped to [0, 1] (NaN -> 0),
 *    q = trunc(u * 2^b) clamped to 2^b - 1;
 *  - direction components map [-1, 1] -> [0, 1] as (d + 1) * 0.5;
 *  - termination point t = o + min(L, tmax) * d with L = ratio * largest
 *    extent of the quantisation box, quantised in that same box;
 *  - 64-bit layouts extend the 32-bit ones: origin-direction with 44 origin
 *    slots then 20 direction slots, Two Point with the same 6-cycle for 64
 *    slots.  The other layouts of the figure exist at 32 bits only (the
 *    paper's method comparison uses 32-bit keys, Section 4.1).
 *
 * Layouts of the figure, as runs of slots (each run cycles x, y, z, or u, v
 * for the octahedral direction):
 *  Origin (3)        o32
 *  Costa (4)         d8 o24                   direction first (Section 3.1.3)
 *  Aila (5)          (o3 d3) x 5, o2, where every direction component's first
 *                    three slots are zeros (Section 3.1.4: three leading
 *                    zero bits per direction component)
 *  Aila Compact (6)  o12 d3 o3 d3 o3 d3 o3 d2
 *  Octahedron (7)    o15 q2 o3 q2 o3 q2 o3 q2, q = octahedral (u, v)
 *  Two Point Adaptive (8) and Two Point Real (9): the Two Point layout, with
 *                    the length taken from the length table or from the
 *                    traced hit (Section 3.1.6).
 */

enum { SRC_ZERO = -1, SRC_O = 0, SRC_D = 1, SRC_T = 2, SRC_Q = 3 };
enum { KIND_CODE20 = 100 };

typedef struct {
  int n;          /* slots */
  int8_t src[64]; /* SRC_* per slot, MSB first */
  int8_t comp[64];
} orc_layout;

/* Append `count` slots cycling over the components of `srcs` (each entry a
 * (vector, component) pair), starting at the first. */
static void lay_cycle(orc_layout* L, int count, int nsrc, const int8_t* vec, const int8_t* cmp) {
  for (int i = 0; i < count; ++i) {
    L->src[L->n] = vec[i % nsrc];
    L->comp[L->n] = cmp[i % nsrc];
    L->n++;
  }
}

/* A run of `count` slots of one vector, cycling its components from x. */
static void lay_run(orc_layout* L, int src, int count) {
  static const int8_t xyz[3] = {0, 1, 2};
  int8_t v[3] = {(int8_t)src, (int8_t)src, (int8_t)src};
  lay_cycle(L, count, src == SRC_Q ? 2 : 3, v, xyz);
}

/* kind 1 = origin-direction, 2 = Two Point (origin-termination), 3-9 and
 * KIND_CODE20 as listed above. */
static int make_layout(int kind, int key_bits, int origin_bits, orc_layout* L) {
  memset(L, 0, sizeof *L);
  static const int8_t xyz[3] = {0, 1, 2};
  if (kind == 1) {
    int ob = origin_bits ? origin_bits : (key_bits == 32 ? 22 : 44);
    if (ob < 0 || ob > key_bits) return -1;
    int8_t vo[3] = {SRC_O, SRC_O, SRC_O}, vd[3] = {SRC_D, SRC_D, SRC_D};
    lay_cycle(L, ob, 3, vo, xyz);
    lay_cycle(L, key_bits - ob, 3, vd, xyz);
    return 0;
  }
  if (kind == 2 || kind == 8 || kind == 9) {
    int8_t v6[6] = {SRC_O, SRC_O, SRC_O, SRC_T, SRC_T, SRC_T};
    int8_t c6[6] = {0, 1, 2, 0, 1, 2};
    lay_cycle(L, key_bits, 6, v6, c6);
    return 0;
  }
  if (kind >= 3 && kind <= 7 && key_bits != 32) return -1;
  switch (kind) {
    case 3:
      lay_run(L, SRC_O, 32);
      return 0;
    case 4:
      lay_run(L, SRC_D, 8);
      lay_run(L, SRC_O, 24);
      return 0;
    case 5: {
      int8_t v6[6] = {SRC_O, SRC_O, SRC_O, SRC_D, SRC_D, SRC_D};
      int8_t c6[6] = {0, 1, 2, 0, 1, 2};
      lay_cycle(L, 32, 6, v6, c6);
      int seen[3] = {0, 0, 0};
      for (int j = 0; j < L->n; ++j)
        if (L->src[j] == SRC_D && seen[(int)L->comp[j]]++ < 3) L->src[j] = SRC_ZERO;
      return 0;
    }
    case 6:
      lay_run(L, SRC_O, 12);
      for (int r = 0; r < 3; ++r) {
        lay_run(L, SRC_D, 3);
        lay_run(L, SRC_O, 3);
      }
      lay_run(L, SRC_D, 2);
      return 0;
    case 7:
      lay_run(L, SRC_O, 15);
      for (int r = 0; r < 3; ++r) {
        lay_run(L, SRC_Q, 2);
        lay_run(L, SRC_O, 3);
      }
      lay_run(L, SRC_Q, 2);
      return 0;
    case KIND_CODE20: /* the 20 leading slots of Aila Compact */
      lay_run(L, SRC_O, 12);
      lay_run(L, SRC_D, 3);
      lay_run(L, SRC_O, 3);
      lay_run(L, SRC_D, 2);
      return 0;
    default:
      return -1;
  }
}

static uint32_t quantize(float x, float lo, float inv, int b) {
  float u = (x - lo) * inv;
  if (!(u > 0.0f)) u = 0.0f;
  if (u > 1.0f) u = 1.0f;
  float s = ldexpf(u, b); /* exact: scaling by a power of two */
  uint32_t q = (uint32_t)s;
  uint32_t qmax = (uint32_t)((1ull << b) - 1ull);
  if (q > qmax) q = qmax;
  return q;
}

/* Octahedral parametrisation of a direction (Meyer et al. 2010; the layout
 * of Section 3.1.4): project onto |x| + |y| + |z| = 1; the lower half
 * (z < 0) folds over the diagonals.  sign(x) is +1 for x >= 0, else -1.
 * Binary32 in this order. */
void orc_octahedral(const float* d, float* u_out, float* v_out) {
  float s = (fabsf(d[0]) + fabsf(d[1])) + fabsf(d[2]);
  float px = d[0] / s;
  float py = d[1] / s;
  if (d[2] < 0.0f) {
    float sx = px >= 0.0f ? 1.0f : -1.0f;
    float sy = py >= 0.0f ? 1.0f : -1.0f;
    float fx = (1.0f - fabsf(py)) * sx;
    float fy = (1.0f - fabsf(px)) * sy;
    px = fx;
    py = fy;
  }
  *u_out = px;
  *v_out = py;
}

/* ------------------------------------------------------- length table
 * Two Point Adaptive (Section 3.1.6): a table of 2^20 cells indexed by the
 * 20-bit Aila Compact code of the ray (origin and direction), holding the
 * sum of the traced lengths of the rays that fell in the cell and their
 * count; the estimate is their mean.  Every cell starts with one dummy ray of
 * length ratio x the largest extent.
 * Readings: a cell is {uint64 sum; uint32 count; uint32 unused} (16 bytes);
 * lengths are summed in fixed point, in units of E / 2^24 (E the largest
 * extent), truncated: fixed(t) = trunc(t * (2^24 / E)) clamped to
 * [0, 2^40], so the sums do not depend on the order of accumulation; only
 * hits (prim >= 0) are accumulated; the estimate is
 * (float)((double)sum * E / ((double)count * 2^24)). */
typedef struct {
  uint64_t sum;
  uint32_t count;
  uint32_t unused;
} orc_cell;

#define ORC_CELLS (1u << 20)

static float box_extent(const float* box_lo, const float* box_hi) {
  float E = box_hi[0] - box_lo[0];
  for (int k = 1; k < 3; ++k) {
    float e = box_hi[k] - box_lo[k];
    if (e > E) E = e;
  }
  return E;
}

void orc_len_init(void* table, float ratio) {
  orc_cell* c = (orc_cell*)table;
  uint64_t s0 = (uint64_t)(ratio * 16777216.0f);
  for (uint32_t i = 0; i < ORC_CELLS; ++i) {
    c[i].sum = s0;
    c[i].count = 1;
    c[i].unused = 0;
  }
}

static uint64_t len_fixed(float t, float s24) {
  float x = t * s24;
  if (!(x > 0.0f)) return 0;
  if (x > 1099511627776.0f) return 1099511627776ull;
  return (uint64_t)x;
}

static float len_estimate(const orc_cell* c, float E) {
  double num = (double)c->sum * (double)E;
  double den = (double)c->count * 16777216.0;
  return (float)(num / den);
}

/* Slot layout as (src, comp) per bit, MSB first, for inspection by tests. */
int orc_key_layout(int32_t kind, int32_t key_bits, int32_t origin_bits, int8_t* src, int8_t* comp) {
  orc_layout L;
  if (make_layout(kind, key_bits, origin_bits, &L) != 0 || L.n != key_bits) return -1;
  memcpy(src, L.src, (size_t)L.n);
  memcpy(comp, L.comp, (size_t)L.n);
  return 0;
}

/* Quantised values q[vector][component] of one ray for layout L (bits per
 * (vector, component) in `bits`); `len` is the termination length used for
 * the T vector. */
static void ray_values(const float* r, const float* box_lo, const float* inv, int bits[4][3], float len,
                       uint32_t q[4][3]) {
  memset(q, 0, sizeof(uint32_t) * 12);
  for (int k = 0; k < 3; ++k) {
    q[SRC_O][k] = quantize(r[k], box_lo[k], inv[k], bits[SRC_O][k]);
    q[SRC_D][k] = quantize(r[4 + k], -1.0f, 0.5f, bits[SRC_D][k]);
    float step = len * r[4 + k];
    float tk = r[k] + step;
    q[SRC_T][k] = quantize(tk, box_lo[k], inv[k], bits[SRC_T][k]);
  }
  float u, v;
  orc_octahedral(r + 4, &u, &v);
  q[SRC_Q][0] = quantize(u, -1.0f, 0.5f, bits[SRC_Q][0]);
  q[SRC_Q][1] = quantize(v, -1.0f, 0.5f, bits[SRC_Q][1]);
}

static void layout_bits(const orc_layout* L, int bits[4][3]) {
  memset(bits, 0, sizeof(int) * 12);
  for (int j = 0; j < L->n; ++j)
    if (L->src[j] >= 0) bits[(int)L->src[j]][(int)L->comp[j]]++;
}

/* Assemble a key from the slot list, each component's bits MSB first. */
static uint64_t assemble(const orc_layout* L, int bits[4][3], uint32_t q[4][3]) {
  int used[4][3] = {{0}};
  uint64_t key = 0;
  for (int j = 0; j < L->n; ++j) {
    uint64_t bit = 0;
    int s = L->src[j], c = L->comp[j];
    if (s >= 0) {
      int b = bits[s][c];
      int which = b - 1 - used[s][c];
      used[s][c]++;
      bit = (q[s][c] >> which) & 1u;
    }
    key |= bit << (L->n - 1 - j);
  }
  return key;
}

/* 20-bit cell code of a ray (the Aila Compact prefix) for the length table. */
uint32_t orc_cell_code(const float* ray, const float* box_lo, const float* box_hi) {
  orc_layout L;
  make_layout(KIND_CODE20, 20, 0, &L);
  int bits[4][3];
  layout_bits(&L, bits);
  float inv[3];
  for (int k = 0; k < 3; ++k) {
    float e = box_hi[k] - box_lo[k];
    inv[k] = e > 0.0f ? 1.0f / e : 0.0f;
  }
  uint32_t q[4][3];
  ray_values(ray, box_lo, inv, bits, 0.0f, q);
  return (uint32_t)assemble(&L, bits, q);
}

/* Adds the traced lengths of n rays to the table (hits[i] belongs to
 * rays[i]). */
void orc_len_accumulate(void* table, const float* rays, const void* hits, int64_t n, const float* box_lo,
                        const float* box_hi) {
  orc_cell* c = (orc_cell*)table;
  float E = box_extent(box_lo, box_hi);
  float s24 = 16777216.0f / E;
  const unsigned char* h = (const unsigned char*)hits;
  for (int64_t i = 0; i < n; ++i) {
    float t;
    int32_t prim;
    memcpy(&t, h + 16 * i, 4);
    memcpy(&prim, h + 16 * i + 4, 4);
    if (prim < 0) continue;
    uint32_t cell = orc_cell_code(rays + 8 * i, box_lo, box_hi);
    c[cell].sum += len_fixed(t, s24);
    c[cell].count += 1;
  }
}

/* Length estimate the table gives a ray. */
float orc_len_lookup(const void* table, const float* ray, const float* box_lo, const float* box_hi) {
  const orc_cell* c = (const orc_cell*)table;
  return len_estimate(&c[orc_cell_code(ray, box_lo, box_hi)], box_extent(box_lo, box_hi));
}

/* Keys for n rays.  keys_out holds n uint64 values (32-bit keys occupy the
 * low half).  aux: the length table (kind 8) or the hits of the rays, 16
 * bytes each (kind 9); unused otherwise.  Returns 0, or -1 on a bad
 * argument. */
int orc_keys(const float* rays, int64_t n, int32_t kind, int32_t key_bits, const float* box_lo,
             const float* box_hi, float ratio, int32_t origin_bits, const void* aux, uint64_t* keys_out) {
  if (key_bits != 32 && key_bits != 64) return -1;
  orc_layout L;
  if (make_layout(kind, key_bits, origin_bits, &L) != 0 || L.n != key_bits) return -1;
  if ((kind == 8 || kind == 9) && !aux) return -1;
  int bits[4][3];
  layout_bits(&L, bits);

  float ext[3], inv[3];
  for (int k = 0; k < 3; ++k) {
    ext[k] = box_hi[k] - box_lo[k];
    inv[k] = ext[k] > 0.0f ? 1.0f / ext[k] : 0.0f;
  }
  float E = ext[0];
  if (ext[1] > E) E = ext[1];
  if (ext[2] > E) E = ext[2];
  float Lfix = ratio * E;

  for (int64_t i = 0; i < n; ++i) {
    const float* r = rays + 8 * i;
    float tmax = r[7];
    float len = (tmax < Lfix) ? tmax : Lfix;
    if (kind == 8) {
      float est = orc_len_lookup(aux, r, box_lo, box_hi);
      len = (tmax < est) ? tmax : est;
    } else if (kind == 9) {
      const unsigned char* h = (const unsigned char*)aux + 16 * i;
      float t;
      int32_t prim;
      memcpy(&t, h, 4);
      memcpy(&prim, h + 4, 4);
      if (prim >= 0) len = t;
    }
    uint32_t q[4][3];
    ray_values(r, box_lo, inv, bits, len, q);
    keys_out[i] = assemble(&L, bits, q);
  }
  return 0;
}

/* =========================================================== triangle test
 * Closest-hit trace (Section 4.1 uses nearest-hit tracing for secondary
 * rays).  The paper never writes an intersection formula; the reading is
 * the Moller-Trumbore test (Moller and Trumbore, "Fast, Minimum Storage
 * Ray/Triangle Intersection", JGT 1997), two-sided, in binary32 with this
 * operation order.  Returns 1 with (t, u, v) when the ray meets the
 * triangle; the caller applies the ray interval tmin < t < tmax. */
int orc_mt(const float* o, const float* d, const float* tri, float* t_out, float* u_out, float* v_out) {
  const float* v0 = tri;
  const float* v1 = tri + 3;
  const float* v2 = tri + 6;
  float e1[3], e2[3], s[3], p[3], q[3];
  for (int k = 0; k < 3; ++k) {
    e1[k] = v1[k] - v0[k];
    e2[k] = v2[k] - v0[k];
    s[k] = o[k] - v0[k];
  }
  p[0] = d[1] * e2[2] - d[2] * e2[1];
  p[1] = d[2] * e2[0] - d[0] * e2[2];
  p[2] = d[0] * e2[1] - d[1] * e2[0];
  float det = (e1[0] * p[0] + e1[1] * p[1]) + e1[2] * p[2];
  if (det == 0.0f) return 0;
  float inv = 1.0f / det;
  float u = ((s[0] * p[0] + s[1] * p[1]) + s[2] * p[2]) * inv;
  if (!(u >= 0.0f && u <= 1.0f)) return 0;
  q[0] = s[1] * e1[2] - s[2] * e1[1];
  q[1] = s[2] * e1[0] - s[0] * e1[2];
  q[2] = s[0] * e1[1] - s[1] * e1[0];
  float v = ((d[0] * q[0] + d[1] * q[1]) + d[2] * q[2]) * inv;
  if (!(v >= 0.0f && u + v <= 1.0f)) return 0;
  float t = ((e2[0] * q[0] + e2[1] * q[1]) + e2[2] * q[2]) * inv;
  *t_out = t;
  *u_out = u;
  *v_out = v;
  return 1;
}

typedef struct {
  float t;
  int32_t prim;
  float u, v;
} orc_hit;

/* The closest hit is the lexicographic minimum of (t, primitive id) over
 * every triangle whose test passes with tmin < t < tmax: equal t goes to the
 * lower id, so the result does not depend on traversal order. */
static void consider(const float* ray, const float* tris, int32_t j, orc_hit* best) {
  float t, u, v;
  if (!orc_mt(ray, ray + 4, tris + 9 * (int64_t)j, &t, &u, &v)) return;
  if (!(t > ray[3] && t < ray[7])) return;
  if (t < best->t || (t == best->t && j < best->prim)) {
    best->t = t;
    best->prim = j;
    best->u = u;
    best->v = v;
  }
}

static void miss(orc_hit* h) {
  h->t = INFINITY;
  h->prim = -1;
  h->u = 0.0f;
  h->v = 0.0f;
}

/* ------------------------------------------------------------ threading */

typedef void (*orc_range_fn)(void* ctx, int64_t lo, int64_t hi);
typedef struct {
  orc_range_fn fn;
  void* ctx;
  int64_t lo, hi;
  int ok;
} orc_job;

static void* orc_thread(void* p) {
  orc_job* j = (orc_job*)p;
  j->fn(j->ctx, j->lo, j->hi);
  return NULL;
}

static void orc_parallel(int64_t n, int nthreads, orc_range_fn fn, void* ctx) {
  if (nthreads > 256) nthreads = 256;
  if (nthreads <= 1 || n < 64) {
    fn(ctx, 0, n);
    return;
  }
  pthread_t th[256];
  orc_job job[256];
  int64_t chunk = (n + nthreads - 1) / nthreads;
  int m = 0;
  for (int t = 0; t < nthreads; ++t) {
    int64_t lo = t * chunk, hi = lo + chunk;
    if (lo >= n) break;
    if (hi > n) hi = n;
    job[m].fn = fn;
    job[m].ctx = ctx;
    job[m].lo = lo;
    job[m].hi = hi;
    job[m].ok = pthread_create(&th[m], NULL, orc_thread, &job[m]) == 0;
    if (!job[m].ok) fn(ctx, lo, hi);
    ++m;
  }
  for (int t = 0; t < m; ++t)
    if (job[t].ok) pthread_join(th[t], NULL);
}

/* ============================================================ brute force */

typedef struct {
  const float* tris;
  int64_t ntris;
  const float* rays;
  orc_hit* hits;
} brute_ctx;

static void brute_range(void* p, int64_t lo, int64_t hi) {
  brute_ctx* c = (brute_ctx*)p;
  for (int64_t i = lo; i < hi; ++i) {
    orc_hit best;
    miss(&best);
    for (int64_t j = 0; j < c->ntris; ++j) consider(c->rays + 8 * i, c->tris, (int32_t)j, &best);
    c->hits[i] = best;
  }
}

/* Closest hit of every ray against every triangle. */
void orc_brute_force(const float* tris, int64_t ntris, const float* rays, int64_t n, void* hits, int32_t nthreads) {
  brute_ctx c = {tris, ntris, rays, (orc_hit*)hits};
  orc_parallel(n, nthreads, brute_range, &c);
}

/* ============================================================ median BVH
 * The paper's method is agnostic to the acceleration structure (Section 1).
 * Reading: a binary BVH split at the median primitive along the largest
 * extent of the centroid bounds (lowest axis index on a tie), primitives
 * ordered by (centroid coordinate, primitive id), leaves of at most 4
 * primitives.  Boxes are held in double precision and widened, and the box
 * test in double precision keeps a relative slack, so pruning never drops a
 * triangle that the brute-force definition above would pick. */

typedef struct {
  double lo[3], hi[3];
  int32_t left, right; /* children, -1 for a leaf */
  int32_t first, count;
} orc_node;

typedef struct {
  orc_node* nodes;
  int32_t nnodes;
  int32_t* prims;
  const float* tris; /* borrowed: the caller keeps the array alive */
  int64_t ntris;
  double* cent; /* 3 per triangle */
  int depth;
} orc_bvh;

typedef struct {
  double key;
  int32_t id;
} keyed;

static int keyed_cmp(const void* a, const void* b) {
  const keyed* x = (const keyed*)a;
  const keyed* y = (const keyed*)b;
  if (x->key < y->key) return -1;
  if (x->key > y->key) return 1;
  return (x->id > y->id) - (x->id < y->id);
}

static int32_t build_rec(orc_bvh* B, keyed* scratch, int32_t b, int32_t e, int depth) {
  int32_t me = B->nnodes++;
  orc_node* N = &B->nodes[me];
  if (depth > B->depth) B->depth = depth;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int32_t i = b; i < e; ++i) {
    int32_t p = B->prims[i];
    for (int v = 0; v < 3; ++v)
      for (int k = 0; k < 3; ++k) {
        double x = B->tris[9 * (int64_t)p + 3 * v + k];
        if (x < lo[k]) lo[k] = x;
        if (x > hi[k]) hi[k] = x;
      }
    for (int k = 0; k < 3; ++k) {
      double c = B->cent[3 * (int64_t)p + k];
      if (c < clo[k]) clo[k] = c;
      if (c > chi[k]) chi[k] = c;
    }
  }
  for (int k = 0; k < 3; ++k) {
    double pad = 1e-6 * (fabs(lo[k]) + fabs(hi[k]) + (hi[k] - lo[k])) + 1e-30;
    N->lo[k] = lo[k] - pad;
    N->hi[k] = hi[k] + pad;
  }
  N->first = b;
  N->count = e - b;
  N->left = N->right = -1;
  if (e - b <= 4) return me;
  int axis = 0;
  double best = chi[0] - clo[0];
  for (int k = 1; k < 3; ++k)
    if (chi[k] - clo[k] > best) {
      best = chi[k] - clo[k];
      axis = k;
    }
  for (int32_t i = b; i < e; ++i) {
    scratch[i].id = B->prims[i];
    scratch[i].key = B->cent[3 * (int64_t)B->prims[i] + axis];
  }
  qsort(scratch + b, (size_t)(e - b), sizeof(keyed), keyed_cmp);
  for (int32_t i = b; i < e; ++i) B->prims[i] = scratch[i].id;
  int32_t mid = b + (e - b) / 2;
  int32_t l = build_rec(B, scratch, b, mid, depth + 1);
  int32_t r = build_rec(B, scratch, mid, e, depth + 1);
  B->nodes[me].left = l;
  B->nodes[me].right = r;
  B->nodes[me].count = 0;
  return me;
}

void* orc_bvh_build(const float* tris, int64_t ntris) {
  if (ntris <= 0 || ntris > (1ll << 30)) return NULL;
  orc_bvh* B = (orc_bvh*)calloc(1, sizeof(orc_bvh));
  B->tris = tris;
  B->ntris = ntris;
  B->nodes = (orc_node*)malloc(sizeof(orc_node) * (size_t)(2 * ntris));
  B->prims = (int32_t*)malloc(sizeof(int32_t) * (size_t)ntris);
  B->cent = (double*)malloc(sizeof(double) * 3 * (size_t)ntris);
  keyed* scratch = (keyed*)malloc(sizeof(keyed) * (size_t)ntris);
  for (int64_t i = 0; i < ntris; ++i) {
    B->prims[i] = (int32_t)i;
    for (int k = 0; k < 3; ++k)
      B->cent[3 * i + k] =
          ((double)tris[9 * i + k] + (double)tris[9 * i + 3 + k] + (double)tris[9 * i + 6 + k]) / 3.0;
  }
  build_rec(B, scratch, 0, (int32_t)ntris, 0);
  free(scratch);
  return B;
}

void orc_bvh_free(void* h) {
  orc_bvh* B = (orc_bvh*)h;
  if (!B) return;
  free(B->nodes);
  free(B->prims);
  free(B->cent);
  free(B);
}

int32_t orc_bvh_depth(void* h) { return ((orc_bvh*)h)->depth; }
int32_t orc_bvh_nodes(void* h) { return ((orc_bvh*)h)->nnodes; }

/* Does the ray's interval [tmin, tbest] (with slack) meet the node box?
 * Double precision; an axis with zero direction keeps the whole line when
 * the origin lies inside the slab. */
static int box_meets(const orc_node* N, const float* r, double tbest) {
  double tn = (double)r[3];
  tn -= 1e-5 * fabs(tn);
  double tf = tbest;
  if (tf > (double)r[7]) tf = (double)r[7];
  tf += 1e-5 * fabs(tf);
  for (int k = 0; k < 3; ++k) {
    double o = r[k], d = r[4 + k];
    if (d == 0.0) {
      if (o < N->lo[k] || o > N->hi[k]) return 0;
      continue;
    }
    double t0 = (N->lo[k] - o) / d, t1 = (N->hi[k] - o) / d;
    if (t0 > t1) {
      double s = t0;
      t0 = t1;
      t1 = s;
    }
    if (t0 > tn) tn = t0;
    if (t1 < tf) tf = t1;
  }
  return tn <= tf;
}

static void visit(const orc_bvh* B, int32_t ni, const float* ray, orc_hit* best) {
  const orc_node* N = &B->nodes[ni];
  if (!box_meets(N, ray, (double)best->t)) return;
  if (N->left < 0) {
    for (int32_t i = N->first; i < N->first + N->count; ++i) consider(ray, B->tris, B->prims[i], best);
    return;
  }
  /* visiting the child whose centre is nearer along the ray first only
   * prunes sooner; the result is the same minimum either way */
  const orc_node* L = &B->nodes[N->left];
  const orc_node* R = &B->nodes[N->right];
  double dl = 0, dr = 0;
  for (int k = 0; k < 3; ++k) {
    dl += (0.5 * (L->lo[k] + L->hi[k]) - ray[k]) * ray[4 + k];
    dr += (0.5 * (R->lo[k] + R->hi[k]) - ray[k]) * ray[4 + k];
  }
  if (dl <= dr) {
    visit(B, N->left, ray, best);
    visit(B, N->right, ray, best);
  } else {
    visit(B, N->right, ray, best);
    visit(B, N->left, ray, best);
  }
}

typedef struct {
  const orc_bvh* B;
  const float* rays;
  const uint32_t* idx; /* optional indirection */
  orc_hit* hits;
} trace_ctx;

static void trace_range(void* p, int64_t lo, int64_t hi) {
  trace_ctx* c = (trace_ctx*)p;
  for (int64_t i = lo; i < hi; ++i) {
    int64_t r = c->idx ? (int64_t)c->idx[i] : i;
    orc_hit best;
    miss(&best);
    visit(c->B, 0, c->rays + 8 * r, &best);
    c->hits[i] = best;
  }
}

/* Closest hit of rays[i] (or rays[idx[i]] when idx is given) for i < n. */
void orc_bvh_trace(void* h, const float* rays, const uint32_t* idx, int64_t n, void* hits, int32_t nthreads) {
  trace_ctx c = {(const orc_bvh*)h, rays, idx, (orc_hit*)hits};
  orc_parallel(n, nthreads, trace_range, &c);
}

/* ============================================================ compaction
 * Ascending indices of the live slots; returns their count. */
int64_t orc_compact(const uint8_t* alive, int64_t n, uint32_t* idx_out) {
  int64_t m = 0;
  for (int64_t i = 0; i < n; ++i)
    if (alive[i]) idx_out[m++] = (uint32_t)i;
  return m;
}

/* ==================================================== coherence measure
 * M^64_CPS of Section 4.3: for every group of n consecutive rays (n = 64;
 * the last group may be shorter), a capsule fitted to the group -- its axis
 * through the centroid of the origins and the centroid of the termination
 * points, its two hemispheres and the cone between them with radii equal to
 * the mean distance of the origins, respectively of the termination points,
 * from that axis -- and the capsule's surface area
 *   2 pi r_o^2 + 2 pi r_t^2 + pi (r_o + r_t) sqrt(h^2 + (r_o - r_t)^2),
 * h the distance between the centroids.  The measure of a ray set is the
 * mean over its groups.  Readings: a hit terminates at o + t d; a miss at
 * o + min(tmax, E) d, E the largest extent of the box (where it leaves the
 * scene); with coincident centroids the axis degenerates to a point and the
 * distances are taken to that point.  Double precision throughout. */
static double cps_group(const float* rays, const unsigned char* hits, int64_t first, int64_t cnt, float E) {
  double co[3] = {0, 0, 0}, ct[3] = {0, 0, 0};
  double P[64][3], T[64][3];
  for (int64_t j = 0; j < cnt; ++j) {
    const float* r = rays + 8 * (first + j);
    float t;
    int32_t prim;
    memcpy(&t, hits + 16 * (first + j), 4);
    memcpy(&prim, hits + 16 * (first + j) + 4, 4);
    double len = prim >= 0 ? (double)t : (double)(r[7] < E ? r[7] : E);
    for (int k = 0; k < 3; ++k) {
      P[j][k] = (double)r[k];
      T[j][k] = (double)r[k] + len * (double)r[4 + k];
      co[k] += P[j][k];
      ct[k] += T[j][k];
    }
  }
  double axis[3], h2 = 0;
  for (int k = 0; k < 3; ++k) {
    co[k] /= (double)cnt;
    ct[k] /= (double)cnt;
    axis[k] = ct[k] - co[k];
    h2 += axis[k] * axis[k];
  }
  double h = sqrt(h2);
  double ro = 0, rt = 0;
  for (int64_t j = 0; j < cnt; ++j) {
    double dp[3], dt[3], sp = 0, st = 0;
    for (int k = 0; k < 3; ++k) {
      dp[k] = P[j][k] - co[k];
      dt[k] = T[j][k] - co[k];
    }
    if (h > 0) {
      double ap = 0, at = 0;
      for (int k = 0; k < 3; ++k) {
        ap += dp[k] * axis[k] / h;
        at += dt[k] * axis[k] / h;
      }
      for (int k = 0; k < 3; ++k) {
        double x = dp[k] - ap * axis[k] / h, y = dt[k] - at * axis[k] / h;
        sp += x * x;
        st += y * y;
      }
    } else {
      for (int k = 0; k < 3; ++k) {
        sp += dp[k] * dp[k];
        st += dt[k] * dt[k];
      }
    }
    ro += sqrt(sp);
    rt += sqrt(st);
  }
  ro /= (double)cnt;
  rt /= (double)cnt;
  const double pi = 3.14159265358979323846;
  return 2 * pi * ro * ro + 2 * pi * rt * rt + pi * (ro + rt) * sqrt(h2 + (ro - rt) * (ro - rt));
}

/* Per-group measures (ceil(n / 64) of them) and their mean. */
void orc_cps(const float* rays, const void* hits, int64_t n, const float* box_lo, const float* box_hi,
             double* per_group, double* mean) {
  float E = box_extent(box_lo, box_hi);
  int64_t G = (n + 63) / 64;
  double s = 0;
  for (int64_t g = 0; g < G; ++g) {
    int64_t cnt = n - 64 * g < 64 ? n - 64 * g : 64;
    per_group[g] = cps_group(rays, (const unsigned char*)hits, 64 * g, cnt, E);
    s += per_group[g];
  }
  *mean = G ? s / (double)G : 0.0;
}
