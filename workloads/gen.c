/*
 * Seeded synthetic workloads: triangle scenes and ray wavefronts.
 *
 * This module feeds identical arrays to the CPU oracle and to the HIP path.
 * It holds none of the reordering method's arithmetic (no sort keys, no
 * sort, no BVH, no ray/triangle test).  To place secondary-ray origins on
 * surfaces it intersects rays with the procedural city analytically (a 2D
 * grid walk over axis-aligned boxes plus the ground plane, in double
 * precision); the thin clutter triangles are ignored for that purpose.
 *
 * Randomness: a counter-based generator, the SplitMix64 finaliser
 * (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
 * OOPSLA 2014) applied to (seed, stream, counter), so every value is a pure
 * function of its indices and the output does not depend on threading.
 *
 * Ray record: 8 floats {org.x, org.y, org.z, tmin, dir.x, dir.y, dir.z, tmax}.
 * Triangle record: 9 floats {v0.xyz, v1.xyz, v2.xyz}.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PI_D 3.14159265358979323846

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* 64 random bits for (seed, stream, counter). */
static inline uint64_t rng64(uint64_t seed, uint64_t stream, uint64_t ctr) {
  uint64_t a = mix64(seed * 0x9E3779B97F4A7C15ULL + 0x632BE59BD9B4E019ULL);
  uint64_t b = mix64(a ^ (stream * 0xD1B54A32D192ED03ULL));
  return mix64(b + ctr * 0x9E3779B97F4A7C15ULL);
}

/* Uniform double in [0, 1). */
static inline double rngu(uint64_t seed, uint64_t stream, uint64_t ctr) {
  return (double)(rng64(seed, stream, ctr) >> 11) * (1.0 / 9007199254740992.0);
}

uint64_t wl_rng64(uint64_t seed, uint64_t stream, uint64_t ctr) { return rng64(seed, stream, ctr); }
double wl_rngu(uint64_t seed, uint64_t stream, uint64_t ctr) { return rngu(seed, stream, ctr); }

/* ---------------------------------------------------------------- threads */

typedef void (*range_fn)(void* ctx, int64_t lo, int64_t hi);
typedef struct { range_fn fn; void* ctx; int64_t lo, hi; } range_job;

static void* range_thread(void* p) {
  range_job* j = (range_job*)p;
  j->fn(j->ctx, j->lo, j->hi);
  return NULL;
}

static void parallel_for(int64_t n, int nthreads, range_fn fn, void* ctx) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  if (n < 4096 || nthreads == 1) { fn(ctx, 0, n); return; }
  pthread_t th[256];
  range_job jobs[256];
  int64_t chunk = (n + nthreads - 1) / nthreads;
  int started = 0;
  for (int t = 0; t < nthreads; ++t) {
    int64_t lo = t * chunk, hi = lo + chunk;
    if (lo >= n) break;
    if (hi > n) hi = n;
    jobs[t].fn = fn; jobs[t].ctx = ctx; jobs[t].lo = lo; jobs[t].hi = hi;
    if (pthread_create(&th[t], NULL, range_thread, &jobs[t]) != 0) { fn(ctx, lo, hi); jobs[t].fn = NULL; }
    started = t + 1;
  }
  for (int t = 0; t < started; ++t)
    if (jobs[t].fn) pthread_join(th[t], NULL);
}

/* --------------------------------------------------------------- geometry */

static void unit_sphere(double u1, double u2, double out[3]) {
  double z = 1.0 - 2.0 * u1;
  double r = sqrt(fmax(0.0, 1.0 - z * z));
  double phi = 2.0 * PI_D * u2;
  out[0] = r * cos(phi); out[1] = r * sin(phi); out[2] = z;
}

/* Orthonormal tangent frame (a, b) for unit n. */
static void tangent_frame(const double n[3], double a[3], double b[3]) {
  double h[3] = {0, 0, 0};
  if (fabs(n[0]) < 0.9) h[0] = 1.0; else h[1] = 1.0;
  /* a = normalize(h x n) */
  a[0] = h[1] * n[2] - h[2] * n[1];
  a[1] = h[2] * n[0] - h[0] * n[2];
  a[2] = h[0] * n[1] - h[1] * n[0];
  double l = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
  a[0] /= l; a[1] /= l; a[2] /= l;
  b[0] = n[1] * a[2] - n[2] * a[1];
  b[1] = n[2] * a[0] - n[0] * a[2];
  b[2] = n[0] * a[1] - n[1] * a[0];
}

/* Equilateral triangle with centroid c, edge length s, random orientation
 * drawn from two sphere uniforms and one angle uniform. */
static void equilateral(const double c[3], double s, double u1, double u2, double u3, float* out9) {
  double n[3], a[3], b[3];
  unit_sphere(u1, u2, n);
  tangent_frame(n, a, b);
  double R = s / sqrt(3.0);
  double th = 2.0 * PI_D * u3;
  for (int k = 0; k < 3; ++k) {
    double ang = th + 2.0 * PI_D * k / 3.0;
    double ca = cos(ang), sa = sin(ang);
    for (int i = 0; i < 3; ++i) out9[3 * k + i] = (float)(c[i] + R * (ca * a[i] + sa * b[i]));
  }
}

/* ---------------------------------------------------- random-soup scene */

/* n random equilateral triangles: centroid uniform in [0,1]^3, edge length
 * uniform in (edge_lo, edge_hi). */
void wl_random_tris(uint64_t seed, int64_t n, double edge_lo, double edge_hi, float* out) {
  for (int64_t i = 0; i < n; ++i) {
    double c[3] = {rngu(seed, 1, 8 * i + 0), rngu(seed, 1, 8 * i + 1), rngu(seed, 1, 8 * i + 2)};
    double s = edge_lo + (edge_hi - edge_lo) * rngu(seed, 1, 8 * i + 3);
    equilateral(c, s, rngu(seed, 1, 8 * i + 4), rngu(seed, 1, 8 * i + 5), rngu(seed, 1, 8 * i + 6),
                out + 9 * i);
  }
}

/* n rays: origin uniform in [0,1]^3, direction uniform on the unit sphere,
 * tmin = 0, tmax = +inf. */
void wl_random_rays(uint64_t seed, int64_t n, float* out) {
  for (int64_t i = 0; i < n; ++i) {
    double d[3];
    unit_sphere(rngu(seed, 2, 8 * i + 3), rngu(seed, 2, 8 * i + 4), d);
    float* r = out + 8 * i;
    r[0] = (float)rngu(seed, 2, 8 * i + 0);
    r[1] = (float)rngu(seed, 2, 8 * i + 1);
    r[2] = (float)rngu(seed, 2, 8 * i + 2);
    r[3] = 0.0f;
    r[4] = (float)d[0]; r[5] = (float)d[1]; r[6] = (float)d[2];
    r[7] = INFINITY;
  }
}

/* ------------------------------------------------------------ grid city */

/* Box heights of an nx-by-nz city: LogNormal(0, 0.5) via Box-Muller. */
void wl_city_heights(uint64_t seed, int32_t nx, int32_t nz, double* heights) {
  for (int64_t c = 0; c < (int64_t)nx * nz; ++c) {
    double u1 = 1.0 - rngu(seed, 3, 2 * c), u2 = rngu(seed, 3, 2 * c + 1);
    double g = sqrt(-2.0 * log(u1)) * cos(2.0 * PI_D * u2);
    heights[c] = exp(0.5 * g);
  }
}

#define CITY_LO 0.1
#define CITY_HI 0.9

static void box_tris(double x0, double y0, double z0, double x1, double y1, double z1, float* o) {
  /* corners: bit0 -> x, bit1 -> y, bit2 -> z */
  double P[8][3];
  for (int k = 0; k < 8; ++k) {
    P[k][0] = (k & 1) ? x1 : x0;
    P[k][1] = (k & 2) ? y1 : y0;
    P[k][2] = (k & 4) ? z1 : z0;
  }
  static const int F[12][3] = {
      {0, 2, 6}, {0, 6, 4},  /* -x */
      {1, 5, 7}, {1, 7, 3},  /* +x */
      {0, 4, 5}, {0, 5, 1},  /* -y */
      {2, 3, 7}, {2, 7, 6},  /* +y */
      {0, 1, 3}, {0, 3, 2},  /* -z */
      {4, 6, 7}, {4, 7, 5},  /* +z */
  };
  for (int t = 0; t < 12; ++t)
    for (int v = 0; v < 3; ++v)
      for (int i = 0; i < 3; ++i) o[9 * t + 3 * v + i] = (float)P[F[t][v]][i];
}

/* Triangles of the city: 12 per box (cell (i,j) holds the box
 * [i+0.1, i+0.9] x [0, h] x [j+0.1, j+0.9]), then n_clutter random
 * equilateral triangles (centroid uniform in [0,nx] x [0,3] x [0,nz], edge
 * uniform in (0.05, 0.5)), then the ground quad y = 0 over [0,nx] x [0,nz]
 * as 2 triangles.  Returns the triangle count; out must hold
 * 9 * (12*nx*nz + n_clutter + 2) floats. */
int64_t wl_city_tris(uint64_t seed, int32_t nx, int32_t nz, int64_t n_clutter, const double* heights,
                     float* out) {
  int64_t t = 0;
  for (int32_t j = 0; j < nz; ++j)
    for (int32_t i = 0; i < nx; ++i) {
      double h = heights[(int64_t)j * nx + i];
      box_tris(i + CITY_LO, 0.0, j + CITY_LO, i + CITY_HI, h, j + CITY_HI, out + 9 * t);
      t += 12;
    }
  for (int64_t k = 0; k < n_clutter; ++k) {
    double c[3] = {nx * rngu(seed, 4, 8 * k + 0), 3.0 * rngu(seed, 4, 8 * k + 1), nz * rngu(seed, 4, 8 * k + 2)};
    double s = 0.05 + 0.45 * rngu(seed, 4, 8 * k + 3);
    equilateral(c, s, rngu(seed, 4, 8 * k + 4), rngu(seed, 4, 8 * k + 5), rngu(seed, 4, 8 * k + 6), out + 9 * t);
    ++t;
  }
  float g[2][9] = {{0, 0, 0, (float)nx, 0, 0, (float)nx, 0, (float)nz},
                   {0, 0, 0, (float)nx, 0, (float)nz, 0, 0, (float)nz}};
  memcpy(out + 9 * t, g, sizeof g);
  t += 2;
  return t;
}

typedef struct {
  const double* h;
  int32_t nx, nz;
  double hmax;
} city;

/* Closest analytic hit of the ray (o, d), t > tlo, against the city boxes and
 * the ground quad.  Returns 1 and the hit t and outward axis normal, or 0. */
static int city_hit(const city* C, const double o[3], const double d[3], double tlo, double* thit, double nrm[3]) {
  double best = INFINITY;
  int axis = -1;
  double sign = 0;
  /* ground */
  if (d[1] < 0.0) {
    double tg = -o[1] / d[1];
    if (tg > tlo) {
      double x = o[0] + tg * d[0], z = o[2] + tg * d[2];
      if (x >= 0.0 && x <= C->nx && z >= 0.0 && z <= C->nz) { best = tg; axis = 1; sign = 1.0; }
    }
  }
  /* clip the ray to the grid's xz rectangle */
  double t0 = tlo, t1 = best;
  double lo2[2] = {0.0, 0.0}, hi2[2] = {(double)C->nx, (double)C->nz};
  const int ax2[2] = {0, 2};
  for (int k = 0; k < 2; ++k) {
    int a = ax2[k];
    if (d[a] == 0.0) {
      if (o[a] < lo2[k] || o[a] > hi2[k]) t1 = -1.0;
    } else {
      double ta = (lo2[k] - o[a]) / d[a], tb = (hi2[k] - o[a]) / d[a];
      if (ta > tb) { double s = ta; ta = tb; tb = s; }
      if (ta > t0) t0 = ta;
      if (tb < t1) t1 = tb;
    }
  }
  /* above every roof and not descending: no box can be hit */
  if (d[1] >= 0.0 && o[1] + (d[1] > 0 ? t0 * d[1] : 0.0) > C->hmax) t1 = -1.0;
  if (t0 <= t1) {
    double px = o[0] + t0 * d[0], pz = o[2] + t0 * d[2];
    int ix = (int)floor(px), iz = (int)floor(pz);
    if (ix < 0) ix = 0;
    if (ix >= C->nx) ix = C->nx - 1;
    if (iz < 0) iz = 0;
    if (iz >= C->nz) iz = C->nz - 1;
    int sx = d[0] > 0 ? 1 : -1, sz = d[2] > 0 ? 1 : -1;
    double tnx = d[0] != 0.0 ? ((ix + (sx > 0 ? 1 : 0)) - o[0]) / d[0] : INFINITY;
    double tnz = d[2] != 0.0 ? ((iz + (sz > 0 ? 1 : 0)) - o[2]) / d[2] : INFINITY;
    double dtx = d[0] != 0.0 ? fabs(1.0 / d[0]) : INFINITY;
    double dtz = d[2] != 0.0 ? fabs(1.0 / d[2]) : INFINITY;
    for (int guard = 0; guard < 4 * (C->nx + C->nz) + 8; ++guard) {
      double h = C->h[(int64_t)iz * C->nx + ix];
      double blo[3] = {ix + CITY_LO, 0.0, iz + CITY_LO}, bhi[3] = {ix + CITY_HI, h, iz + CITY_HI};
      double tn = tlo, tf = INFINITY;
      int na = -1;
      double ns = 0;
      int ok = 1;
      for (int a = 0; a < 3 && ok; ++a) {
        if (d[a] == 0.0) {
          if (o[a] < blo[a] || o[a] > bhi[a]) ok = 0;
          continue;
        }
        double ta = (blo[a] - o[a]) / d[a], tb = (bhi[a] - o[a]) / d[a];
        double sa = -1.0;
        if (ta > tb) { double s = ta; ta = tb; tb = s; sa = 1.0; }
        if (ta > tn) { tn = ta; na = a; ns = sa; }
        if (tb < tf) tf = tb;
      }
      if (ok && na >= 0 && tn <= tf && tn > tlo && tn < best) {
        best = tn; axis = na; sign = ns;
        break; /* boxes lie inside their cells: the first cell hit is the closest */
      }
      double tcell = tnx < tnz ? tnx : tnz;
      if (tcell > t1) break;
      if (tnx < tnz) { ix += sx; tnx += dtx; if (ix < 0 || ix >= C->nx) break; }
      else { iz += sz; tnz += dtz; if (iz < 0 || iz >= C->nz) break; }
    }
  }
  if (axis < 0) return 0;
  *thit = best;
  nrm[0] = nrm[1] = nrm[2] = 0.0;
  nrm[axis] = sign;
  return 1;
}

/* Pinhole camera at eye looking straight down (-y), up = +z, vertical field
 * of view vfov_deg, image w x h, one jittered sample per pixel. */
void wl_camera_rays(uint64_t seed, int32_t w, int32_t h, const double eye[3], double vfov_deg, float* out) {
  double th = tan(0.5 * vfov_deg * PI_D / 180.0), asp = (double)w / h;
  /* forward (0,-1,0), up (0,0,1), right = forward x up = (-1,0,0) */
  for (int64_t p = 0; p < (int64_t)w * h; ++p) {
    int64_t px = p % w, py = p / w;
    double sx = (2.0 * (px + rngu(seed, 5, 2 * p)) / w - 1.0) * th * asp;
    double sy = (1.0 - 2.0 * (py + rngu(seed, 5, 2 * p + 1)) / h) * th;
    double d[3] = {-sx, -1.0, sy};
    double l = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    float* r = out + 8 * p;
    r[0] = (float)eye[0]; r[1] = (float)eye[1]; r[2] = (float)eye[2]; r[3] = 0.0f;
    r[4] = (float)(d[0] / l); r[5] = (float)(d[1] / l); r[6] = (float)(d[2] / l); r[7] = INFINITY;
  }
}

typedef struct {
  city C;
  uint64_t seed, stream;
  double offset;
  const float* in;
  float* out;
  uint8_t* alive;
} bounce_ctx;

static void bounce_range(void* p, int64_t lo, int64_t hi) {
  bounce_ctx* b = (bounce_ctx*)p;
  for (int64_t i = lo; i < hi; ++i) {
    const float* r = b->in + 8 * i;
    float* q = b->out + 8 * i;
    double o[3] = {r[0], r[1], r[2]}, d[3] = {r[4], r[5], r[6]};
    double t, n[3];
    int hit = b->alive[i] && city_hit(&b->C, o, d, 0.0, &t, n);
    if (!hit) {
      /* terminated slot: keep a well-formed ray so that untouched slots are still traceable */
      memcpy(q, r, 8 * sizeof(float));
      b->alive[i] = 0;
      continue;
    }
    if (n[0] * d[0] + n[1] * d[1] + n[2] * d[2] > 0.0) { n[0] = -n[0]; n[1] = -n[1]; n[2] = -n[2]; }
    double a[3], c[3];
    tangent_frame(n, a, c);
    /* Malley's method: uniform point on the unit disk lifted to the hemisphere */
    double u1 = rngu(b->seed, b->stream, 2 * i), u2 = rngu(b->seed, b->stream, 2 * i + 1);
    double rr = sqrt(u1), ph = 2.0 * PI_D * u2;
    double lx = rr * cos(ph), ly = rr * sin(ph), lz = sqrt(fmax(0.0, 1.0 - u1));
    double nd[3];
    for (int k = 0; k < 3; ++k) nd[k] = lx * a[k] + ly * c[k] + lz * n[k];
    double l = sqrt(nd[0] * nd[0] + nd[1] * nd[1] + nd[2] * nd[2]);
    for (int k = 0; k < 3; ++k) {
      q[k] = (float)(o[k] + t * d[k] + b->offset * n[k]);
      q[4 + k] = (float)(nd[k] / l);
    }
    q[3] = 0.0f;
    q[7] = INFINITY;
  }
}

/* One diffuse bounce in the analytic city: for each input ray whose alive
 * flag is set, find its hit, and emit a cosine-weighted ray about the
 * geometric normal (flipped against the incoming ray) from the hit point
 * pushed off the surface by `offset`.  alive is updated in place (0 where the
 * input ray escapes).  Returns the number of live output rays. */
int64_t wl_city_bounce(uint64_t seed, uint64_t stream, int32_t nx, int32_t nz, const double* heights,
                       const float* rays_in, int64_t n, double offset, float* rays_out, uint8_t* alive,
                       int32_t nthreads) {
  bounce_ctx b;
  b.C.h = heights; b.C.nx = nx; b.C.nz = nz;
  b.C.hmax = 0.0;
  for (int64_t c = 0; c < (int64_t)nx * nz; ++c) if (heights[c] > b.C.hmax) b.C.hmax = heights[c];
  b.seed = seed; b.stream = stream; b.offset = offset;
  b.in = rays_in; b.out = rays_out; b.alive = alive;
  parallel_for(n, nthreads, bounce_range, &b);
  int64_t live = 0;
  for (int64_t i = 0; i < n; ++i) live += alive[i] ? 1 : 0;
  return live;
}

/* Analytic city hit distance per ray (INFINITY on escape); used by the
 * generator's self-checks. */
typedef struct { city C; const float* in; double* t; } hitd_ctx;
static void hitd_range(void* p, int64_t lo, int64_t hi) {
  hitd_ctx* c = (hitd_ctx*)p;
  for (int64_t i = lo; i < hi; ++i) {
    const float* r = c->in + 8 * i;
    double o[3] = {r[0], r[1], r[2]}, d[3] = {r[4], r[5], r[6]}, t, n[3];
    c->t[i] = city_hit(&c->C, o, d, 0.0, &t, n) ? t : INFINITY;
  }
}
void wl_city_hit_t(int32_t nx, int32_t nz, const double* heights, const float* rays, int64_t n, double* t_out,
                   int32_t nthreads) {
  hitd_ctx c;
  c.C.h = heights; c.C.nx = nx; c.C.nz = nz; c.C.hmax = 0.0;
  for (int64_t k = 0; k < (int64_t)nx * nz; ++k) if (heights[k] > c.C.hmax) c.C.hmax = heights[k];
  c.in = rays; c.t = t_out;
  parallel_for(n, nthreads, hitd_range, &c);
}

/* n indices drawn uniformly with replacement from [0, pool). */
void wl_sample(uint64_t seed, uint64_t stream, int64_t n, int64_t pool, int64_t* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = (int64_t)(rng64(seed, stream, (uint64_t)i) % (uint64_t)pool);
}

/* Shadow rays toward a square area light of side `size` centred at lc and
 * lying in the plane y = lc[1]: `spp` rays per origin (the origins of
 * rays_in), light points uniform on the square from the counter generator
 * (stream `stream`, two draws per ray); direction normalised in double,
 * tmin 0, tmax the distance to the light point. */
void wl_shadow_rays(uint64_t seed, uint64_t stream, const float* rays_in, int64_t n, const double* lc, double size,
                    int32_t spp, float* out) {
  for (int64_t i = 0; i < n; ++i) {
    const float* o = rays_in + 8 * i;
    for (int32_t s = 0; s < spp; ++s) {
      const int64_t k = i * spp + s;
      const double u1 = rngu(seed, stream, 2 * (uint64_t)k), u2 = rngu(seed, stream, 2 * (uint64_t)k + 1);
      const double L[3] = {lc[0] + (u1 - 0.5) * size, lc[1], lc[2] + (u2 - 0.5) * size};
      const double d[3] = {L[0] - o[0], L[1] - o[1], L[2] - o[2]};
      const double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      float* r = out + 8 * k;
      r[0] = o[0];
      r[1] = o[1];
      r[2] = o[2];
      r[3] = 0.0f;
      r[4] = (float)(d[0] / len);
      r[5] = (float)(d[1] / len);
      r[6] = (float)(d[2] / len);
      r[7] = (float)len;
    }
  }
}
