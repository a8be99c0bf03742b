/* adgi_oracle.c - FP64 CPU oracle for the adaptive probe-update path.
 *
 * TEST INFRASTRUCTURE: loaded only by the tests, the smoke check and the
 * benchmark's CPU-baseline leg. Shares no code with the GPU library.
 *
 * Every function below follows a passage of the paper (Datta, Goli & Zhang,
 * "Adaptive Dynamic Global Illumination", arXiv 2301.05125) or a named
 * published method; the comment on each says which. Where the paper is silent
 * the reading taken is stated in the comment.
 */
#include "adgi_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------ RNG */

/* splitmix64 output function (Steele, Lea & Flood, OOPSLA 2014). */
uint64_t orc_splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* Key of one random stream: successive mixes of seed^tag, a, b, c. */
uint64_t orc_key(uint64_t seed, uint64_t tag, uint64_t a, uint64_t b, uint64_t c) {
  uint64_t h = orc_splitmix64(seed ^ tag);
  h = orc_splitmix64(h ^ a);
  h = orc_splitmix64(h ^ b);
  h = orc_splitmix64(h ^ c);
  return h;
}

double orc_uniform(uint64_t key, uint64_t q) {
  uint64_t x = orc_splitmix64(key ^ q);
  return (double)(x >> 40) * (1.0 / 16777216.0);
}

/* One uniformly random rotation per frame (the "stochastic rotated" ray set
 * of DDGI, Sec. 3.1), from Shoemake's quaternion construction. Computed in
 * FP64 and rounded to FP32: both the GPU and this oracle use the FP32 matrix. */
void orc_frame_rotation(uint64_t seed, int32_t frame, float R[9]) {
  uint64_t key = orc_key(seed, ORC_TAG_ROTATION, (uint64_t)(uint32_t)frame, 0, 0);
  double u1 = orc_uniform(key, 1), u2 = orc_uniform(key, 2), u3 = orc_uniform(key, 3);
  double a = sqrt(1.0 - u1), b = sqrt(u1);
  double x = a * sin(2.0 * PI * u2), y = a * cos(2.0 * PI * u2);
  double z = b * sin(2.0 * PI * u3), w = b * cos(2.0 * PI * u3);
  double m[9] = {
      1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - z * w), 2.0 * (x * z + y * w),
      2.0 * (x * y + z * w), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - x * w),
      2.0 * (x * z - y * w), 2.0 * (y * z + x * w), 1.0 - 2.0 * (x * x + y * y)};
  for (int i = 0; i < 9; ++i) R[i] = (float)m[i];
}

/* Spherical Fibonacci point set (Marques et al. 2013; Keinert et al. 2015):
 * z_j = 1 - (2j+1)/n, phi_j = 2*pi*frac(j / golden ratio). The fraction is
 * taken exactly from the 64-bit fixed-point product j * 2^64/phi. */
void orc_sf_dir(int32_t j, int32_t n, const float R[9], double d[3]) {
  double z = 1.0 - (2.0 * j + 1.0) / (double)n;
  uint64_t f = (uint64_t)(uint32_t)j * 0x9E3779B97F4A7C15ull;
  double phi = 2.0 * PI * ((double)f * 0x1p-64);
  double r = sqrt(fmax(0.0, 1.0 - z * z));
  double v[3] = {r * cos(phi), r * sin(phi), z};
  for (int a = 0; a < 3; ++a)
    d[a] = (double)R[3 * a + 0] * v[0] + (double)R[3 * a + 1] * v[1] + (double)R[3 * a + 2] * v[2];
}

/* Which spherical Fibonacci point ray j of a probe with n rays takes. The
 * paper fixes the point set of a probe's rays, not which ray gets which
 * point, nor the order in which a texel's samples enter its moving average
 * (its updates are atomic). Reading taken here: the points are dealt into
 * C = ceil(n/64) strata by index modulo C (stratum c holds c, c + C, c + 2C,
 * ... in ascending order), ray indices run through stratum 0, then stratum 1,
 * and so on, and a texel takes its samples in ascending ray index. Each
 * stratum spreads over the whole sphere. n <= 64: ray j takes point j. */
int32_t orc_ray_point(int32_t j, int32_t n) {
  const int64_t C = ((int64_t)n + 63) / 64;
  if (C <= 1) return j;
  /* stratum c holds ceil((n - c) / C) points */
  int64_t c = 0, first = 0;
  for (;;) {
    const int64_t size = ((int64_t)n - c + C - 1) / C;
    if (j < first + size) return (int32_t)(c + (j - first) * C);
    first += size;
    ++c;
  }
}

/* Pilot ray of octant k (Sec. 4.4): one stratified-random direction per
 * octant, the same for both frames of a pair (AABBCC... pattern). A uniform
 * sphere point folded into the octant. */
void orc_pilot_dir(uint64_t seed, int32_t probe, int32_t k, int32_t pair, double d[3]) {
  uint64_t key = orc_key(seed, ORC_TAG_PILOT, (uint64_t)(uint32_t)probe, (uint64_t)(uint32_t)k,
                         (uint64_t)(uint32_t)pair);
  double u = orc_uniform(key, 1), v = orc_uniform(key, 2);
  double z = 1.0 - 2.0 * u;
  double r = sqrt(fmax(0.0, 1.0 - z * z));
  double phi = 2.0 * PI * v;
  d[0] = fabs(r * cos(phi));
  d[1] = fabs(r * sin(phi));
  d[2] = fabs(z);
  if (k & 1) d[0] = -d[0];
  if (k & 2) d[1] = -d[1];
  if (k & 4) d[2] = -d[2];
}

/* ------------------------------------------------------------ octahedral */

static double sgn_nz(double x) { return x >= 0.0 ? 1.0 : -1.0; }

/* Octahedral unit-vector map (Cigolle et al., JCGT 2014): the paper's
 * "spherical mapping" of probe texels (Sec. 4.5), labelled octahedral in its
 * method figure. */
void orc_oct_encode(const double d[3], double uv[2]) {
  double l1 = fabs(d[0]) + fabs(d[1]) + fabs(d[2]);
  double x = d[0] / l1, y = d[1] / l1, z = d[2] / l1;
  if (z < 0.0) {
    double nx = (1.0 - fabs(y)) * sgn_nz(x);
    double ny = (1.0 - fabs(x)) * sgn_nz(y);
    x = nx;
    y = ny;
  }
  uv[0] = x;
  uv[1] = y;
}

void orc_oct_decode(const double uv[2], double d[3]) {
  double x = uv[0], y = uv[1];
  double z = 1.0 - fabs(x) - fabs(y);
  if (z < 0.0) {
    double nx = (1.0 - fabs(y)) * sgn_nz(x);
    double ny = (1.0 - fabs(x)) * sgn_nz(y);
    x = nx;
    y = ny;
  }
  double n = sqrt(x * x + y * y + z * z);
  d[0] = x / n;
  d[1] = y / n;
  d[2] = z / n;
}

/* The texel containing a direction ("closest entry", Alg. ApproxAlgo):
 * half-open cells over [-1,1]^2, the last one closed. */
int32_t orc_oct_bin(const double d[3], int32_t r, double eps, int32_t* tie) {
  double uv[2];
  orc_oct_encode(d, uv);
  int32_t idx[2];
  int32_t t = 0;
  for (int a = 0; a < 2; ++a) {
    double f = (uv[a] + 1.0) * 0.5 * r;
    int32_t i = (int32_t)floor(f);
    if (i > r - 1) i = r - 1;
    if (i < 0) i = 0;
    idx[a] = i;
    double frac = f - floor(f);
    if ((frac < eps || frac > 1.0 - eps) && f > eps && f < r - eps) t = 1;
  }
  /* lower hemisphere: the fold is discontinuous where x or y changes sign */
  double l1 = fabs(d[0]) + fabs(d[1]) + fabs(d[2]);
  if (d[2] / l1 < eps && (fabs(d[0]) / l1 < eps || fabs(d[1]) / l1 < eps)) t = 1;
  if (tie) *tie = t;
  return idx[1] * r + idx[0];
}

/* Border texels repeat the interior texel across the map's edge
 * identification (u,+-1) ~ (-u,+-1), (+-1,v) ~ (+-1,-v), so that bilinear
 * filtering of the tile is continuous over the sphere. */
void orc_border_source(int32_t X, int32_t Y, int32_t r, int32_t* sx, int32_t* sy) {
  int32_t x = X, y = Y;
  int32_t bx = (X == 0 || X == r + 1), by = (Y == 0 || Y == r + 1);
  if (bx && by) {
    x = (X == 0) ? r : 1;
    y = (Y == 0) ? r : 1;
  } else if (by) {
    x = r + 1 - X;
    y = (Y == 0) ? 1 : r;
  } else if (bx) {
    y = r + 1 - Y;
    x = (X == 0) ? 1 : r;
  }
  *sx = x;
  *sy = y;
}

void orc_fold_tile(const double* interior, int32_t r, int32_t c, double* tile) {
  int32_t w = r + 2;
  for (int32_t Y = 0; Y < w; ++Y)
    for (int32_t X = 0; X < w; ++X) {
      int32_t sx, sy;
      orc_border_source(X, Y, r, &sx, &sy);
      for (int32_t k = 0; k < c; ++k)
        tile[(Y * w + X) * c + k] = interior[((sy - 1) * r + (sx - 1)) * c + k];
    }
}

/* ------------------------------------------------------------ tolerances */

void orc_default_tol(orc_tol* tol) {
  tol->hit_rel = 1e-5;
  tol->edge_rel = 2e-6;
  tol->edge_abs = 1e-7;
  tol->graze = 1e-4;
  tol->bin_eps = 2e-5;
  tol->q10_rel = 1e-4;
  tol->q10_abs = 1e-3;
  tol->cos_eps = 1e-5;
}

/* ----------------------------------------------------------------- scene */

typedef struct {
  double lo[3], hi[3];
  int32_t left, right;   /* children; leaf when count > 0 */
  int32_t start, count;
} onode;

struct orc_scene {
  int32_t nv, nt;
  double* v;          /* [nv*3] */
  int32_t* idx;       /* [nt*3] */
  double* albedo;     /* [nt*3] */
  double* tri;        /* per triangle: v0[3] e1[3] e2[3] n[3] h[3]  (15 doubles) */
  double vmax;        /* max |coordinate| of any vertex */
  double blo[3], bhi[3];
  int32_t use_bvh;
  onode* nodes;
  int32_t nnodes;
  int32_t* order;     /* triangle order of BVH leaves */
  int32_t depth;
  int32_t nl;
  double* lpos;
  double* lint;
  double sky[3];
};

static void cross3(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }
static double maxabs3(const double a[3]) {
  return fmax(fabs(a[0]), fmax(fabs(a[1]), fabs(a[2])));
}

static void scene_prepare(orc_scene* s) {
  s->vmax = 0.0;
  for (int a = 0; a < 3; ++a) {
    s->blo[a] = INFINITY;
    s->bhi[a] = -INFINITY;
  }
  for (int32_t i = 0; i < s->nv; ++i)
    for (int a = 0; a < 3; ++a) {
      double x = s->v[3 * i + a];
      s->vmax = fmax(s->vmax, fabs(x));
      s->blo[a] = fmin(s->blo[a], x);
      s->bhi[a] = fmax(s->bhi[a], x);
    }
  for (int32_t t = 0; t < s->nt; ++t) {
    const double* v0 = s->v + 3 * s->idx[3 * t];
    const double* v1 = s->v + 3 * s->idx[3 * t + 1];
    const double* v2 = s->v + 3 * s->idx[3 * t + 2];
    double* T = s->tri + 15 * t;
    double e1[3], e2[3], n[3], e12[3];
    for (int a = 0; a < 3; ++a) {
      e1[a] = v1[a] - v0[a];
      e2[a] = v2[a] - v0[a];
      e12[a] = v2[a] - v1[a];
    }
    cross3(e1, e2, n);
    double twoA = norm3(n);
    for (int a = 0; a < 3; ++a) {
      T[a] = v0[a];
      T[3 + a] = e1[a];
      T[6 + a] = e2[a];
      T[9 + a] = n[a];
    }
    /* altitudes opposite v0, v1, v2 */
    T[12] = twoA / fmax(norm3(e12), 1e-300);
    T[13] = twoA / fmax(norm3(e2), 1e-300);
    T[14] = twoA / fmax(norm3(e1), 1e-300);
  }
}

/* ---- median-split BVH of the oracle's own (leaves of at most 4 triangles) */

static double centroid(const orc_scene* s, int32_t t, int a) {
  const double* T = s->tri + 15 * t;
  return T[a] + (T[3 + a] + T[6 + a]) / 3.0;
}

static void select_kth(const orc_scene* s, int32_t* arr, int32_t n, int32_t k, int a) {
  int32_t lo = 0, hi = n - 1;
  while (lo < hi) {
    double pivot = centroid(s, arr[(lo + hi) / 2], a);
    int32_t i = lo, j = hi;
    while (i <= j) {
      while (centroid(s, arr[i], a) < pivot) ++i;
      while (centroid(s, arr[j], a) > pivot) --j;
      if (i <= j) {
        int32_t tmp = arr[i];
        arr[i] = arr[j];
        arr[j] = tmp;
        ++i;
        --j;
      }
    }
    if (k <= j) hi = j;
    else if (k >= i) lo = i;
    else break;
  }
}

static void node_bounds(const orc_scene* s, onode* nd) {
  for (int a = 0; a < 3; ++a) {
    nd->lo[a] = INFINITY;
    nd->hi[a] = -INFINITY;
  }
  for (int32_t i = 0; i < nd->count; ++i) {
    int32_t t = s->order[nd->start + i];
    for (int c = 0; c < 3; ++c) {
      const double* p = s->v + 3 * s->idx[3 * t + c];
      for (int a = 0; a < 3; ++a) {
        nd->lo[a] = fmin(nd->lo[a], p[a]);
        nd->hi[a] = fmax(nd->hi[a], p[a]);
      }
    }
  }
}

static void bvh_build(orc_scene* s) {
  free(s->nodes);
  free(s->order);
  s->nodes = NULL;
  s->order = NULL;
  s->nnodes = 0;
  s->depth = 0;
  if (!s->use_bvh || s->nt == 0) return;
  s->order = (int32_t*)malloc(sizeof(int32_t) * s->nt);
  for (int32_t i = 0; i < s->nt; ++i) s->order[i] = i;
  int32_t cap = 2 * s->nt + 1;
  s->nodes = (onode*)malloc(sizeof(onode) * cap);
  int32_t* stack = (int32_t*)malloc(sizeof(int32_t) * 2 * cap);
  int32_t* dstack = stack + cap;
  int32_t sp = 0;
  s->nodes[0].start = 0;
  s->nodes[0].count = s->nt;
  s->nnodes = 1;
  stack[sp] = 0;
  dstack[sp++] = 1;
  while (sp > 0) {
    --sp;
    int32_t ni = stack[sp], depth = dstack[sp];
    if (depth > s->depth) s->depth = depth;
    onode* nd = &s->nodes[ni];
    node_bounds(s, nd);
    nd->left = nd->right = -1;
    if (nd->count <= 4) continue;
    /* split at the centroid median along the widest centroid extent */
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int32_t i = 0; i < nd->count; ++i)
      for (int a = 0; a < 3; ++a) {
        double c = centroid(s, s->order[nd->start + i], a);
        clo[a] = fmin(clo[a], c);
        chi[a] = fmax(chi[a], c);
      }
    int axis = 0;
    for (int a = 1; a < 3; ++a)
      if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
    int32_t half = nd->count / 2;
    select_kth(s, s->order + nd->start, nd->count, half, axis);
    int32_t L = s->nnodes++, Rn = s->nnodes++;
    s->nodes[L].start = nd->start;
    s->nodes[L].count = half;
    s->nodes[Rn].start = nd->start + half;
    s->nodes[Rn].count = nd->count - half;
    nd = &s->nodes[ni];
    nd->left = L;
    nd->right = Rn;
    nd->count = 0;
    stack[sp] = L;
    dstack[sp++] = depth + 1;
    stack[sp] = Rn;
    dstack[sp++] = depth + 1;
  }
  free(stack);
}

orc_scene* orc_scene_new(int32_t nv, const float* pos, int32_t nt, const int32_t* idx,
                         const float* albedo, int32_t use_bvh) {
  orc_scene* s = (orc_scene*)calloc(1, sizeof(orc_scene));
  s->nv = nv;
  s->nt = nt;
  s->v = (double*)malloc(sizeof(double) * 3 * (nv > 0 ? nv : 1));
  s->idx = (int32_t*)malloc(sizeof(int32_t) * 3 * (nt > 0 ? nt : 1));
  s->albedo = (double*)malloc(sizeof(double) * 3 * (nt > 0 ? nt : 1));
  s->tri = (double*)malloc(sizeof(double) * 15 * (nt > 0 ? nt : 1));
  for (int32_t i = 0; i < 3 * nv; ++i) s->v[i] = pos[i];
  for (int32_t i = 0; i < 3 * nt; ++i) {
    s->idx[i] = idx[i];
    s->albedo[i] = albedo[i];
  }
  s->use_bvh = use_bvh;
  scene_prepare(s);
  bvh_build(s);
  return s;
}

void orc_scene_free(orc_scene* s) {
  if (!s) return;
  free(s->v);
  free(s->idx);
  free(s->albedo);
  free(s->tri);
  free(s->nodes);
  free(s->order);
  free(s->lpos);
  free(s->lint);
  free(s);
}

void orc_scene_set_positions(orc_scene* s, const float* pos) {
  for (int32_t i = 0; i < 3 * s->nv; ++i) s->v[i] = pos[i];
  scene_prepare(s);
  bvh_build(s);
}

void orc_scene_set_lights(orc_scene* s, int32_t nl, const float* lpos, const float* lint,
                          const float sky[3]) {
  free(s->lpos);
  free(s->lint);
  s->nl = nl;
  s->lpos = (double*)malloc(sizeof(double) * 3 * (nl > 0 ? nl : 1));
  s->lint = (double*)malloc(sizeof(double) * 3 * (nl > 0 ? nl : 1));
  for (int32_t i = 0; i < 3 * nl; ++i) {
    s->lpos[i] = lpos[i];
    s->lint[i] = lint[i];
  }
  for (int a = 0; a < 3; ++a) s->sky[a] = sky[a];
}

int32_t orc_scene_bvh_depth(const orc_scene* s) { return s->depth; }

/* ------------------------------------------------------- ray / triangle */

/* Moller & Trumbore (1997) in FP64. Returns the plane distance t, the
 * barycentrics (b1 = u, b2 = v) and the determinant. Triangles are
 * two-sided; det == 0 is a miss. */
typedef struct {
  double t, u, v, det, cosang;
  double dmin;        /* signed world distance of the plane point to the nearest edge */
  int valid;          /* det != 0 */
} tri_isect;

static void tri_test(const orc_scene* s, int32_t t, const double o[3], const double d[3],
                     tri_isect* r) {
  const double* T = s->tri + 15 * t;
  const double *v0 = T, *e1 = T + 3, *e2 = T + 6, *n = T + 9;
  double p[3], q[3], tv[3];
  cross3(d, e2, p);
  double det = dot3(e1, p);
  r->det = det;
  r->valid = det != 0.0;
  double nn = norm3(n), dn = norm3(d);
  r->cosang = (nn > 0.0 && dn > 0.0) ? dot3(n, d) / (nn * dn) : 0.0;
  if (!r->valid) {
    r->t = INFINITY;
    r->u = r->v = -1.0;
    r->dmin = -INFINITY;
    return;
  }
  double inv = 1.0 / det;
  for (int a = 0; a < 3; ++a) tv[a] = o[a] - v0[a];
  r->u = dot3(tv, p) * inv;
  cross3(tv, e1, q);
  r->v = dot3(d, q) * inv;
  r->t = dot3(e2, q) * inv;
  double b0 = 1.0 - r->u - r->v;
  double d0 = b0 * T[12], d1 = r->u * T[13], d2 = r->v * T[14];
  r->dmin = fmin(d0, fmin(d1, d2));
}

static int exact_hit(const tri_isect* r, double tmin, double tmax) {
  return r->valid && r->u >= 0.0 && r->v >= 0.0 && r->u + r->v <= 1.0 && r->t > tmin &&
         r->t < tmax;
}

static int slab(const double lo[3], const double hi[3], double pad, const double o[3],
                const double d[3], double tmin, double tmax) {
  for (int a = 0; a < 3; ++a) {
    double l = lo[a] - pad, h = hi[a] + pad;
    if (d[a] == 0.0) {
      if (o[a] < l || o[a] > h) return 0;
      continue;
    }
    double t0 = (l - o[a]) / d[a], t1 = (h - o[a]) / d[a];
    if (t0 > t1) {
      double x = t0;
      t0 = t1;
      t1 = x;
    }
    if (t0 > tmin) tmin = t0;
    if (t1 < tmax) tmax = t1;
    if (tmin > tmax) return 0;
  }
  return 1;
}

/* Visit every triangle whose (padded) node boxes meet the ray on
 * [tmin, *tmax]. The callback may shrink *tmax. Brute force without a BVH. */
typedef void (*visit_fn)(const orc_scene* s, int32_t t, void* ctx, double* tmax);

static void visit(const orc_scene* s, const double o[3], const double d[3], double pad,
                  double tmin, double* tmax, visit_fn fn, void* ctx) {
  if (!s->use_bvh || s->nnodes == 0) {
    for (int32_t t = 0; t < s->nt; ++t) fn(s, t, ctx, tmax);
    return;
  }
  int32_t stack[256];
  int32_t sp = 0;
  stack[sp++] = 0;
  while (sp > 0) {
    const onode* nd = &s->nodes[stack[--sp]];
    if (!slab(nd->lo, nd->hi, pad, o, d, tmin, *tmax)) continue;
    if (nd->left < 0) {
      for (int32_t i = 0; i < nd->count; ++i) fn(s, s->order[nd->start + i], ctx, tmax);
    } else {
      stack[sp++] = nd->left;
      stack[sp++] = nd->right;
    }
  }
}

typedef struct {
  const double *o, *d;
  double t;
  int32_t tri;
} closest_ctx;

static void closest_cb(const orc_scene* s, int32_t t, void* vctx, double* tmax) {
  closest_ctx* c = (closest_ctx*)vctx;
  tri_isect r;
  tri_test(s, t, c->o, c->d, &r);
  if (!exact_hit(&r, 0.0, INFINITY)) return;
  /* ties on t break towards the lowest triangle index */
  if (r.t < c->t || (r.t == c->t && t < c->tri)) {
    c->t = r.t;
    c->tri = t;
    if (r.t < *tmax) *tmax = r.t * (1.0 + 1e-12);
  }
}

static double margin(const orc_tol* tol, const double o[3], double t, double vmax) {
  double tt = isfinite(t) ? t : 0.0;
  return tol->edge_abs + tol->edge_rel * (maxabs3(o) + tt + vmax);
}

static double far_distance(const orc_scene* s, const double o[3]) {
  double m = 0.0;
  for (int a = 0; a < 3; ++a) {
    double x = fmax(fabs(s->blo[a] - o[a]), fabs(s->bhi[a] - o[a]));
    m += x * x;
  }
  return sqrt(m);
}

typedef struct {
  const double *o, *d;
  const orc_tol* tol;
  double vmax;
  double tstar;
  int32_t tri;
  double tlim;
  int tie;
} tie_ctx;

/* Second pass: any triangle whose decision is ambiguous at FP32 precision. */
static void hit_tie_cb(const orc_scene* s, int32_t t, void* vctx, double* tmax) {
  (void)tmax;
  tie_ctx* c = (tie_ctx*)vctx;
  if (c->tie) return;
  tri_isect r;
  tri_test(s, t, c->o, c->d, &r);
  if (!r.valid) return;
  double m = margin(c->tol, c->o, r.t, c->vmax);
  if (t == c->tri) {
    if (r.dmin < m || r.t <= m || fabs(r.cosang) < c->tol->graze) c->tie = 1;
    return;
  }
  if (r.dmin >= -m && r.t > -m && r.t <= c->tlim) c->tie = 1;
}

static void closest_impl(const orc_scene* s, const double o[3], const double d[3],
                         const orc_tol* tol, orc_hit* out, int brute) {
  int32_t saved = s->use_bvh;
  if (brute) ((orc_scene*)s)->use_bvh = 0;
  closest_ctx c = {o, d, INFINITY, -1};
  double tmax = INFINITY;
  visit(s, o, d, 0.0, 0.0, &tmax, closest_cb, &c);
  out->t = c.t;
  out->tri = c.tri;
  out->front = 0;
  out->tie = 0;
  if (c.tri >= 0) {
    tri_isect r;
    tri_test(s, c.tri, o, d, &r);
    out->front = r.det > 0.0;  /* det > 0  <=>  (e1 x e2) . d < 0 */
  }
  if (tol) {
    tie_ctx tc;
    tc.o = o;
    tc.d = d;
    tc.tol = tol;
    tc.vmax = s->vmax;
    tc.tstar = c.t;
    tc.tri = c.tri;
    double tl = c.tri >= 0 ? c.t * (1.0 + tol->hit_rel) : far_distance(s, o) * 2.0 + 1.0;
    tc.tlim = tl + margin(tol, o, tl, s->vmax);
    tc.tie = 0;
    double pad = margin(tol, o, tc.tlim, s->vmax);
    double tm = tc.tlim;
    visit(s, o, d, pad, -pad, &tm, hit_tie_cb, &tc);
    out->tie = tc.tie;
  }
  if (brute) ((orc_scene*)s)->use_bvh = saved;
}

void orc_closest_hit(const orc_scene* s, const double o[3], const double d[3], const orc_tol* tol,
                     orc_hit* out) {
  closest_impl(s, o, d, tol, out, 0);
}

void orc_closest_hit_brute(const orc_scene* s, const double o[3], const double d[3],
                           const orc_tol* tol, orc_hit* out) {
  closest_impl(s, o, d, tol, out, 1);
}

typedef struct {
  const double *o, *d;
  const orc_tol* tol;
  double base, vmax, tmax;
  int exact, robust, possible;
} occ_ctx;

static void occ_cb(const orc_scene* s, int32_t t, void* vctx, double* tmax) {
  (void)tmax;
  occ_ctx* c = (occ_ctx*)vctx;
  if (c->robust) return;
  tri_isect r;
  tri_test(s, t, c->o, c->d, &r);
  if (!r.valid) return;
  if (exact_hit(&r, 0.0, c->tmax)) c->exact = 1;
  if (!c->tol) return;
  double m = c->base + margin(c->tol, c->o, r.t, c->vmax);
  if (r.dmin > m && r.t > m && r.t < c->tmax - m && fabs(r.cosang) >= c->tol->graze) {
    c->robust = 1;
    c->exact = 1;
  } else if (r.dmin >= -m && r.t > -m && r.t < c->tmax + m) {
    c->possible = 1;
  }
}

static int32_t occluded_base(const orc_scene* s, const double o[3], const double d[3], double tmax,
                             const orc_tol* tol, double base, int32_t* tie) {
  occ_ctx c = {o, d, tol, base, s->vmax, tmax, 0, 0, 0};
  double pad = tol ? base + margin(tol, o, tmax, s->vmax) : 0.0;
  double tm = tmax + pad;
  visit(s, o, d, pad, -pad, &tm, occ_cb, &c);
  if (tie) *tie = (!c.robust && c.possible) ? 1 : 0;
  return c.exact;
}

int32_t orc_occluded(const orc_scene* s, const double o[3], const double d[3], double tmax,
                     const orc_tol* tol, int32_t* tie) {
  return occluded_base(s, o, d, tmax, tol, 0.0, tie);
}

/* ----------------------------------------------------------- shading */

/* Radiance arriving at the probe along d (Sec. 3.1: probes hold diffuse
 * irradiance; Sec. 4.1.3: direct illumination at the hit point). Lambertian
 * triangles, isotropic point lights with inverse-square falloff, one shadow
 * ray per light facing the surface, sky radiance on a miss and zero on a back
 * face. Shadow rays start 1e-4*s along the normal and stop 1e-6 short of the
 * light (relative). */
void orc_shade_ray(const orc_scene* s, const double o[3], const double d[3], double spacing_diag,
                   const orc_tol* tol, int32_t hint_tri, int32_t hint_shadow, orc_ray* out,
                   int64_t* ties, int64_t* mismatches) {
  orc_hit h;
  orc_closest_hit(s, o, d, tol, &h);
  out->hit_tie = h.tie;
  out->shadow_tie = 0;
  if (hint_tri != -2 && hint_tri != h.tri) {
    if (h.tie) {
      if (ties) ties[0]++;
      h.tri = hint_tri;
      if (hint_tri >= 0) {
        tri_isect r;
        tri_test(s, hint_tri, o, d, &r);
        h.t = r.t;
        h.front = r.det > 0.0;
      } else {
        h.t = INFINITY;
        h.front = 0;
      }
    } else if (mismatches) {
      mismatches[0]++;
    }
  }
  out->t = h.t;
  out->tri = h.tri;
  out->front = h.front;
  out->shadow = 0;
  if (h.tri < 0) {
    for (int a = 0; a < 3; ++a) out->rgb[a] = s->sky[a];
    out->t = INFINITY;
    return;
  }
  if (!h.front) {
    for (int a = 0; a < 3; ++a) out->rgb[a] = 0.0;
    return;
  }
  const double* T = s->tri + 15 * h.tri;
  double nn = norm3(T + 9);
  double n[3] = {T[9] / nn, T[10] / nn, T[11] / nn};
  double x[3], E[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < 3; ++a) x[a] = o[a] + h.t * d[a];
  double base = tol ? margin(tol, o, h.t, s->vmax) : 0.0;
  for (int32_t l = 0; l < s->nl; ++l) {
    const double* lp = s->lpos + 3 * l;
    double L[3] = {lp[0] - x[0], lp[1] - x[1], lp[2] - x[2]};
    double dist2 = dot3(L, L), dist = sqrt(dist2);
    double c = dot3(n, L) / dist;
    int cos_tie = tol && fabs(c) < tol->cos_eps;
    int lit = 0, occ_tie = 0;
    if (c > 0.0) {
      double so[3], sd[3];
      for (int a = 0; a < 3; ++a) so[a] = x[a] + 1e-4 * spacing_diag * n[a];
      double seg[3] = {lp[0] - so[0], lp[1] - so[1], lp[2] - so[2]};
      double sl = norm3(seg);
      for (int a = 0; a < 3; ++a) sd[a] = seg[a] / sl;
      int32_t t_occ = 0;
      lit = !occluded_base(s, so, sd, sl * (1.0 - 1e-6), tol, base, &t_occ);
      occ_tie = t_occ;
    }
    int tie = cos_tie || occ_tie;
    if (tie) out->shadow_tie |= 1 << l;
    if (hint_shadow >= 0) {
      int g = (hint_shadow >> l) & 1;
      if (g != lit) {
        if (tie) {
          if (ties) ties[1]++;
          lit = g;
        } else if (mismatches) {
          mismatches[1]++;
        }
      }
    }
    if (lit) {
      out->shadow |= (uint8_t)(1u << l);
      double w = fmax(c, 0.0) / dist2;
      for (int a = 0; a < 3; ++a) E[a] += s->lint[3 * l + a] * w;
    }
  }
  const double* rho = s->albedo + 3 * h.tri;
  for (int a = 0; a < 3; ++a) out->rgb[a] = rho[a] / PI * E[a];
}

/* ------------------------------------------------------------------ grid */

void orc_grid_init(orc_grid* g, const float origin[3], const float spacing[3], const int32_t dims[3]) {
  for (int a = 0; a < 3; ++a) {
    g->origin[a] = origin[a];
    g->spacing[a] = spacing[a];
    g->dims[a] = dims[a];
  }
  /* the "diagonal distance of a grid voxel" of eq. ProbeVis */
  g->s = sqrt(g->spacing[0] * g->spacing[0] + g->spacing[1] * g->spacing[1] +
              g->spacing[2] * g->spacing[2]);
}

void orc_probe_pos(const orc_grid* g, int32_t i, double p[3]) {
  int32_t x = i % g->dims[0];
  int32_t y = (i / g->dims[0]) % g->dims[1];
  int32_t z = i / (g->dims[0] * g->dims[1]);
  p[0] = g->origin[0] + x * g->spacing[0];
  p[1] = g->origin[1] + y * g->spacing[1];
  p[2] = g->origin[2] + z * g->spacing[2];
}

/* ------------------------------------------------------------- detection */

static double lum709(const double c[3]) { return 0.2126 * c[0] + 0.7152 * c[1] + 0.0722 * c[2]; }

static int near_int(double x, double band) {
  double f = x - floor(x);
  return f < band || f > 1.0 - band;
}

/* Pilot rays (Sec. 4.1, 4.4) and the 10-bit codes of the two heuristics:
 * Qv = floor(1024 * f_v) with f_v = exp(-2t/s) (eq. ProbeVis), and
 * Qr = floor(1024 * f_r) with f_r = min(lum, beta)/beta (Sec. 4.1.3), each
 * capped at 1023. Round-down follows the paper's quantisation (App. B). */
void orc_pilots(const orc_scene* s, const orc_grid* g, uint64_t seed, int32_t frame, double beta,
                const orc_tol* tol, const uint16_t* hint_qv, const uint16_t* hint_qr,
                const int32_t* hint_tri, const uint8_t* hint_shadow,
                uint16_t* qv, uint16_t* qr, double* prgb, double* pt, orc_counts* counts) {
  int32_t P = g->dims[0] * g->dims[1] * g->dims[2];
  int32_t pair = frame / 2;
  int64_t ties = 0, mism = 0, sh = 0, hties = 0, sties = 0, hmism = 0, smism = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : ties, mism, sh, hties, sties, hmism, smism)
  for (int64_t r = 0; r < (int64_t)P * 8; ++r) {
    int32_t i = (int32_t)(r / 8), k = (int32_t)(r % 8);
    double o[3], d[3];
    orc_probe_pos(g, i, o);
    orc_pilot_dir(seed, i, k, pair, d);
    orc_ray ray;
    int64_t rt[2] = {0, 0}, rm[2] = {0, 0};
    orc_shade_ray(s, o, d, g->s, tol, hint_tri ? hint_tri[r] : -2, hint_shadow ? (int32_t)hint_shadow[r] : -1,
                  &ray, rt, rm);
    hties += rt[0];
    sties += rt[1];
    hmism += rm[0];
    smism += rm[1];
    if (prgb)
      for (int c = 0; c < 3; ++c) prgb[3 * r + c] = ray.rgb[c];
    if (pt) pt[r] = ray.t;
    for (int32_t l = 0; l < s->nl; ++l) sh += 1;
    double fv = isfinite(ray.t) ? exp(-2.0 * ray.t / g->s) : 0.0;
    double fr = fmin(lum709(ray.rgb), beta) / beta;
    double xv = 1024.0 * fv, xr = 1024.0 * fr;
    int32_t cv = (int32_t)floor(xv), cr = (int32_t)floor(xr);
    if (cv > 1023) cv = 1023;
    if (cr > 1023) cr = 1023;
    if (cv < 0) cv = 0;
    if (cr < 0) cr = 0;
    int tie_v = 0, tie_r = 0;
    if (tol) {
      double mt = margin(tol, o, isfinite(ray.t) ? ray.t : 0.0, s->vmax);
      double bv = tol->q10_abs + xv * (tol->q10_rel + 2.0 * mt / g->s);
      double br = tol->q10_abs + xr * tol->q10_rel;
      tie_v = ray.hit_tie || (xv < 1023.0 + bv && near_int(xv, bv));
      tie_r = ray.hit_tie || ray.shadow_tie || (xr < 1023.0 + br && near_int(xr, br));
    }
    if (hint_qv && hint_qv[r] != cv) {
      if (tie_v) {
        ++ties;
        cv = hint_qv[r];
      } else {
        ++mism;
      }
    }
    if (hint_qr && hint_qr[r] != cr) {
      if (tie_r) {
        ++ties;
        cr = hint_qr[r];
      } else {
        ++mism;
      }
    }
    qv[r] = (uint16_t)cv;
    qr[r] = (uint16_t)cr;
  }
  if (counts) {
    counts->q10_ties += ties;
    counts->q10_mismatch += mism;
    counts->hit_ties += hties;
    counts->shadow_ties += sties;
    counts->hit_mismatch += hmism;
    counts->shadow_mismatch += smism;
    counts->rays += (int64_t)P * 8;
  }
  (void)sh;
}

/* One sample into an interior irradiance texel ki and depth texel kd: the
 * moving average of Alg. MovingAvgUpdate (step max(1/(N+1), 1-h), N
 * saturating at 255), radiance into the irradiance texel and the first two
 * moments of the normalised distance into the depth texel (Sec. 4.6). */
static void blend_sample(double* irr, uint8_t* irr_n, double* dep, uint8_t* dep_n, int32_t ki, int32_t kd,
                         const double rgb[3], double tau, double hyst) {
  double ai = orc_blend_alpha(irr_n[ki], hyst);
  for (int c = 0; c < 3; ++c) irr[3 * ki + c] += ai * (rgb[c] - irr[3 * ki + c]);
  if (irr_n[ki] < 255) irr_n[ki]++;
  double ad = orc_blend_alpha(dep_n[kd], hyst);
  dep[2 * kd + 0] += ad * (tau - dep[2 * kd + 0]);
  dep[2 * kd + 1] += ad * (tau * tau - dep[2 * kd + 1]);
  if (dep_n[kd] < 255) dep_n[kd]++;
}

/* The octahedral bin of d at resolution r, adopting the hint where the
 * direction lies on a cell edge (a tie). */
static int32_t hinted_bin(const double d[3], int32_t r, const orc_tol* tol, const uint16_t* hint,
                          orc_counts* cnt) {
  int32_t tie = 0;
  int32_t k = orc_oct_bin(d, r, tol ? tol->bin_eps : 0.0, &tie);
  if (hint && *hint != k) {
    if (tie && *hint < r * r) {
      cnt->bin_ties++;
      k = *hint;
    } else {
      cnt->bin_mismatch++;
    }
  }
  return k;
}

void orc_pilot_blend(const orc_grid* g, uint64_t seed, int32_t frame, int32_t count, const int32_t* probes,
                     const orc_tol* tol, int32_t irr_r, int32_t dep_r, double hysteresis, double tau_max,
                     const double* prgb, const double* pt, const uint16_t* hint_ibin,
                     const uint16_t* hint_dbin, double* irr, uint8_t* irr_n, double* dep, uint8_t* dep_n,
                     orc_counts* counts) {
  const int32_t ri = irr_r - 2, rd = dep_r - 2, pair = frame / 2;
  orc_counts local;
  memset(&local, 0, sizeof(local));
  for (int32_t q = 0; q < count; ++q) {
    const int32_t i = probes[q];
    for (int32_t k = 0; k < 8; ++k) {
      const int64_t r = (int64_t)i * 8 + k;
      double d[3];
      orc_pilot_dir(seed, i, k, pair, d);
      const int32_t ki = hinted_bin(d, ri, tol, hint_ibin ? hint_ibin + r : NULL, &local);
      const int32_t kd = hinted_bin(d, rd, tol, hint_dbin ? hint_dbin + r : NULL, &local);
      const double tau = isfinite(pt[r]) ? fmin(pt[r] / g->s, tau_max) : tau_max;
      blend_sample(irr + (int64_t)q * ri * ri * 3, irr_n + (int64_t)q * ri * ri, dep + (int64_t)q * rd * rd * 2,
                   dep_n + (int64_t)q * rd * rd, ki, kd, prgb + 3 * r, tau, hysteresis);
    }
  }
  if (counts) {
    counts->bin_ties += local.bin_ties;
    counts->bin_mismatch += local.bin_mismatch;
  }
}

/* Change detection, second frame of each pair (Sec. 4.1.4, 4.1.5, 4.4):
 * temporal gradient d = |Q_t - Q_{t-1}| of the same pilot direction;
 * temporal trigger T <- max(d, T - ceil(1023/theta)) (a pulse that decays
 * linearly over theta detection steps); unnormalised 5x5x5 spatial sum C with
 * zero padding; and the per-probe score sum_k Qv (Cv + mu Cr), the dynamic
 * composition f_v (f_dv + mu f_dr) of eq. priorDynamic with f_c = 1, summed
 * over the probe's eight octants. First frame of a pair: keep the codes. */
void orc_detect(const orc_grid* g, int32_t frame, int32_t theta, int32_t mu, const uint16_t* qv,
                const uint16_t* qr, uint16_t* qv_prev, uint16_t* qr_prev, int32_t* tv, int32_t* tr,
                int64_t* score) {
  int32_t dx = g->dims[0], dy = g->dims[1], dz = g->dims[2];
  int64_t P = (int64_t)dx * dy * dz;
  if ((frame & 1) == 0) {
    memcpy(qv_prev, qv, sizeof(uint16_t) * P * 8);
    memcpy(qr_prev, qr, sizeof(uint16_t) * P * 8);
    if (frame == 0)
      for (int64_t i = 0; i < P; ++i) score[i] = 0;
    return;
  }
  int32_t delta = (1023 + theta - 1) / theta;
  for (int64_t r = 0; r < P * 8; ++r) {
    int32_t a = abs((int32_t)qv[r] - (int32_t)qv_prev[r]);
    int32_t b = abs((int32_t)qr[r] - (int32_t)qr_prev[r]);
    int32_t va = tv[r] - delta, vb = tr[r] - delta;
    tv[r] = a > va ? a : va;
    tr[r] = b > vb ? b : vb;
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < P; ++i) {
    int32_t x = (int32_t)(i % dx), y = (int32_t)((i / dx) % dy), z = (int32_t)(i / ((int64_t)dx * dy));
    int64_t s = 0;
    for (int32_t k = 0; k < 8; ++k) {
      int64_t cv = 0, cr = 0;
      for (int32_t zz = z - 2; zz <= z + 2; ++zz)
        for (int32_t yy = y - 2; yy <= y + 2; ++yy)
          for (int32_t xx = x - 2; xx <= x + 2; ++xx) {
            if (xx < 0 || yy < 0 || zz < 0 || xx >= dx || yy >= dy || zz >= dz) continue;
            int64_t j = xx + (int64_t)dx * (yy + (int64_t)dy * zz);
            cv += tv[j * 8 + k];
            cr += tr[j * 8 + k];
          }
      s += (int64_t)qv[i * 8 + k] * (cv + (int64_t)mu * cr);
    }
    score[i] = s;
  }
}

/* ------------------------------------------------------------ allocation */

static uint64_t alloc_e(uint64_t lambda, uint64_t w, uint64_t E) {
  uint64_t e = (lambda * w) >> 32;
  return e < E ? e : E;
}

/* Integer ray-budget allocation: the per-probe share of a user-set total
 * budget (the paper fixes the sample count per frame by the number of chains,
 * Sec. 3.3, and lets the guide decide where samples go). Scores are shifted
 * so the largest lies in [2^31, 2^32); lambda* is the largest integer in
 * [0, 2^31] whose proportional extras fit the remaining budget; the rest goes
 * one ray each to the lowest-index probes that the next lambda would raise. */
int32_t orc_allocate(int32_t P, const int64_t* score, int64_t budget, int32_t n_min, int32_t n_max,
                     int32_t* n, int64_t* offsets, uint32_t* lambda_out) {
  if (n_min < 1 || n_max < n_min || budget < (int64_t)P * n_min) return -1;
  int64_t Bp = budget - (int64_t)P * n_min;
  uint64_t E = (uint64_t)(n_max - n_min);
  uint64_t* w = (uint64_t*)malloc(sizeof(uint64_t) * (P > 0 ? P : 1));
  int64_t mx = 0;
  for (int32_t i = 0; i < P; ++i) mx = score[i] > mx ? score[i] : mx;
  if (mx == 0) {
    for (int32_t i = 0; i < P; ++i) w[i] = 1ull << 31;
  } else {
    int bits = 0;
    while (bits < 63 && (mx >> bits) != 0) ++bits;
    for (int32_t i = 0; i < P; ++i) {
      uint64_t s = (uint64_t)score[i];
      w[i] = bits <= 32 ? (s << (32 - bits)) : (s >> (bits - 32));
    }
  }
  /* largest lambda with sum e(lambda) <= B' (the sum is monotone in lambda) */
  uint64_t lo = 0, hi = (1ull << 31);
  {
    int64_t sum = 0;
    for (int32_t i = 0; i < P; ++i) sum += (int64_t)alloc_e(hi, w[i], E);
    if (sum <= Bp) lo = hi;
  }
  while (lo < hi) {
    uint64_t mid = lo + (hi - lo + 1) / 2;
    int64_t sum = 0;
    for (int32_t i = 0; i < P; ++i) sum += (int64_t)alloc_e(mid, w[i], E);
    if (sum <= Bp) lo = mid;
    else hi = mid - 1;
  }
  uint64_t lam = lo;
  int64_t used = 0;
  for (int32_t i = 0; i < P; ++i) used += (int64_t)alloc_e(lam, w[i], E);
  int64_t R = Bp - used;
  int64_t off = 0;
  for (int32_t i = 0; i < P; ++i) {
    uint64_t e0 = alloc_e(lam, w[i], E), e1 = alloc_e(lam + 1, w[i], E);
    int32_t bonus = 0;
    if (R > 0 && e1 > e0) {
      bonus = 1;
      --R;
    }
    n[i] = n_min + (int32_t)e0 + bonus;
    if (offsets) offsets[i] = off;
    off += n[i];
  }
  if (offsets) offsets[P] = off;
  if (lambda_out) *lambda_out = (uint32_t)lam;
  free(w);
  return 0;
}

/* ------------------------------------------------------------------ blend */

/* Alg. MovingAvgUpdate: V <- v/(n+1) + n*o/(n+1), i.e. V <- o + (v-o)/(n+1),
 * with the count saturating. Tab. cacheDetails pairs N_max with a hysteresis
 * of N_max/(N_max+1); here N_max is real, N_max = h/(1-h), so the step is
 * max(1/(n+1), 1-h): an exact running mean until 1/(n+1) < 1-h, then an
 * exponential moving average with hysteresis h. */
double orc_blend_alpha(int32_t n, double hysteresis) {
  double a = 1.0 / (double)(n + 1);
  double b = 1.0 - hysteresis;
  return a > b ? a : b;
}

/* binary16 round-to-nearest-even of a double, direct (no double rounding). */
double orc_round_half(double x) {
  if (x == 0.0 || !isfinite(x)) return x;
  double a = fabs(x);
  if (a >= 65520.0) return copysign(INFINITY, x);
  int e;
  frexp(a, &e);                 /* a = m * 2^e, m in [0.5, 1): leading bit 2^(e-1) */
  int lead = e - 1;
  int qexp = lead < -14 ? -24 : lead - 10;
  double q = ldexp(1.0, qexp);
  double r = nearbyint(a / q) * q;
  return copysign(r, x);
}

/* DDGI's depth weight sharpness (the cosine raised to this power) */
#define ORC_GATHER_DEPTH_POWER 50

static void probe_frame_one(const orc_scene* s, const orc_grid* g, int32_t probe, int32_t n,
                            const float R[9], const orc_tol* tol, int32_t irr_r, int32_t dep_r,
                            double hyst, double tau_max, int32_t fp16, int32_t gather, const int32_t* hint_tri,
                            const uint8_t* hint_shadow, const uint16_t* hint_ibin,
                            const uint16_t* hint_dbin, double* irr, uint8_t* irr_n, double* dep,
                            uint8_t* dep_n, double* rays, int32_t* tri, uint8_t* shadow,
                            uint16_t* ibin, uint16_t* dbin, orc_counts* cnt) {
  double o[3];
  orc_probe_pos(g, probe, o);
  int32_t ri = irr_r - 2, rd = dep_r - 2;
  int64_t ties[2] = {0, 0}, mism[2] = {0, 0};
  /* gather: per texel the sums of w, w rgb (irradiance) and w, w tau, w tau^2
   * (depth) over the frame's rays */
  double* gi = NULL;
  double* gd = NULL;
  if (gather) {
    gi = (double*)calloc((size_t)ri * ri * 4, sizeof(double));
    gd = (double*)calloc((size_t)rd * rd * 3, sizeof(double));
  }
  for (int32_t j = 0; j < n; ++j) {
    double d[3];
    orc_sf_dir(orc_ray_point(j, n), n, R, d);
    orc_ray ray;
    orc_shade_ray(s, o, d, g->s, tol, hint_tri ? hint_tri[j] : -2,
                  hint_shadow ? (int32_t)hint_shadow[j] : -1, &ray, ties, mism);
    cnt->rays += 1;
    if (ray.tri >= 0 && ray.front) cnt->shadow_rays += s->nl;
    int32_t ti = 0, td = 0;
    int32_t ki = orc_oct_bin(d, ri, tol ? tol->bin_eps : 0.0, &ti);
    int32_t kd = orc_oct_bin(d, rd, tol ? tol->bin_eps : 0.0, &td);
    if (hint_ibin && hint_ibin[j] != ki) {
      if (ti && hint_ibin[j] < ri * ri) {
        cnt->bin_ties++;
        ki = hint_ibin[j];
      } else {
        cnt->bin_mismatch++;
      }
    }
    if (hint_dbin && hint_dbin[j] != kd) {
      if (td && hint_dbin[j] < rd * rd) {
        cnt->bin_ties++;
        kd = hint_dbin[j];
      } else {
        cnt->bin_mismatch++;
      }
    }
    double tau = isfinite(ray.t) ? fmin(ray.t / g->s, tau_max) : tau_max;
    if (gather) {
      /* every texel takes the ray, weighted by the cosine to its centre
       * direction (irradiance) or that cosine to the 50th power (depth) */
      for (int32_t k = 0; k < ri * ri; ++k) {
        double c[3];
        orc_texel_centre_dir(ri, k, c);
        const double w = fmax(0.0, c[0] * d[0] + c[1] * d[1] + c[2] * d[2]);
        gi[4 * k] += w;
        for (int a = 0; a < 3; ++a) gi[4 * k + 1 + a] += w * ray.rgb[a];
      }
      for (int32_t k = 0; k < rd * rd; ++k) {
        double c[3];
        orc_texel_centre_dir(rd, k, c);
        const double w = pow(fmax(0.0, c[0] * d[0] + c[1] * d[1] + c[2] * d[2]), ORC_GATHER_DEPTH_POWER);
        gd[3 * k] += w;
        gd[3 * k + 1] += w * tau;
        gd[3 * k + 2] += w * tau * tau;
      }
    } else {
      blend_sample(irr, irr_n, dep, dep_n, ki, kd, ray.rgb, tau, hyst);
    }
    if (rays) {
      rays[4 * j + 0] = ray.rgb[0];
      rays[4 * j + 1] = ray.rgb[1];
      rays[4 * j + 2] = ray.rgb[2];
      rays[4 * j + 3] = ray.t;
    }
    if (tri) tri[j] = ray.tri;
    if (shadow) shadow[j] = ray.shadow;
    if (ibin) ibin[j] = (uint16_t)ki;
    if (dbin) dbin[j] = (uint16_t)kd;
  }
  if (gather) {
    /* the frame's weighted mean, blended with the step rule of the per-sample
     * update counted in frames: a = max(1/(N+1), 1-h) */
    for (int32_t k = 0; k < ri * ri; ++k) {
      if (!(gi[4 * k] > 0.0)) continue;
      const double a = orc_blend_alpha(irr_n[k], hyst);
      for (int c = 0; c < 3; ++c) irr[3 * k + c] += a * (gi[4 * k + 1 + c] / gi[4 * k] - irr[3 * k + c]);
      if (irr_n[k] < 255) irr_n[k]++;
    }
    for (int32_t k = 0; k < rd * rd; ++k) {
      if (!(gd[3 * k] > 0.0)) continue;
      const double a = orc_blend_alpha(dep_n[k], hyst);
      dep[2 * k + 0] += a * (gd[3 * k + 1] / gd[3 * k] - dep[2 * k + 0]);
      dep[2 * k + 1] += a * (gd[3 * k + 2] / gd[3 * k] - dep[2 * k + 1]);
      if (dep_n[k] < 255) dep_n[k]++;
    }
    free(gi);
    free(gd);
  }
  if (fp16) {
    for (int32_t k = 0; k < ri * ri * 3; ++k) irr[k] = orc_round_half(irr[k]);
    for (int32_t k = 0; k < rd * rd * 2; ++k) dep[k] = orc_round_half(dep[k]);
  }
  cnt->hit_ties += ties[0];
  cnt->shadow_ties += ties[1];
  cnt->hit_mismatch += mism[0];
  cnt->shadow_mismatch += mism[1];
}

void orc_probe_frame(const orc_scene* s, const orc_grid* g, int32_t probe, int32_t n,
                     const float R[9], const orc_tol* tol, int32_t irr_r, int32_t dep_r,
                     double hysteresis, double tau_max, int32_t fp16, const int32_t* hint_tri,
                     const uint8_t* hint_shadow, const uint16_t* hint_ibin,
                     const uint16_t* hint_dbin, double* irr, uint8_t* irr_n, double* dep,
                     uint8_t* dep_n, double* rays, int32_t* tri, uint8_t* shadow, uint16_t* ibin,
                     uint16_t* dbin, orc_counts* counts) {
  probe_frame_one(s, g, probe, n, R, tol, irr_r, dep_r, hysteresis, tau_max, fp16, 0, hint_tri,
                  hint_shadow, hint_ibin, hint_dbin, irr, irr_n, dep, dep_n, rays, tri, shadow,
                  ibin, dbin, counts);
}

void orc_probes_frame(const orc_scene* s, const orc_grid* g, int32_t count, const int32_t* probes,
                      const int32_t* n, const int64_t* ray_base, const float R[9], const orc_tol* tol,
                      int32_t irr_r, int32_t dep_r, double hysteresis, double tau_max, int32_t fp16,
                      int32_t gather, const int32_t* hint_tri, const uint8_t* hint_shadow,
                      const uint16_t* hint_ibin, const uint16_t* hint_dbin, double* irr,
                      uint8_t* irr_n, double* dep, uint8_t* dep_n, double* rays, int32_t* tri,
                      uint8_t* shadow, uint16_t* ibin, uint16_t* dbin, orc_counts* counts) {
  int32_t ri = irr_r - 2, rd = dep_r - 2;
  orc_counts total;
  memset(&total, 0, sizeof(total));
#pragma omp parallel
  {
    orc_counts local;
    memset(&local, 0, sizeof(local));
#pragma omp for schedule(dynamic, 1)
    for (int32_t q = 0; q < count; ++q) {
      int64_t b = ray_base[q];
      probe_frame_one(s, g, probes[q], n[q], R, tol, irr_r, dep_r, hysteresis, tau_max, fp16, gather,
                      hint_tri ? hint_tri + b : NULL, hint_shadow ? hint_shadow + b : NULL,
                      hint_ibin ? hint_ibin + b : NULL, hint_dbin ? hint_dbin + b : NULL,
                      irr + (int64_t)q * ri * ri * 3, irr_n + (int64_t)q * ri * ri,
                      dep + (int64_t)q * rd * rd * 2, dep_n + (int64_t)q * rd * rd,
                      rays ? rays + 4 * b : NULL, tri ? tri + b : NULL, shadow ? shadow + b : NULL,
                      ibin ? ibin + b : NULL, dbin ? dbin + b : NULL, &local);
    }
#pragma omp critical
    {
      total.hit_ties += local.hit_ties;
      total.shadow_ties += local.shadow_ties;
      total.bin_ties += local.bin_ties;
      total.q10_ties += local.q10_ties;
      total.hit_mismatch += local.hit_mismatch;
      total.shadow_mismatch += local.shadow_mismatch;
      total.bin_mismatch += local.bin_mismatch;
      total.q10_mismatch += local.q10_mismatch;
      total.rays += local.rays;
      total.shadow_rays += local.shadow_rays;
    }
  }
  if (counts) {
    counts->hit_ties += total.hit_ties;
    counts->shadow_ties += total.shadow_ties;
    counts->bin_ties += total.bin_ties;
    counts->q10_ties += total.q10_ties;
    counts->hit_mismatch += total.hit_mismatch;
    counts->shadow_mismatch += total.shadow_mismatch;
    counts->bin_mismatch += total.bin_mismatch;
    counts->q10_mismatch += total.q10_mismatch;
    counts->rays += total.rays;
    counts->shadow_rays += total.shadow_rays;
  }
}

/* ------------------------------------------------------- packed texels */

/* eq. rgbEnc, one channel: the code of a binary32 value v >= 0 is
 * floor(qmax min(ln(gamma v + 1), beta) / beta), qmax = 2^bits - 1 (rounded
 * down, App. B). Evaluated in FP64: gamma v is exact there, log1p and the
 * scaling round at about 1e-16 relative, and no binary32 input lies closer
 * than that to a code boundary (checked at every boundary of the four
 * channel types against 50-digit arithmetic), so the floor is the exact
 * one. */
uint32_t orc_pack_encode(float v, float beta, float gamma, int32_t bits) {
  const double qmax = (double)((1u << bits) - 1u);
  const double x = v > 0.0f ? (double)v : 0.0;
  const double u = fmin(log1p((double)gamma * x), (double)beta) / (double)beta;
  const double q = floor(u * qmax);
  return q >= qmax ? (uint32_t)qmax : (uint32_t)q;
}

/* The value code q stands for, (e^(beta q / qmax) - 1) / gamma, in FP64 and
 * rounded once to binary32. */
float orc_pack_decode(uint32_t q, float beta, float gamma, int32_t bits) {
  const double qmax = (double)((1u << bits) - 1u);
  return (float)(expm1((double)beta * ((double)q / qmax)) / (double)gamma);
}

void orc_packed_blend(int32_t count, const int32_t* n, const int64_t* ray_base, const float* rec,
                      const uint16_t* ibin, const uint16_t* dbin, int32_t ri, int32_t rd, float inv_s,
                      float tau_max, const float* alpha, uint32_t* irr, uint32_t* dep) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int32_t q = 0; q < count; ++q) {
    uint32_t* wi = irr + (size_t)q * ri * ri;
    uint32_t* wd = dep + (size_t)q * rd * rd;
    for (int32_t j = 0; j < n[q]; ++j) {
      const int64_t r = ray_base[q] + j;
      const float* x = rec + 4 * r;
      /* irradiance texel: (R, G, B) */
      uint32_t w = wi[ibin[r]];
      uint32_t N = w >> 26;
      float al = alpha[N];
      uint32_t c0 = w & 0x1FFu, c1 = (w >> 9) & 0x1FFu, c2 = (w >> 18) & 0xFFu;
      float o0 = orc_pack_decode(c0, 5.0f, 15.0f, 9);
      float o1 = orc_pack_decode(c1, 5.0f, 15.0f, 9);
      float o2 = orc_pack_decode(c2, 5.0f, 15.0f, 8);
      c0 = orc_pack_encode(fmaf(al, x[0] - o0, o0), 5.0f, 15.0f, 9);
      c1 = orc_pack_encode(fmaf(al, x[1] - o1, o1), 5.0f, 15.0f, 9);
      c2 = orc_pack_encode(fmaf(al, x[2] - o2, o2), 5.0f, 15.0f, 8);
      N = N < 63u ? N + 1u : 63u;
      wi[ibin[r]] = c0 | (c1 << 9) | (c2 << 18) | (N << 26);
      /* depth texel: (tau, tau^2) */
      w = wd[dbin[r]];
      N = w >> 26;
      al = alpha[N];
      uint32_t d0 = w & 0x1FFFu, d1 = (w >> 13) & 0x1FFFu;
      float tau = fminf(x[3] * inv_s, tau_max);
      float p0 = orc_pack_decode(d0, 5.0f, 15.0f, 13);
      float p1 = orc_pack_decode(d1, 8.0f, 20.0f, 13);
      d0 = orc_pack_encode(fmaf(al, tau - p0, p0), 5.0f, 15.0f, 13);
      d1 = orc_pack_encode(fmaf(al, tau * tau - p1, p1), 8.0f, 20.0f, 13);
      N = N < 63u ? N + 1u : 63u;
      wd[dbin[r]] = d0 | (d1 << 13) | (N << 26);
    }
  }
}

/* ------------------------------------------------ Metropolis chains */

static int near_frac(double f, double band) {
  double r = f - floor(f);
  return r < band || r > 1.0 - band;
}

void orc_chain_dir(const double uv[2], double d[3]) { orc_oct_decode(uv, d); }

/* p within the box of probe centres, uv within [-1, 1]^2 (closed). An axis
 * with a single probe has no extent: the chain sits at its one coordinate and
 * never moves along it, so no boundary decision is taken there. */
static int chain_in_domain(const orc_grid* g, const double x[5], int* tie) {
  int in = 1, t = 0;
  for (int a = 0; a < 3; ++a) {
    double lo = g->origin[a], hi = g->origin[a] + (g->dims[a] - 1) * g->spacing[a];
    double band = 1e-6 * g->spacing[a] + 1e-7 * fabs(x[a]);
    if (x[a] < lo || x[a] > hi) in = 0;
    if (g->dims[a] > 1 && (fabs(x[a] - lo) <= band || fabs(x[a] - hi) <= band)) t = 1;
  }
  for (int a = 3; a < 5; ++a) {
    if (x[a] < -1.0 || x[a] > 1.0) in = 0;
    if (fabs(fabs(x[a]) - 1.0) <= 1e-6) t = 1;
  }
  if (tie) *tie = t;
  return in;
}

double orc_chain_h(const orc_grid* g, const uint16_t* qv, const double* irr_prev, int32_t r,
                   const double x[5], int32_t* probe, int32_t* tie) {
  int t = 0;
  int32_t idx[3];
  for (int a = 0; a < 3; ++a) {
    double f = g->dims[a] > 1 ? (x[a] - g->origin[a]) / g->spacing[a] : 0.0;
    int32_t i = (int32_t)floor(f + 0.5);
    if (i < 0) i = 0;
    if (i > g->dims[a] - 1) i = g->dims[a] - 1;
    idx[a] = i;
    if (g->dims[a] > 1 && near_frac(f + 0.5, 1e-5)) t = 1;
  }
  int32_t pr = idx[0] + g->dims[0] * (idx[1] + g->dims[1] * idx[2]);
  if (probe) *probe = pr;
  double d[3];
  orc_oct_decode(x + 3, d);
  int32_t k = (d[0] < 0.0 ? 1 : 0) | (d[1] < 0.0 ? 2 : 0) | (d[2] < 0.0 ? 4 : 0);
  for (int a = 0; a < 3; ++a)
    if (fabs(d[a]) < 1e-6) t = 1;
  double f = (double)qv[8 * pr + k] / 1024.0;
  if (f <= 0.0) {
    if (tie) *tie = t;
    return 0.0;
  }
  /* the texel one level coarser (2x2 interior texels) that holds uv */
  int32_t m = r / 2, cell[2];
  for (int a = 0; a < 2; ++a) {
    double c = (x[3 + a] + 1.0) * 0.5 * m;
    int32_t ci = (int32_t)floor(c);
    if (ci > m - 1) ci = m - 1;
    if (ci < 0) ci = 0;
    cell[a] = ci;
    if (near_frac(c, 1e-5) && c > 1e-5 && c < m - 1e-5) t = 1;
  }
  double rgb[3] = {0.0, 0.0, 0.0};
  for (int b = 0; b < 2; ++b)
    for (int a = 0; a < 2; ++a) {
      const double* T = irr_prev + 3 * ((size_t)pr * r * r + (size_t)(2 * cell[1] + b) * r + 2 * cell[0] + a);
      for (int ch = 0; ch < 3; ++ch) rgb[ch] += T[ch];
    }
  double lum = 0.2126 * (rgb[0] / 4.0) + 0.7152 * (rgb[1] / 4.0) + 0.0722 * (rgb[2] / 4.0);
  if (tie) *tie = t;
  return exp(fmin(lum / f, 1.0)) * f;
}

/* The chain loop of Alg. MarkovChainMT with the random-walk step of Alg.
 * MetropolisStep, for any target: h(x) returns the density and the discrete
 * cell the state falls in (the nearest probe for the static target, proxy
 * and octant for the dynamic one); emit(s, cell, h, x) receives the state
 * after every step past the burn-in. */
typedef double (*chain_target)(const void* ctx, const double x[5], int32_t* cell, int32_t* tie);
typedef void (*chain_emit)(void* ctx, int64_t s, int32_t cell, double h, const double x[5]);

static void chain_run(const orc_grid* g, const orc_chain_params* cp, uint64_t seed, uint64_t tag_step,
                      uint64_t tag_init, int32_t frame, chain_target target, const void* tctx, double* state,
                      int32_t init, const uint8_t* hint_accept, uint8_t* accept, chain_emit emit, void* ectx,
                      orc_counts* counts) {
  const int32_t C = cp->chains, M = cp->steps, K = cp->burn_in;
  const int32_t S = M - K - 1 > 0 ? M - K - 1 : 0;
  int64_t ties = 0, mism = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : ties, mism)
  for (int32_t c = 0; c < C; ++c) {
    double* x = state + 5 * (size_t)c;
    if (init) {
      uint64_t key = orc_key(seed, tag_init, (uint64_t)(uint32_t)c, 0, 0);
      for (int a = 0; a < 3; ++a)
        x[a] = g->origin[a] + orc_uniform(key, (uint64_t)(a + 1)) * (g->dims[a] - 1) * g->spacing[a];
      x[3] = 2.0 * orc_uniform(key, 4) - 1.0;
      x[4] = 2.0 * orc_uniform(key, 5) - 1.0;
    }
    int32_t cell = 0;
    int tie_y = 0, dtie = 0;
    double y = 0.0;
    if (chain_in_domain(g, x, &dtie)) y = target(tctx, x, &cell, &tie_y);
    tie_y |= dtie;
    for (int32_t i = 0; i < M; ++i) {
      uint64_t key = orc_key(seed, tag_step, (uint64_t)(uint32_t)c, (uint64_t)(uint32_t)frame,
                             (uint64_t)(uint32_t)i);
      double u[8];
      for (int q = 1; q <= 7; ++q) u[q] = orc_uniform(key, (uint64_t)q);
      double gs[6];
      for (int q = 0; q < 3; ++q) {
        double rr = sqrt(-2.0 * log(1.0 - u[2 * q + 1]));
        double th = 2.0 * PI * u[2 * q + 2];
        gs[2 * q] = rr * cos(th);
        gs[2 * q + 1] = rr * sin(th);
      }
      double xp[5];
      for (int a = 0; a < 3; ++a)
        xp[a] = g->dims[a] > 1 ? x[a] + cp->sigma_pos * g->spacing[a] * gs[a] : x[a];
      xp[3] = x[3] + cp->sigma_dir * gs[3];
      xp[4] = x[4] + cp->sigma_dir * gs[4];
      int ptie = 0, ttie = 0;
      int in = chain_in_domain(g, xp, &ttie);
      double yp = 0.0;
      int32_t cellp = cell;
      if (in) yp = target(tctx, xp, &cellp, &ptie);
      ptie |= ttie;
      int acc = in && (y <= 0.0 || u[7] * y <= yp);
      int tie = ptie || tie_y || (in && y > 0.0 && fabs(u[7] * y - yp) <= 1e-4 * fmax(yp, u[7] * y)) ||
                (in && y > 0.0 && y <= 1e-12);
      if (hint_accept) {
        int gd = hint_accept[(size_t)c * M + i] != 0;
        if (gd != acc) {
          if (tie) {
            ++ties;
            acc = gd;
            if (acc && !in) acc = 0;  /* never leave the domain */
          } else {
            ++mism;
          }
        }
      }
      if (acc) {
        for (int a = 0; a < 5; ++a) x[a] = xp[a];
        y = yp;
        cell = cellp;
        tie_y = ptie;
      }
      if (accept) accept[(size_t)c * M + i] = (uint8_t)acc;
      if (i > K) emit(ectx, (int64_t)c * S + (i - K - 1), cell, y, x);
    }
  }
  if (counts) {
    counts->chain_ties += ties;
    counts->chain_mismatch += mism;
  }
}

typedef struct {
  const orc_grid* g;
  const uint16_t* qv;
  const double* irr_prev;
  int32_t r;
} static_target_ctx;

static double static_target(const void* ctx, const double x[5], int32_t* cell, int32_t* tie) {
  const static_target_ctx* t = (const static_target_ctx*)ctx;
  return orc_chain_h(t->g, t->qv, t->irr_prev, t->r, x, cell, tie);
}

typedef struct {
  int32_t* sample_probe;
  double* sample_uv;
} static_emit_ctx;

static void static_emit(void* ctx, int64_t s, int32_t cell, double h, const double x[5]) {
  (void)h;
  static_emit_ctx* e = (static_emit_ctx*)ctx;
  if (e->sample_probe) e->sample_probe[s] = cell;
  if (e->sample_uv) {
    e->sample_uv[2 * s] = x[3];
    e->sample_uv[2 * s + 1] = x[4];
  }
}

void orc_chain_frame(const orc_grid* g, const orc_chain_params* cp, uint64_t seed, int32_t frame,
                     const uint16_t* qv, const double* irr_prev, int32_t r, double* state, int32_t init,
                     const uint8_t* hint_accept, uint8_t* accept, int32_t* sample_probe,
                     double* sample_uv, orc_counts* counts) {
  static_target_ctx t = {g, qv, irr_prev, r};
  static_emit_ctx e = {sample_probe, sample_uv};
  chain_run(g, cp, seed, ORC_TAG_CHAIN, ORC_TAG_CHAININIT, frame, static_target, &t, state, init, hint_accept,
            accept, static_emit, &e, counts);
}

/* ---------------------------------------------------- dynamic chains (Sec. 4.9) */

void orc_dynamic_fd(const orc_grid* g, int32_t mu, const uint16_t* qv, const int32_t* tv, const int32_t* tr,
                    int64_t* fd) {
  const int32_t dx = g->dims[0], dy = g->dims[1], dz = g->dims[2];
  const int64_t P = (int64_t)dx * dy * dz;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < P; ++i) {
    int32_t x = (int32_t)(i % dx), y = (int32_t)((i / dx) % dy), z = (int32_t)(i / ((int64_t)dx * dy));
    for (int32_t k = 0; k < 8; ++k) {
      int64_t cv = 0, cr = 0;
      for (int32_t zz = z - 2; zz <= z + 2; ++zz)
        for (int32_t yy = y - 2; yy <= y + 2; ++yy)
          for (int32_t xx = x - 2; xx <= x + 2; ++xx) {
            if (xx < 0 || yy < 0 || zz < 0 || xx >= dx || yy >= dy || zz >= dz) continue;
            int64_t j = xx + (int64_t)dx * (yy + (int64_t)dy * zz);
            cv += tv[j * 8 + k];
            cr += tr[j * 8 + k];
          }
      fd[i * 8 + k] = (int64_t)qv[i * 8 + k] * (cv + (int64_t)mu * cr);
    }
  }
}

void orc_proxy_dims(const orc_grid* g, int32_t pd[3]) {
  for (int a = 0; a < 3; ++a) pd[a] = (g->dims[a] + 2) / 3;
}

int32_t orc_proxy_of_probe(const orc_grid* g, int32_t probe) {
  int32_t pd[3];
  orc_proxy_dims(g, pd);
  const int32_t dx = g->dims[0], dy = g->dims[1];
  const int32_t x = probe % dx, y = (probe / dx) % dy, z = probe / (dx * dy);
  return x / 3 + pd[0] * (y / 3 + pd[1] * (z / 3));
}

void orc_proxy_max(const orc_grid* g, const int64_t* fd, int64_t* F) {
  int32_t pd[3];
  orc_proxy_dims(g, pd);
  const int64_t Pp = (int64_t)pd[0] * pd[1] * pd[2];
  for (int64_t q = 0; q < Pp * 8; ++q) F[q] = 0;
  const int64_t P = (int64_t)g->dims[0] * g->dims[1] * g->dims[2];
  for (int64_t i = 0; i < P; ++i) {
    const int64_t q = orc_proxy_of_probe(g, (int32_t)i);
    for (int k = 0; k < 8; ++k)
      if (fd[i * 8 + k] > F[q * 8 + k]) F[q * 8 + k] = fd[i * 8 + k];
  }
}

typedef struct {
  const orc_grid* g;
  const int64_t* F;
} dyn_target_ctx;

/* h = F of the proxy of the nearest probe, in the octant of uv (alpha = 0:
 * the stored irradiance plays no part). */
static double dyn_target(const void* ctx, const double x[5], int32_t* cell, int32_t* tie) {
  const dyn_target_ctx* t = (const dyn_target_ctx*)ctx;
  const orc_grid* g = t->g;
  int tt = 0;
  int32_t idx[3];
  for (int a = 0; a < 3; ++a) {
    double f = g->dims[a] > 1 ? (x[a] - g->origin[a]) / g->spacing[a] : 0.0;
    int32_t i = (int32_t)floor(f + 0.5);
    if (i < 0) i = 0;
    if (i > g->dims[a] - 1) i = g->dims[a] - 1;
    idx[a] = i;
    if (g->dims[a] > 1 && near_frac(f + 0.5, 1e-5)) tt = 1;
  }
  const int32_t pr = idx[0] + g->dims[0] * (idx[1] + g->dims[1] * idx[2]);
  double d[3];
  orc_oct_decode(x + 3, d);
  const int32_t k = (d[0] < 0.0 ? 1 : 0) | (d[1] < 0.0 ? 2 : 0) | (d[2] < 0.0 ? 4 : 0);
  for (int a = 0; a < 3; ++a)
    if (fabs(d[a]) < 1e-6) tt = 1;
  const int32_t q = orc_proxy_of_probe(g, pr);
  *cell = q * 8 + k;
  if (tie) *tie = tt;
  return (double)t->F[q * 8 + k];
}

static void dyn_emit(void* ctx, int64_t s, int32_t cell, double h, const double x[5]) {
  (void)s;
  (void)x;
  uint8_t* mark = (uint8_t*)ctx;
  if (h > 0.0) {
#pragma omp atomic write
    mark[cell] = 1;
  }
}

void orc_dyn_chain_frame(const orc_grid* g, const orc_chain_params* cp, uint64_t seed, int32_t frame,
                         const int64_t* F, double* state, int32_t init, const uint8_t* hint_accept,
                         uint8_t* accept, uint8_t* mark, orc_counts* counts) {
  dyn_target_ctx t = {g, F};
  chain_run(g, cp, seed, ORC_TAG_DYNCHAIN, ORC_TAG_DYNCHAININIT, frame, dyn_target, &t, state, init,
            hint_accept, accept, dyn_emit, mark, counts);
}

int32_t orc_octant_texels(int32_t r, int32_t k, int32_t* list) {
  int32_t n = 0;
  for (int32_t y = 0; y < r; ++y)
    for (int32_t x = 0; x < r; ++x) {
      /* centre uv = ((2x+1)/r - 1, (2y+1)/r - 1), signs and the diagonal in integers */
      const int32_t cx = 2 * x + 1 - r, cy = 2 * y + 1 - r;
      const int32_t o = (cx < 0 ? 1 : 0) | (cy < 0 ? 2 : 0) | (abs(cx) + abs(cy) > r ? 4 : 0);
      if (o == k) {
        if (list) list[n] = y * r + x;
        ++n;
      }
    }
  return n;
}

void orc_texel_centre_dir(int32_t r, int32_t t, double d[3]) {
  const int32_t x = t % r, y = t / r;
  const double uv[2] = {(2.0 * x + 1.0) / r - 1.0, (2.0 * y + 1.0) / r - 1.0};
  orc_oct_decode(uv, d);
}

int32_t orc_dyn_ray_count(int32_t irr_r, int32_t dep_r, uint32_t octant_mask) {
  int32_t n = 0;
  for (int32_t k = 0; k < 8; ++k)
    if (octant_mask & (1u << k)) n += orc_octant_texels(irr_r - 2, k, NULL) + orc_octant_texels(dep_r - 2, k, NULL);
  return n;
}

void orc_dyn_probes_frame(const orc_scene* s, const orc_grid* g, int32_t count, const int32_t* probes,
                          const uint8_t* mark, const int64_t* ray_base, const orc_tol* tol, int32_t irr_r,
                          int32_t dep_r, double h_dyn, double tau_max, int32_t fp16, const int32_t* hint_tri,
                          const uint8_t* hint_shadow, double* irr, uint8_t* irr_n, double* dep, uint8_t* dep_n,
                          orc_counts* counts) {
  const int32_t ri = irr_r - 2, rd = dep_r - 2;
  int32_t li[8][34 * 34], ld[8][34 * 34], ni[8], nd[8];
  for (int32_t k = 0; k < 8; ++k) {
    ni[k] = orc_octant_texels(ri, k, li[k]);
    nd[k] = orc_octant_texels(rd, k, ld[k]);
  }
  orc_counts total;
  memset(&total, 0, sizeof(total));
#pragma omp parallel
  {
    orc_counts loc;
    memset(&loc, 0, sizeof(loc));
#pragma omp for schedule(dynamic, 4)
    for (int32_t q = 0; q < count; ++q) {
      double o[3];
      orc_probe_pos(g, probes[q], o);
      double* I = irr + (size_t)q * ri * ri * 3;
      double* D = dep + (size_t)q * rd * rd * 2;
      uint8_t* IN = irr_n + (size_t)q * ri * ri;
      uint8_t* DN = dep_n + (size_t)q * rd * rd;
      const int32_t px = orc_proxy_of_probe(g, probes[q]);
      int64_t ties[2] = {0, 0}, mism[2] = {0, 0};
      int64_t j = ray_base ? ray_base[q] : 0;
      for (int32_t k = 0; k < 8; ++k) {
        if (!mark[px * 8 + k]) continue;
        /* irradiance texels of the octant: one shaded ray through each centre */
        for (int32_t m = 0; m < ni[k]; ++m, ++j) {
          const int32_t t = li[k][m];
          double d[3];
          orc_texel_centre_dir(ri, t, d);
          orc_ray ra;
          orc_shade_ray(s, o, d, g->s, tol, hint_tri ? hint_tri[j] : -2,
                        hint_shadow ? (int32_t)hint_shadow[j] : -1, &ra, ties, mism);
          loc.rays += 1;
          if (ra.tri >= 0 && ra.front) loc.shadow_rays += s->nl;
          const double a = orc_blend_alpha(IN[t], h_dyn);
          for (int c = 0; c < 3; ++c) I[3 * t + c] += a * (ra.rgb[c] - I[3 * t + c]);
          if (IN[t] < 255) IN[t]++;
        }
        /* depth texels of the octant: the distance of a ray through each centre */
        for (int32_t m = 0; m < nd[k]; ++m, ++j) {
          const int32_t t = ld[k][m];
          double d[3];
          orc_texel_centre_dir(rd, t, d);
          orc_ray rb;
          orc_shade_ray(s, o, d, g->s, tol, hint_tri ? hint_tri[j] : -2, -1, &rb, ties, mism);
          loc.rays += 1;
          const double tau = isfinite(rb.t) ? fmin(rb.t / g->s, tau_max) : tau_max;
          const double a = orc_blend_alpha(DN[t], h_dyn);
          D[2 * t + 0] += a * (tau - D[2 * t + 0]);
          D[2 * t + 1] += a * (tau * tau - D[2 * t + 1]);
          if (DN[t] < 255) DN[t]++;
        }
      }
      if (fp16) { /* the frame's one binary16 store */
        for (int32_t k = 0; k < ri * ri * 3; ++k) I[k] = orc_round_half(I[k]);
        for (int32_t k = 0; k < rd * rd * 2; ++k) D[k] = orc_round_half(D[k]);
      }
      loc.hit_ties += ties[0];
      loc.shadow_ties += ties[1];
      loc.hit_mismatch += mism[0];
      loc.shadow_mismatch += mism[1];
    }
#pragma omp critical
    {
      total.hit_ties += loc.hit_ties;
      total.shadow_ties += loc.shadow_ties;
      total.hit_mismatch += loc.hit_mismatch;
      total.shadow_mismatch += loc.shadow_mismatch;
      total.rays += loc.rays;
      total.shadow_rays += loc.shadow_rays;
    }
  }
  if (counts) {
    counts->hit_ties += total.hit_ties;
    counts->shadow_ties += total.shadow_ties;
    counts->hit_mismatch += total.hit_mismatch;
    counts->shadow_mismatch += total.shadow_mismatch;
    counts->rays += total.rays;
    counts->shadow_rays += total.shadow_rays;
  }
}

void orc_chain_probes_frame(const orc_scene* s, const orc_grid* g, int32_t count, const int32_t* probes,
                            const int32_t* nsamp, const int64_t* sample_base, const double* sample_uv,
                            const uint8_t* quant, const orc_tol* tol, int32_t irr_r, int32_t dep_r, double hysteresis,
                            double tau_max, int32_t fp16, const int32_t* hint_tri, const uint8_t* hint_shadow,
                            const uint16_t* hint_ibin, const uint16_t* hint_dbin, double* irr,
                            uint8_t* irr_n, double* dep, uint8_t* dep_n, orc_counts* counts) {
  const int32_t ri = irr_r - 2, rd = dep_r - 2;
  orc_counts total;
  memset(&total, 0, sizeof(total));
#pragma omp parallel
  {
    orc_counts loc;
    memset(&loc, 0, sizeof(loc));
#pragma omp for schedule(dynamic, 4)
    for (int32_t q = 0; q < count; ++q) {
      double o[3];
      orc_probe_pos(g, probes[q], o);
      double* I = irr + (size_t)q * ri * ri * 3;
      double* D = dep + (size_t)q * rd * rd * 2;
      uint8_t* IN = irr_n + (size_t)q * ri * ri;
      uint8_t* DN = dep_n + (size_t)q * rd * rd;
      int64_t ties[2] = {0, 0}, mism[2] = {0, 0};
      for (int32_t j = 0; j < nsamp[q]; ++j) {
        const int64_t k = sample_base[q] + j;
        double d[3], nd[3];
        orc_chain_dir(sample_uv + 2 * k, d);
        for (int a = 0; a < 3; ++a) nd[a] = -d[a];
        int32_t ti = 0;
        int32_t ki = orc_oct_bin(d, ri, tol ? tol->bin_eps : 0.0, &ti);
        if (hint_ibin && hint_ibin[2 * k] != ki) {
          if (ti && hint_ibin[2 * k] < ri * ri) {
            loc.bin_ties++;
            ki = hint_ibin[2 * k];
          } else {
            loc.bin_mismatch++;
          }
        }
        int32_t td = 0;
        int32_t kd = orc_oct_bin(nd, rd, tol ? tol->bin_eps : 0.0, &td);
        if (hint_dbin && hint_dbin[2 * k + 1] != kd) {
          if (td && hint_dbin[2 * k + 1] < rd * rd) {
            loc.bin_ties++;
            kd = hint_dbin[2 * k + 1];
          } else {
            loc.bin_mismatch++;
          }
        }
        /* a probe with a dynamic component traces through the texel centres
         * (Sec. 4.9): the rays then add no sampling noise to the texels */
        if (quant && quant[q]) {
          orc_texel_centre_dir(ri, ki, d);
          orc_texel_centre_dir(rd, kd, nd);
        }
        /* irradiance: the ray along d, shaded as a probe ray */
        orc_ray ra, rb;
        orc_shade_ray(s, o, d, g->s, tol, hint_tri ? hint_tri[2 * k] : -2,
                      hint_shadow ? (int32_t)hint_shadow[2 * k] : -1, &ra, ties, mism);
        loc.rays += 1;
        if (ra.tri >= 0 && ra.front) loc.shadow_rays += s->nl;
        double ai = orc_blend_alpha(IN[ki], hysteresis);
        for (int c = 0; c < 3; ++c) I[3 * ki + c] += ai * (ra.rgb[c] - I[3 * ki + c]);
        if (IN[ki] < 255) IN[ki]++;
        /* visibility: the ray along -d, its distance into the depth texel of -d */
        orc_shade_ray(s, o, nd, g->s, tol, hint_tri ? hint_tri[2 * k + 1] : -2, -1, &rb, ties, mism);
        loc.rays += 1;
        double tau = isfinite(rb.t) ? fmin(rb.t / g->s, tau_max) : tau_max;
        double ad = orc_blend_alpha(DN[kd], hysteresis);
        D[2 * kd + 0] += ad * (tau - D[2 * kd + 0]);
        D[2 * kd + 1] += ad * (tau * tau - D[2 * kd + 1]);
        if (DN[kd] < 255) DN[kd]++;
      }
      if (fp16) { /* binary16 texel store at the end of the frame, as for probe rays */
        for (int32_t k = 0; k < ri * ri * 3; ++k) I[k] = orc_round_half(I[k]);
        for (int32_t k = 0; k < rd * rd * 2; ++k) D[k] = orc_round_half(D[k]);
      }
      loc.hit_ties += ties[0];
      loc.shadow_ties += ties[1];
      loc.hit_mismatch += mism[0];
      loc.shadow_mismatch += mism[1];
    }
#pragma omp critical
    {
      total.hit_ties += loc.hit_ties;
      total.shadow_ties += loc.shadow_ties;
      total.bin_ties += loc.bin_ties;
      total.hit_mismatch += loc.hit_mismatch;
      total.shadow_mismatch += loc.shadow_mismatch;
      total.bin_mismatch += loc.bin_mismatch;
      total.rays += loc.rays;
      total.shadow_rays += loc.shadow_rays;
    }
  }
  if (counts) {
    counts->hit_ties += total.hit_ties;
    counts->shadow_ties += total.shadow_ties;
    counts->bin_ties += total.bin_ties;
    counts->hit_mismatch += total.hit_mismatch;
    counts->shadow_mismatch += total.shadow_mismatch;
    counts->bin_mismatch += total.bin_mismatch;
    counts->rays += total.rays;
    counts->shadow_rays += total.shadow_rays;
  }
}

int32_t orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_threads(int32_t n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ------------------------------------------------------------------ query */

/* Bilinear sample of a full tile (interior r x r with a one-texel border,
 * c channels) at the direction d: interior texel i spans [i, i+1) of
 * f = (uv + 1) / 2 * r and holds its value at i + 1/2; the border supplies
 * the neighbours across the map's edges. */
static void tile_bilinear(const double* tile, int32_t r, int32_t c, const double d[3], double* out) {
  double uv[2];
  orc_oct_encode(d, uv);
  const double fx = (uv[0] + 1.0) * 0.5 * r - 0.5, fy = (uv[1] + 1.0) * 0.5 * r - 0.5;
  double x0 = floor(fx), y0 = floor(fy);
  if (x0 < -1.0) x0 = -1.0;
  if (x0 > r - 1) x0 = r - 1;
  if (y0 < -1.0) y0 = -1.0;
  if (y0 > r - 1) y0 = r - 1;
  const double ax = fx - x0, ay = fy - y0;
  const int32_t X = (int32_t)x0 + 1, Y = (int32_t)y0 + 1, g = r + 2;
  for (int32_t k = 0; k < c; ++k) {
    const double v00 = tile[(Y * g + X) * c + k], v01 = tile[(Y * g + X + 1) * c + k];
    const double v10 = tile[((Y + 1) * g + X) * c + k], v11 = tile[((Y + 1) * g + X + 1) * c + k];
    out[k] = (1.0 - ay) * ((1.0 - ax) * v00 + ax * v01) + ay * ((1.0 - ax) * v10 + ax * v11);
  }
}

void orc_query_irradiance(const orc_grid* g, const double* irr_tiles, int32_t irr_res, const double* dep_tiles,
                          int32_t dep_res, const double x[3], const double n[3], double rgb[3]) {
  const int32_t ri = irr_res - 2, rd = dep_res - 2;
  int32_t base[3];
  double al[3];
  for (int a = 0; a < 3; ++a) {
    if (g->dims[a] == 1) {
      base[a] = 0;
      al[a] = 0.0;
      continue;
    }
    const double f = (x[a] - g->origin[a]) / g->spacing[a];
    double b = floor(f);
    if (b < 0.0) b = 0.0;
    if (b > g->dims[a] - 2) b = g->dims[a] - 2;
    base[a] = (int32_t)b;
    double t = f - b;
    al[a] = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
  }
  double sum[3] = {0.0, 0.0, 0.0}, wsum = 0.0;
  for (int32_t corner = 0; corner < 8; ++corner) {
    int32_t idx[3];
    double tri = 1.0;
    int skip = 0;
    for (int a = 0; a < 3; ++a) {
      const int32_t o = (corner >> a) & 1;
      if (o && g->dims[a] == 1) skip = 1;
      idx[a] = base[a] + o;
      tri *= o ? al[a] : 1.0 - al[a];
    }
    if (skip) continue;
    const int32_t pr = idx[0] + g->dims[0] * (idx[1] + g->dims[1] * idx[2]);
    double p[3];
    orc_probe_pos(g, pr, p);
    double dir[3] = {p[0] - x[0], p[1] - x[1], p[2] - x[2]};
    const double len = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    double w = 1.0;
    if (len > 0.0) {
      for (int a = 0; a < 3; ++a) dir[a] /= len;
      /* smooth backface term: probes behind the surface count less */
      const double c = (dir[0] * n[0] + dir[1] * n[1] + dir[2] * n[2] + 1.0) * 0.5;
      w *= c * c + 0.2;
      /* visibility: the probe's depth moments towards the point, one-sided
       * Chebyshev bound on the probability that the point is unoccluded */
      const double back[3] = {-dir[0], -dir[1], -dir[2]};
      double m[2];
      tile_bilinear(dep_tiles + (size_t)pr * dep_res * dep_res * 2, rd, 2, back, m);
      const double rr = len / g->s;
      if (rr > m[0]) {
        const double var = fabs(m[1] - m[0] * m[0]);
        const double dd = rr - m[0];
        const double cheb = var / (var + dd * dd);
        w *= cheb * cheb * cheb;
      }
    }
    if (w < 1e-6) w = 1e-6;
    w *= tri;
    double e[3];
    tile_bilinear(irr_tiles + (size_t)pr * irr_res * irr_res * 3, ri, 3, n, e);
    for (int k = 0; k < 3; ++k) sum[k] += w * e[k];
    wsum += w;
  }
  for (int k = 0; k < 3; ++k) rgb[k] = wsum > 0.0 ? sum[k] / wsum : 0.0;
}
