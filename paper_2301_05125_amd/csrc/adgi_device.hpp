// adgi_device.hpp - device primitives for the gfx950 probe-update kernels.
//
// Counter-based random numbers, ray directions, the octahedral texel map,
// ray/box and ray/triangle tests, and wave-level ballot/prefix helpers. All
// arithmetic is FP32 or integer; nothing here uses FP64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "adgi_layout.hpp"

namespace adgi {

// ------------------------------------------------------------------ hashing
// splitmix64 output function (Steele, Lea & Flood, OOPSLA 2014).
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Key of one stream: seed^tag, then a, b, c mixed in turn.
__device__ __forceinline__ uint64_t stream_key(uint64_t seed, uint64_t tag, uint64_t a, uint64_t b,
                                               uint64_t c) {
  uint64_t h = splitmix64(seed ^ tag);
  h = splitmix64(h ^ a);
  h = splitmix64(h ^ b);
  return splitmix64(h ^ c);
}

// Uniform in [0,1) from the top 24 bits: exact in FP32.
__device__ __forceinline__ float uniform24(uint64_t key, uint64_t q) {
  return (float)(uint32_t)(splitmix64(key ^ q) >> 40) * (1.0f / 16777216.0f);
}

// ------------------------------------------------------------- directions
constexpr float kTwoPi = 6.28318530717958647692f;

// Spherical Fibonacci point j of n (z_j = 1-(2j+1)/n, phi_j = 2*pi*frac(j/golden)),
// rotated by the row-major frame rotation R. The azimuth fraction is the top
// 32 bits of the 64-bit fixed-point product j * 2^64/golden.
__device__ __forceinline__ float3 sf_direction(uint32_t j, uint32_t n, const float* R) {
  // 1 - z with the hardware reciprocal (<= 1 ulp); every kernel that needs
  // a probe-ray direction calls this same function, so they agree bitwise
  float a = (float)(2u * j + 1u) * __builtin_amdgcn_rcpf((float)n);
  float z = 1.0f - a;
  float r = sqrtf(fmaxf(0.0f, a * (2.0f - a)));  // sqrt(1 - z^2) without cancellation
  uint64_t f = (uint64_t)j * 0x9E3779B97F4A7C15ull;
  float phi = (float)(uint32_t)(f >> 32) * (kTwoPi / 4294967296.0f);
  float s, c;
  sincosf(phi, &s, &c);
  float vx = r * c, vy = r * s;
  return make_float3(fmaf(R[0], vx, fmaf(R[1], vy, R[2] * z)),
                     fmaf(R[3], vx, fmaf(R[4], vy, R[5] * z)),
                     fmaf(R[6], vx, fmaf(R[7], vy, R[8] * z)));
}

// Which spherical Fibonacci point ray j of a probe with n rays takes. The
// points are dealt into C = ceil(n/64) strata by index modulo C (stratum c:
// points c, c + C, c + 2C, ...), and the ray indices run through stratum 0,
// then stratum 1, and so on. Stratum c holds q + 1 points for c < n mod C and
// q otherwise (q = n / C, at most 64) and spreads over the whole sphere, where
// 64 consecutive points form a thin band in z; the blend takes one stratum per
// step, so few of a step's samples share a texel. n <= 64: ray j takes point j.
struct RayStrata {
  uint32_t C, q, rem;
  __host__ __device__ explicit RayStrata(uint32_t n)
      : C((n + 63u) >> 6), q(n > 0u ? n / ((n + 63u) >> 6) : 0u), rem(n > 0u ? n % ((n + 63u) >> 6) : 0u) {}
  __host__ __device__ uint32_t size(uint32_t c) const { return q + (c < rem ? 1u : 0u); }
  __host__ __device__ uint32_t start(uint32_t c) const { return c * q + (c < rem ? c : rem); }
};

// floor(a / d) for a < 2^16 and d >= 1: the hardware reciprocal's estimate
// is within 2^-6 of a / d there, so its truncation is off by at most one and
// one correction step either way makes it exact.
__device__ __forceinline__ uint32_t udiv16(uint32_t a, uint32_t d) {
  uint32_t q = (uint32_t)((float)a * __builtin_amdgcn_rcpf((float)d));
  if (q * d > a) --q;
  if ((q + 1u) * d <= a) ++q;
  return q;
}

__device__ __forceinline__ uint32_t sf_point_of_ray(uint32_t j, uint32_t n) {
  if (n <= 64u) return j;
  const bool small = n < 65536u;
  const uint32_t C = (n + 63u) >> 6;
  const uint32_t q = small ? udiv16(n, C) : n / C, rem = n - q * C;
  const uint32_t big = rem * (q + 1u);  // rays of the strata with q + 1 points
  uint32_t c, k;
  if (j < big) {
    c = small ? udiv16(j, q + 1u) : j / (q + 1u);
    k = j - c * (q + 1u);
  } else {
    const uint32_t t = j - big, cc = small ? udiv16(t, q) : t / q;
    c = rem + cc;
    k = t - cc * q;
  }
  return c + k * C;
}

// The ray that takes spherical Fibonacci point p (the inverse of the above).
__host__ __device__ __forceinline__ uint32_t ray_of_sf_point(uint32_t p, uint32_t n) {
  if (n <= 64u) return p;
  const RayStrata s(n);
  return s.start(p % s.C) + p / s.C;
}

// Pilot direction of octant k (bit0 -x, bit1 -y, bit2 -z) for pair m: a
// uniform sphere point folded into the octant.
__device__ __forceinline__ float3 pilot_direction(uint64_t seed, uint32_t probe, uint32_t k,
                                                  uint32_t pair) {
  uint64_t key = stream_key(seed, kTagPilot, probe, k, pair);
  float u = uniform24(key, 1), v = uniform24(key, 2);
  float z = 1.0f - 2.0f * u;
  float r = 2.0f * sqrtf(fmaxf(0.0f, u * (1.0f - u)));
  float s, c;
  sincosf(kTwoPi * v, &s, &c);
  float dx = fabsf(r * c), dy = fabsf(r * s), dz = fabsf(z);
  return make_float3((k & 1) ? -dx : dx, (k & 2) ? -dy : dy, (k & 4) ? -dz : dz);
}

// ------------------------------------------------------------- octahedral
// Octahedral map (Cigolle et al. 2014) and its half-open texel bins.
__device__ __forceinline__ float2 oct_encode(float3 d) {
  float inv = __builtin_amdgcn_rcpf(fabsf(d.x) + fabsf(d.y) + fabsf(d.z));
  float x = d.x * inv, y = d.y * inv;
  if (d.z < 0.0f) {
    float nx = (1.0f - fabsf(y)) * (x >= 0.0f ? 1.0f : -1.0f);
    float ny = (1.0f - fabsf(x)) * (y >= 0.0f ? 1.0f : -1.0f);
    x = nx;
    y = ny;
  }
  return make_float2(x, y);
}

// Unit direction of octahedral coordinates uv (the map's inverse).
__device__ __forceinline__ float3 oct_decode_dir(float2 uv) {
  float x = uv.x, y = uv.y;
  const float z = 1.0f - fabsf(x) - fabsf(y);
  if (z < 0.0f) {
    const float nx = (1.0f - fabsf(y)) * (x >= 0.0f ? 1.0f : -1.0f);
    const float ny = (1.0f - fabsf(x)) * (y >= 0.0f ? 1.0f : -1.0f);
    x = nx;
    y = ny;
  }
  const float inv = 1.0f / sqrtf(x * x + y * y + z * z);
  return make_float3(x * inv, y * inv, z * inv);
}

__device__ __forceinline__ uint32_t oct_bin(float2 uv, int r) {
  int ix = (int)floorf((uv.x + 1.0f) * 0.5f * (float)r);
  int iy = (int)floorf((uv.y + 1.0f) * 0.5f * (float)r);
  ix = min(max(ix, 0), r - 1);
  iy = min(max(iy, 0), r - 1);
  return (uint32_t)(iy * r + ix);
}

// Direction through the centre of interior texel t of an r x r map.
__device__ __forceinline__ float3 texel_centre_dir(uint32_t t, int r) {
  const int x = (int)(t % (uint32_t)r), y = (int)(t / (uint32_t)r);
  const float inv = 1.0f / (float)r;
  return oct_decode_dir(make_float2((float)(2 * x + 1) * inv - 1.0f, (float)(2 * y + 1) * inv - 1.0f));
}

// Tile coordinate (X,Y) in 0..r+1 -> source interior coordinate (1..r):
// border texels repeat the texel across the map's edge identification.
__device__ __forceinline__ void border_source(int X, int Y, int r, int& sx, int& sy) {
  bool bx = (X == 0) | (X == r + 1), by = (Y == 0) | (Y == r + 1);
  sx = X;
  sy = Y;
  if (bx && by) {
    sx = (X == 0) ? r : 1;
    sy = (Y == 0) ? r : 1;
  } else if (by) {
    sx = r + 1 - X;
    sy = (Y == 0) ? 1 : r;
  } else if (bx) {
    sy = r + 1 - Y;
    sx = (X == 0) ? 1 : r;
  }
}

// ------------------------------------------------------- packed texels
// Code of a binary32 value x >= 0 in a channel of eq. rgbEnc (beta, gamma,
// qmax = 2^bits - 1): floor(qmax min(ln(gamma x + 1), beta) / beta), the
// exact floor (App. B rounds down). Code k begins at t_k = (e^(beta k /
// qmax) - 1) / gamma, and the decoded value D_k is t_k rounded to nearest,
// so x >= t_k exactly when x > D_k, or x == D_k and D_k was rounded up (one
// bit per code, `up`). With k the estimate qmax log2(gamma x + 1) ln 2 /
// beta (hardware base-2 log, 1 ulp: within 2e-3 code units) rounded to the
// nearest integer, the exact code is k or k - 1, and that one comparison
// decides. dec and up are indexed by base + k (the channel's table).
template <int BITS>
__device__ __forceinline__ uint32_t pk_encode(float v, float beta, float gamma, const float* dec, const uint32_t* up,
                                              int base) {
  constexpr uint32_t qmax = (1u << BITS) - 1u;
  const float x = v > 0.0f ? v : 0.0f;
  // qmax ln 2 / beta, rounded once (beta is a literal of the channel)
  const float scale = (float)((double)qmax * 0.69314718055994530942 / (double)beta);
  const float kr = rintf(__builtin_amdgcn_logf(fmaf(gamma, x, 1.0f)) * scale);
  const uint32_t k = kr < 0.5f ? 0u : kr > (float)qmax ? qmax : (uint32_t)kr;
  const int t = base + (int)k;
  const float d = dec[t];
  const bool rounded_up = (up[t >> 5] >> (t & 31)) & 1u;
  const bool reached = x > d || (x == d && rounded_up);  // code 0: D_0 = 0, rounded up
  return reached ? k : k - 1u;
}

// ------------------------------------------------------------ ray tests
struct Ray {
  float3 o, d, inv, oinv;  // origin, direction, 1/d (zero components nudged), o/d
};

__device__ __forceinline__ Ray make_ray(float3 o, float3 d) {
  Ray r;
  r.o = o;
  r.d = d;
  const float tiny = 1e-20f;
  float dx = fabsf(d.x) < tiny ? copysignf(tiny, d.x) : d.x;
  float dy = fabsf(d.y) < tiny ? copysignf(tiny, d.y) : d.y;
  float dz = fabsf(d.z) < tiny ? copysignf(tiny, d.z) : d.z;
  r.inv = make_float3(1.0f / dx, 1.0f / dy, 1.0f / dz);
  r.oinv = make_float3(o.x * r.inv.x, o.y * r.inv.y, o.z * r.inv.z);
  return r;
}

// Slab test against a box whose bounds were padded outward at build/refit
// time, so FP32 rounding here never culls a box a hit lies in.
__device__ __forceinline__ bool box_hit(const Ray& r, float lx, float ly, float lz, float hx,
                                        float hy, float hz, float tmin, float tmax, float& tnear) {
  float t0x = fmaf(lx, r.inv.x, -r.oinv.x), t1x = fmaf(hx, r.inv.x, -r.oinv.x);
  float t0y = fmaf(ly, r.inv.y, -r.oinv.y), t1y = fmaf(hy, r.inv.y, -r.oinv.y);
  float t0z = fmaf(lz, r.inv.z, -r.oinv.z), t1z = fmaf(hz, r.inv.z, -r.oinv.z);
  float tn = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), tmin));
  float tf = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), tmax));
  tnear = tn;
  return tn <= tf;
}

// Moller-Trumbore without division in the accept test: accept when
// u, v >= 0, u + v <= 1 and t in (tmin, tmax] with u = U/det, v = V/det,
// t = T/det, comparisons made on the det-scaled values.
__device__ __forceinline__ bool tri_hit(const Ray& r, float4 a, float4 b, float4 c, float tmin,
                                        float tmax, float& t_out, bool& front) {
  float3 v0 = make_float3(a.x, a.y, a.z);
  float3 e1 = make_float3(b.x, b.y, b.z);
  float3 e2 = make_float3(c.x, c.y, c.z);
  float px = r.d.y * e2.z - r.d.z * e2.y;
  float py = r.d.z * e2.x - r.d.x * e2.z;
  float pz = r.d.x * e2.y - r.d.y * e2.x;
  float det = e1.x * px + e1.y * py + e1.z * pz;
  float tx = r.o.x - v0.x, ty = r.o.y - v0.y, tz = r.o.z - v0.z;
  float U = tx * px + ty * py + tz * pz;
  float qx = ty * e1.z - tz * e1.y;
  float qy = tz * e1.x - tx * e1.z;
  float qz = tx * e1.y - ty * e1.x;
  float V = r.d.x * qx + r.d.y * qy + r.d.z * qz;
  float T = e2.x * qx + e2.y * qy + e2.z * qz;
  float sg = det > 0.0f ? 1.0f : -1.0f;
  float adet = fabsf(det);
  U *= sg;
  V *= sg;
  float Ts = T * sg;
  // every reject test evaluated (no short circuit), one branch: the same
  // decisions as testing them in turn, with less control flow per triangle
  const bool reject = (det == 0.0f) | (U < 0.0f) | (V < 0.0f) | (U + V > adet) | (Ts <= tmin * adet) |
                      (Ts > tmax * adet);
  if (reject) return false;
  t_out = T / det;
  if (!(t_out > tmin && t_out <= tmax)) return false;
  front = det > 0.0f;  // (e1 x e2) . d < 0
  return true;
}

// ----------------------------------------------------------------- waves
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Number of set bits of `mask` in lanes below this one.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

}  // namespace adgi
