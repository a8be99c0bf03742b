// blend.hip - per-probe texel update.
//
// Every sample updates the texel that contains its direction ("the closest
// entry", Alg. ApproxAlgo) with the moving average of Alg. MovingAvgUpdate:
// V <- V + a (x - V), a = max(1/(N+1), 1-h), N <- min(N+1, 255): a running
// mean while 1/(N+1) > 1-h, then an exponential average with hysteresis h.
// Irradiance texels take the ray's radiance; depth texels take the moments
// (tau, tau^2) of tau = min(t/s, tau_max) (Sec. 4.6). Samples of one texel are
// applied in ascending ray order. Two kernels: the general one (any tile
// size, one workgroup per probe) and the scheduled one further below. In the
// general kernel the probe's texel tile is staged in LDS;
// rays are processed in chunks: coalesced load of the chunk's 16-byte
// records, octahedral bins recomputed from the ray index, an LDS counting
// sort by texel (histogram, scan, scatter, then a short insertion sort of each
// texel's list to restore ray order), and one thread per texel applying its
// samples in sequence. The tile is written back with its one-texel border
// folded across the octahedral map's edges. FP32 arithmetic throughout;
// FP16 storage is widened on load and rounded to nearest-even on store.
#include <hip/hip_fp16.h>

#include "adgi_internal.hpp"

namespace adgi {

template <bool HALF>
struct Store;
template <>
struct Store<false> {
  using T = float;
  __device__ static float load(const T* p) { return *p; }
  __device__ static void store(T* p, float x) { *p = x; }
};
template <>
struct Store<true> {
  using T = __half;
  __device__ static float load(const T* p) { return __half2float(*p); }
  __device__ static void store(T* p, float x) { *p = __float2half_rn(x); }
};

// The binary16 value in the low 16 bits of w, and two values rounded to
// binary16 (nearest even) packed low | high << 16.
__device__ __forceinline__ float half_bits(uint32_t w) {
  return __half2float(__ushort_as_half((unsigned short)(w & 0xFFFFu)));
}
__device__ __forceinline__ uint32_t half_word(float lo, float hi) {
  return (uint32_t)__half_as_ushort(__float2half_rn(lo)) | ((uint32_t)__half_as_ushort(__float2half_rn(hi)) << 16);
}

__device__ uint32_t block_scan_u32(uint32_t x, uint32_t* sm, uint32_t& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  uint32_t v = x;
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t y = __shfl_up(v, off);
    if (lane >= off) v += y;
  }
  if (lane == 63) sm[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (int k = 0; k < nw; ++k) {
      uint32_t t = sm[k];
      sm[k] = acc;
      acc += t;
    }
    sm[nw] = acc;
  }
  __syncthreads();
  total = sm[nw];
  uint32_t r = v - x + sm[wave];
  __syncthreads();
  return r;
}

struct BlendLds {
  float* stI;
  float* stD;
  uint32_t* cnt;
  uint32_t* hist;
  uint32_t* start;
  uint32_t* cursor;
  uint32_t* scan;
  float4* rec;
  uint16_t* bins;
  uint16_t* list;
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

__host__ __device__ inline size_t blend_layout(int irr_res, int dep_res, int chunk, BlendLds* L,
                                               uint8_t* base) {
  const int ri = irr_res - 2, rd = dep_res - 2, nI = ri * ri, nD = rd * rd, nT = nI + nD;
  size_t o = 0;
  size_t oStI = o; o += (size_t)nI * 3 * 4;
  size_t oStD = o; o += (size_t)nD * 2 * 4;
  size_t oCnt = o; o += (size_t)nT * 4;
  size_t oHist = o; o += (size_t)nT * 4;
  size_t oStart = o; o += (size_t)nT * 4;
  size_t oCur = o; o += (size_t)nT * 4;
  size_t oScan = o; o += 17 * 4;
  o = align16(o);
  size_t oRec = o; o += (size_t)chunk * 16;
  size_t oBins = o; o += (size_t)chunk * 2 * 2;
  size_t oList = o; o += (size_t)chunk * 2 * 2;
  if (L) {
    L->stI = (float*)(base + oStI);
    L->stD = (float*)(base + oStD);
    L->cnt = (uint32_t*)(base + oCnt);
    L->hist = (uint32_t*)(base + oHist);
    L->start = (uint32_t*)(base + oStart);
    L->cursor = (uint32_t*)(base + oCur);
    L->scan = (uint32_t*)(base + oScan);
    L->rec = (float4*)(base + oRec);
    L->bins = (uint16_t*)(base + oBins);
    L->list = (uint16_t*)(base + oList);
  }
  return align16(o);
}

template <bool HALF>
__global__ __launch_bounds__(256) void blend_kernel(VolumeView v, BlendIO io, int chunk) {
  using S = Store<HALF>;
  using T = typename S::T;
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  BlendLds L;
  blend_layout(v.irr_res, v.dep_res, chunk, &L, smem);
  const int i = blockIdx.x;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int gi = v.irr_res, gd = v.dep_res;
  const int ri = gi - 2, rd = gd - 2, nI = ri * ri, nD = rd * rd, nT = nI + nD;
  const FrameParams& fp = *v.fp;

  // ---- load the interior of both tiles and the counts
  const T* irr_in = (const T*)io.irr_in + (size_t)i * gi * gi * 3;
  const T* dep_in = (const T*)io.dep_in + (size_t)i * gd * gd * 2;
  for (int f = tid; f < nI * 3; f += nt) {
    int k = f / 3, c = f - 3 * k, iy = k / ri, ix = k - iy * ri;
    L.stI[f] = S::load(irr_in + ((iy + 1) * gi + ix + 1) * 3 + c);
  }
  for (int f = tid; f < nD * 2; f += nt) {
    int k = f >> 1, c = f & 1, iy = k / rd, ix = k - iy * rd;
    L.stD[f] = S::load(dep_in + ((iy + 1) * gd + ix + 1) * 2 + c);
  }
  for (int k = tid; k < nT; k += nt)
    L.cnt[k] = k < nI ? io.irr_n_in[(size_t)i * nI + k] : io.dep_n_in[(size_t)i * nD + (k - nI)];

  const uint32_t off = v.offsets[i];
  const uint32_t n = v.offsets[i + 1] - off;
  const float inv_s = 1.0f / v.s_diag;
  for (uint32_t c0 = 0; c0 < n; c0 += (uint32_t)chunk) {
    const int m = (int)min((uint32_t)chunk, n - c0);
    for (int k = tid; k < nT; k += nt) L.hist[k] = 0u;
    for (int j = tid; j < m; j += nt) L.rec[j] = v.rec[off + c0 + j];
    __syncthreads();
    for (int j = tid; j < m; j += nt) {
      float3 d = sf_direction(sf_point_of_ray(c0 + (uint32_t)j, n), n, fp.R);
      float2 uv = oct_encode(d);
      uint32_t bI = oct_bin(uv, ri), bD = oct_bin(uv, rd);
      L.bins[j] = (uint16_t)bI;
      L.bins[chunk + j] = (uint16_t)(nI + bD);
      atomicAdd(&L.hist[bI], 1u);
      atomicAdd(&L.hist[nI + bD], 1u);
    }
    __syncthreads();
    // exclusive scan of the histogram over the combined texel space
    const int seg = (nT + nt - 1) / nt, sb = tid * seg, se = min(nT, sb + seg);
    uint32_t loc = 0;
    for (int k = sb; k < se; ++k) loc += L.hist[k];
    uint32_t tot;
    uint32_t base = block_scan_u32(loc, L.scan, tot);
    for (int k = sb; k < se; ++k) {
      L.start[k] = base;
      L.cursor[k] = base;
      base += L.hist[k];
    }
    __syncthreads();
    for (int j = tid; j < m; j += nt) {
      uint32_t p = atomicAdd(&L.cursor[L.bins[j]], 1u);
      L.list[p] = (uint16_t)j;
      p = atomicAdd(&L.cursor[L.bins[chunk + j]], 1u);
      L.list[p] = (uint16_t)j;
    }
    __syncthreads();
    for (int k = tid; k < nT; k += nt) {
      const uint32_t s = L.start[k], e = s + L.hist[k];
      // restore ascending ray order within the texel
      for (uint32_t a = s + 1; a < e; ++a) {
        uint16_t key = L.list[a];
        uint32_t b = a;
        while (b > s && L.list[b - 1] > key) {
          L.list[b] = L.list[b - 1];
          --b;
        }
        L.list[b] = key;
      }
      uint32_t N = L.cnt[k];
      if (k < nI) {
        float V0 = L.stI[3 * k], V1 = L.stI[3 * k + 1], V2 = L.stI[3 * k + 2];
        for (uint32_t a = s; a < e; ++a) {
          float4 r = L.rec[L.list[a]];
          float al = fmaxf(1.0f / (float)(N + 1u), v.one_minus_h);
          V0 = fmaf(al, r.x - V0, V0);
          V1 = fmaf(al, r.y - V1, V1);
          V2 = fmaf(al, r.z - V2, V2);
          N = min(N + 1u, 255u);
        }
        L.stI[3 * k] = V0;
        L.stI[3 * k + 1] = V1;
        L.stI[3 * k + 2] = V2;
      } else {
        const int kd = k - nI;
        float V0 = L.stD[2 * kd], V1 = L.stD[2 * kd + 1];
        for (uint32_t a = s; a < e; ++a) {
          float t = L.rec[L.list[a]].w;
          float tau = fminf(t * inv_s, v.tau_max);
          float al = fmaxf(1.0f / (float)(N + 1u), v.one_minus_h);
          V0 = fmaf(al, tau - V0, V0);
          V1 = fmaf(al, tau * tau - V1, V1);
          N = min(N + 1u, 255u);
        }
        L.stD[2 * kd] = V0;
        L.stD[2 * kd + 1] = V1;
      }
      L.cnt[k] = N;
    }
    __syncthreads();
  }

  // ---- write both tiles with the border fold, then the counts
  T* irr_out = (T*)io.irr_out + (size_t)i * gi * gi * 3;
  T* dep_out = (T*)io.dep_out + (size_t)i * gd * gd * 2;
  __syncthreads();
  for (int f = tid; f < gi * gi * 3; f += nt) {
    int t = f / 3, c = f - 3 * t, Y = t / gi, X = t - Y * gi, sx, sy;
    border_source(X, Y, ri, sx, sy);
    S::store(irr_out + f, L.stI[((sy - 1) * ri + (sx - 1)) * 3 + c]);
  }
  for (int f = tid; f < gd * gd * 2; f += nt) {
    int t = f >> 1, c = f & 1, Y = t / gd, X = t - Y * gd, sx, sy;
    border_source(X, Y, rd, sx, sy);
    S::store(dep_out + f, L.stD[((sy - 1) * rd + (sx - 1)) * 2 + c]);
  }
  for (int k = tid; k < nT; k += nt) {
    uint8_t c = (uint8_t)L.cnt[k];
    if (k < nI) io.irr_n_out[(size_t)i * nI + k] = c;
    else io.dep_n_out[(size_t)i * nD + (k - nI)] = c;
  }
}

// ---------------------------------------------------------------------------
// Wave-per-probe variant for the common tile sizes. One 64-lane wave owns one
// probe and keeps its interior texels, depth moments and counts in LDS for
// the whole frame (loaded row by row, coalesced). Rays are taken one stratum
// (sf_point_of_ray: at most 64 rays spread over the sphere) at a time, one
// per lane, with the texel indices the trace stored for each ray. Each lane
// ORs its lane bit into a 64-bit LDS mask of its irradiance texel and of its
// depth texel; the set bits below a lane give its rank among the step's
// samples of the same texel. Round r then applies, in every lane of rank r at
// once, that lane's sample to its texel: a texel takes its samples in
// ascending ray order and no two lanes touch one texel in a round, so the
// moving average is the same sequence of FP32 operations as one sample at a
// time, and a step takes as many rounds as its most-hit texel has samples.
// The next step's records are loaded while the current ones are applied.
// Waves take probes in the allocation's order (most rays first) so the
// longest blends start first.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int RI, int RD>
struct WaveTile {
  static constexpr int NI = RI * RI, ND = RD * RD, NT = NI + ND;
  static constexpr int SI = (NI + 63) / 64, SD = (ND + 63) / 64;
  static constexpr int GI = RI + 2, GD = RD + 2;
  // the per-sample wave's LDS: the interior texels as planes, irradiance
  // r[NI] g[NI] b[NI] N[NI] and depth tau[ND] tau^2[ND] N[ND] (N the sample
  // count, one word each), so lanes that update different texels of one map
  // touch consecutive words (distinct banks) instead of strided records
  static constexpr size_t kStI = 0, kStD = 16 * (size_t)NI;
  static constexpr size_t kRankBytes = kStD + 12 * (size_t)ND;
  // then one 64-bit lane mask per interior texel (irradiance, then depth):
  // the lanes of the current chunk whose samples fall in that texel
  static constexpr size_t kMaskI = kRankBytes, kMaskD = kMaskI + 8 * (size_t)NI;
  static constexpr size_t kMaskEnd = kMaskD + 8 * (size_t)ND;
  // the other wave kernels' LDS (packed, gather): a chunk of records and the masks,
  // or the staged interior
  static constexpr size_t kChunkBytes = 64 * 16 + 8 * (size_t)NT;
  static constexpr size_t kStageBytes = 4 * (3 * (size_t)NI + 2 * (size_t)ND) + NT;
  static constexpr size_t kOldBytes = ((kChunkBytes > kStageBytes ? kChunkBytes : kStageBytes) + 15) & ~(size_t)15;
  static constexpr size_t kWaveBytes = kOldBytes > kMaskEnd ? kOldBytes : kMaskEnd;
  static constexpr size_t kTabBytes = (2 * (GI * GI * 3 + GD * GD * 2) + 15) & ~(size_t)15;
  static constexpr size_t kBlockBytes = 4 * kWaveBytes + kTabBytes + 2 * 256 * 4;  // + two step tables
  static_assert(NI % 4 == 0 && ND % 4 == 0, "counts are moved as 32-bit words");
};

// One texel update with the moving average of Alg. MovingAvgUpdate; the
// step weight max(1/(N+1), 1-h) comes from a per-workgroup table.
__device__ __forceinline__ void blend_rgb(float* V, uint32_t& N, float4 r, const float* alpha) {
  const float al = alpha[N];
  V[0] = fmaf(al, r.x - V[0], V[0]);
  V[1] = fmaf(al, r.y - V[1], V[1]);
  V[2] = fmaf(al, r.z - V[2], V[2]);
  N = min(N + 1u, 255u);
}
__device__ __forceinline__ void blend_tau(float* V, uint32_t& N, float t, float inv_s, float tmax,
                                          const float* alpha) {
  const float tau = fminf(t * inv_s, tmax);
  const float al = alpha[N];
  V[0] = fmaf(al, tau - V[0], V[0]);
  V[1] = fmaf(al, tau * tau - V[1], V[1]);
  N = min(N + 1u, 255u);
}

// Tile element -> interior source element (border fold), built once per
// workgroup in LDS: irradiance [GI*GI*3], then depth [GD*GD*2]. Interior
// texel k's channel c sits at 3k + c / 2k + c, or with PLANAR at c NI + k /
// c ND + k.
template <int RI, int RD, bool PLANAR = false>
__device__ void build_fold_tables(uint16_t* tab) {
  using W = WaveTile<RI, RD>;
  constexpr int GI = W::GI, GD = W::GD;
  for (int f = threadIdx.x; f < GI * GI * 3; f += blockDim.x) {
    const int t = f / 3, c = f - 3 * t, Y = t / GI, X = t - Y * GI;
    int sx, sy;
    border_source(X, Y, RI, sx, sy);
    const int k = (sy - 1) * RI + (sx - 1);
    tab[f] = (uint16_t)(PLANAR ? c * W::NI + k : 3 * k + c);
  }
  for (int f = threadIdx.x; f < GD * GD * 2; f += blockDim.x) {
    const int t = f >> 1, c = f & 1, Y = t / GD, X = t - Y * GD;
    int sx, sy;
    border_source(X, Y, RD, sx, sy);
    const int k = (sy - 1) * RD + (sx - 1);
    tab[GI * GI * 3 + f] = (uint16_t)(PLANAR ? c * W::ND + k : 2 * k + c);
  }
}

// Write the staged interior (stI, stD, stN in LDS) as full tiles with the border fold.
template <int RI, int RD, bool HALF>
__device__ void write_tiles(const VolumeView& v, const BlendIO& io, int i, const float* stI,
                            const float* stD, const uint8_t* stN, const uint16_t* tab, int t0,
                            int nthreads) {
  using S = Store<HALF>;
  using T = typename S::T;
  using W = WaveTile<RI, RD>;
  constexpr int NI = W::NI, ND = W::ND, GI = W::GI, GD = W::GD;
  T* irr_out = (T*)io.irr_out + (size_t)i * GI * GI * 3;
  T* dep_out = (T*)io.dep_out + (size_t)i * GD * GD * 2;
  for (int f = t0; f < GI * GI * 3; f += nthreads) S::store(irr_out + f, stI[tab[f]]);
  for (int f = t0; f < GD * GD * 2; f += nthreads) S::store(dep_out + f, stD[tab[GI * GI * 3 + f]]);
  for (int k = t0; k < NI; k += nthreads) io.irr_n_out[(size_t)i * NI + k] = stN[k];
  for (int k = t0; k < ND; k += nthreads) io.dep_n_out[(size_t)i * ND + k] = stN[NI + k];
}

// Light probe: one wave.
// CHAIN: the probe's list holds chain samples k (grouped by probe): the
// irradiance texel of d(uv_k) takes the radiance of ray 2k, the depth texel
// of -d takes the distance of ray 2k+1.
__device__ __forceinline__ float4 chain_record(const VolumeView& v, uint32_t k) {
  const float4 a = v.rec[2 * (size_t)k];
  return make_float4(a.x, a.y, a.z, v.rec[2 * (size_t)k + 1].w);
}

// One sample into texel k of the LDS planes: the moving average of Alg.
// MovingAvgUpdate with the step weight max(1/(N+1), 1-h) from the
// workgroup's table (the same FP32 operations as blend_rgb / blend_tau).
template <int NI>
__device__ __forceinline__ void plane_rgb(float* sI, uint32_t k, float4 r, const float* alpha) {
  uint32_t* nk = (uint32_t*)(sI + 3 * NI) + k;
  const uint32_t n = *nk;
  const float al = alpha[n];
  sI[k] = fmaf(al, r.x - sI[k], sI[k]);
  sI[NI + k] = fmaf(al, r.y - sI[NI + k], sI[NI + k]);
  sI[2 * NI + k] = fmaf(al, r.z - sI[2 * NI + k], sI[2 * NI + k]);
  *nk = min(n + 1u, 255u);
}
template <int ND>
__device__ __forceinline__ void plane_tau(float* sD, uint32_t k, float tau, float tau2, const float* alpha) {
  uint32_t* nk = (uint32_t*)(sD + 2 * ND) + k;
  const uint32_t n = *nk;
  const float al = alpha[n];
  sD[k] = fmaf(al, tau - sD[k], sD[k]);
  sD[ND + k] = fmaf(al, tau2 - sD[ND + k], sD[ND + k]);
  *nk = min(n + 1u, 255u);
}

// What a wave loads for a probe before it works on it: its interior texels
// (row by row, so consecutive lanes read consecutive words), its counts as
// 32-bit words, and the record and texel indices of its first 64 samples.
template <int RI, int RD, bool HALF, bool CHAIN>
struct ProbeRegs {
  using W = WaveTile<RI, RD>;
  // FP32: the interior irradiance values row by row, and each interior
  // depth texel's (tau, tau^2) as one 8-byte value (td, td2); FP16: 32-bit
  // words of two halves, the whole irradiance tile (its rows start at odd
  // halves) and the interior depth texels (one word each)
  static constexpr int kIrrWords = W::GI * W::GI * 3 / 2;
  static constexpr int LI = HALF ? (kIrrWords + 63) / 64 : (3 * W::NI + 63) / 64;
  static constexpr int LD = (W::ND + 63) / 64;
  static constexpr int CI = (W::NI / 4 + 63) / 64, CD = (W::ND / 4 + 63) / 64;
  uint32_t ti[LI], td[LD], td2[HALF ? 1 : LD];
  uint32_t ci[CI], cd[CD];
  float4 rec;
  uint32_t bins;  // budgeted frames: irradiance texel | depth texel << 16
  float2 uv;      // chain frames: the sample's octahedral coordinates
  float4 prec;    // pilot reuse: pilot (lane < 8) record and texel indices
  uint32_t pbins;
};

// Record and texel indices (or chain uv) of sample j of the list at off.
template <bool CHAIN>
__device__ __forceinline__ void load_sample(const VolumeView& v, uint32_t off, uint32_t j, float4& rec,
                                            uint32_t& bins, float2& uv) {
  if (CHAIN) {
    rec = chain_record(v, off + j);
    uv = v.smp_uv[off + j];
  } else {
    rec = v.rec[off + j];
    bins = v.ray_bins[off + j];
  }
}

// Samples per step of a probe's blend: probe rays one stratum at a time
// (sf_point_of_ray: at most 64 rays spread over the sphere), chain samples 64
// at a time. Either way a step holds the next samples in ascending order.
template <bool CHAIN>
__device__ __forceinline__ uint32_t first_step_size(uint32_t n) {
  return CHAIN ? min(64u, n) : RayStrata(n).size(0u);
}

template <int RI, int RD, bool HALF, bool CHAIN>
__device__ __forceinline__ void load_probe(const VolumeView& v, const BlendIO& io, int i, uint32_t off,
                                           uint32_t n, bool reuse, ProbeRegs<RI, RD, HALF, CHAIN>& g) {
  using S = Store<HALF>;
  using T = typename S::T;
  using W = WaveTile<RI, RD>;
  using G = ProbeRegs<RI, RD, HALF, CHAIN>;
  constexpr int NI = W::NI, ND = W::ND, GI = W::GI, GD = W::GD;
  const int lane = threadIdx.x & 63;
  if constexpr (HALF) {
    const uint32_t* irr_w = (const uint32_t*)io.irr_in + (size_t)i * G::kIrrWords;
    const uint32_t* dep_w = (const uint32_t*)io.dep_in + (size_t)i * GD * GD;
#pragma unroll
    for (int s = 0; s < G::LI; ++s)
      if (lane + 64 * s < G::kIrrWords) g.ti[s] = irr_w[lane + 64 * s];
#pragma unroll
    for (int s = 0; s < G::LD; ++s) {
      const int k = lane + 64 * s;
      if (k < ND) {
        const int row = k / RD, col = k - row * RD;
        g.td[s] = dep_w[(row + 1) * GD + col + 1];
      }
    }
  } else {
    const T* irr_in = (const T*)io.irr_in + (size_t)i * GI * GI * 3;
    const T* dep_in = (const T*)io.dep_in + (size_t)i * GD * GD * 2;
#pragma unroll
    for (int s = 0; s < G::LI; ++s) {
      const int f = lane + 64 * s;
      if (f < 3 * NI) {
        const int row = f / (3 * RI), col = f - row * (3 * RI);
        g.ti[s] = __float_as_uint(S::load(irr_in + ((row + 1) * GI + 1) * 3 + col));
      }
    }
    const float2* dep2 = (const float2*)dep_in;
#pragma unroll
    for (int s = 0; s < G::LD; ++s) {
      const int k = lane + 64 * s;
      if (k < ND) {
        const int row = k / RD, col = k - row * RD;
        const float2 m = dep2[(row + 1) * GD + col + 1];
        g.td[s] = __float_as_uint(m.x);
        g.td2[s] = __float_as_uint(m.y);
      }
    }
  }
  const uint32_t* ni_in = (const uint32_t*)(io.irr_n_in + (size_t)i * NI);
  const uint32_t* nd_in = (const uint32_t*)(io.dep_n_in + (size_t)i * ND);
#pragma unroll
  for (int s = 0; s < G::CI; ++s)
    if (lane + 64 * s < NI / 4) g.ci[s] = ni_in[lane + 64 * s];
#pragma unroll
  for (int s = 0; s < G::CD; ++s)
    if (lane + 64 * s < ND / 4) g.cd[s] = nd_in[lane + 64 * s];
  if ((uint32_t)lane < first_step_size<CHAIN>(n)) load_sample<CHAIN>(v, off, (uint32_t)lane, g.rec, g.bins, g.uv);
  if (reuse && lane < 8) {
    g.prec = v.pilot_rec[8 * (size_t)i + lane];
    g.pbins = v.pilot_bins[8 * (size_t)i + lane];
  }
}

template <int RI, int RD, bool HALF, bool CHAIN>
__device__ __forceinline__ void stage_probe(const ProbeRegs<RI, RD, HALF, CHAIN>& g, uint8_t* wbase) {
  using W = WaveTile<RI, RD>;
  using G = ProbeRegs<RI, RD, HALF, CHAIN>;
  constexpr int NI = W::NI, ND = W::ND;
  const int lane = threadIdx.x & 63;
  float* sI = (float*)(wbase + W::kStI);
  float* sD = (float*)(wbase + W::kStD);
  uint32_t* nI = (uint32_t*)(sI + 3 * NI);
  uint32_t* nD = (uint32_t*)(sD + 2 * ND);
  if constexpr (HALF) {
    constexpr int GI = W::GI;
#pragma unroll
    for (int s = 0; s < G::LI; ++s) {
      const int w = lane + 64 * s;
      if (w < G::kIrrWords) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int h = 2 * w + b, t = h / 3, c = h - 3 * t, Y = t / GI, X = t - Y * GI;
          if (X >= 1 && X <= RI && Y >= 1 && Y <= RI)
            sI[c * NI + (Y - 1) * RI + (X - 1)] = half_bits(g.ti[s] >> (16 * b));
        }
      }
    }
#pragma unroll
    for (int s = 0; s < G::LD; ++s) {
      const int k = lane + 64 * s;
      if (k < ND) {
        sD[k] = half_bits(g.td[s]);
        sD[ND + k] = half_bits(g.td[s] >> 16);
      }
    }
  } else {
#pragma unroll
    for (int s = 0; s < G::LI; ++s) {
      const int f = lane + 64 * s;
      if (f < 3 * NI) {
        const int k = f / 3;
        sI[(f - 3 * k) * NI + k] = __uint_as_float(g.ti[s]);
      }
    }
#pragma unroll
    for (int s = 0; s < G::LD; ++s) {
      const int k = lane + 64 * s;
      if (k < ND) {
        sD[k] = __uint_as_float(g.td[s]);
        sD[ND + k] = __uint_as_float(g.td2[s]);
      }
    }
  }
  // counts: word w holds the counts of texels 4w .. 4w+3
#pragma unroll
  for (int s = 0; s < G::CI; ++s) {
    const int w = lane + 64 * s;
    if (w < NI / 4)
#pragma unroll
      for (int b = 0; b < 4; ++b) nI[4 * w + b] = (g.ci[s] >> (8 * b)) & 0xFFu;
  }
#pragma unroll
  for (int s = 0; s < G::CD; ++s) {
    const int w = lane + 64 * s;
    if (w < ND / 4)
#pragma unroll
      for (int b = 0; b < 4; ++b) nD[4 * w + b] = (g.cd[s] >> (8 * b)) & 0xFFu;
  }
}

// The samples of probe i (n of them at off; the first 64 already in
// rec0/bins0/uv0) into its LDS texels, then the dynamic pass of chain frames.
// at_last_chunk() runs once, when the probe's last chunk of records has been
// loaded (before it is applied), so the wave's loads of its next probe go out
// behind every load of this one and overlap the rest of its work.
template <int RI, int RD, bool HALF, bool CHAIN, typename F>
__device__ __forceinline__ void blend_probe_samples(const VolumeView& v, int i, uint32_t off, uint32_t n,
                                                    float4 rec0, uint32_t bins0, float2 uv0, bool reuse,
                                                    float4 prec, uint32_t pbins, uint8_t* wbase,
                                                    const float* alpha, const float* alpha_dyn,
                                                    F&& at_last_chunk) {
  using W = WaveTile<RI, RD>;
  constexpr int NI = W::NI, ND = W::ND;
  const int lane = threadIdx.x & 63;
  float* sI = (float*)(wbase + W::kStI);
  float* sD = (float*)(wbase + W::kStD);
  const FrameParams& fp = *v.fp;
  const float inv_s = 1.0f / v.s_diag;
  const float tmax = v.tau_max;
  uint32_t* nI = (uint32_t*)(sI + 3 * NI);
  uint32_t* nD = (uint32_t*)(sD + 2 * ND);
  // One chunk of up to 64 samples, one per lane (act), each with its record
  // and its texel indices.
  uint64_t* mkI = (uint64_t*)(wbase + W::kMaskI);
  uint64_t* mkD = (uint64_t*)(wbase + W::kMaskD);
  auto apply = [&](const float4 cur, const uint32_t cbin, const bool act) {
    const uint32_t bI = cbin & 0xFFFFu, bD = cbin >> 16;
    // the chunk's lanes in this lane's texels: every lane ORs its bit into
    // the masks of its two texels (OR commutes, so the order in which the
    // lanes land does not matter), reads them back, and clears them for the
    // next chunk (a wave's LDS accesses complete in issue order)
    uint64_t mI = 0ull, mD = 0ull;
    if (act) {
      atomicOr((unsigned long long*)&mkI[bI], 1ull << lane);
      atomicOr((unsigned long long*)&mkD[bD], 1ull << lane);
    }
    wave_sync();
    if (act) {
      mI = mkI[bI];
      mD = mkD[bD];
    }
    wave_sync();
    if (act) {
      mkI[bI] = 0ull;
      mkD[bD] = 0ull;
    }
    // rank of this sample among the chunk's samples of the same texel, and
    // their number
    const uint32_t rI = lanes_below(mI), rD = lanes_below(mD);
    // the sample's count N before it is applied is the texel's count before
    // the chunk plus its rank (saturating at 255), so its step weight is known
    // before any sample of the chunk is applied; the last sample of each
    // texel writes the texel's new count
    float aI = 0.f, aD = 0.f;
    if (act) {
      const uint32_t n0I = nI[bI], n0D = nD[bD];
      aI = alpha[min(n0I + rI, 255u)];
      aD = alpha[min(n0D + rD, 255u)];
      wave_sync();
      if (rI + 1u == (uint32_t)__popcll(mI)) nI[bI] = min(n0I + rI + 1u, 255u);
      if (rD + 1u == (uint32_t)__popcll(mD)) nD[bD] = min(n0D + rD + 1u, 255u);
    }
    const float tau = fminf(cur.w * inv_s, tmax);
    const float tau2 = tau * tau;
    const uint32_t rmax = act ? max(rI, rD) : 0u;
    for (uint32_t r = 0;; ++r) {
      if (act && rI == r) {
        sI[bI] = fmaf(aI, cur.x - sI[bI], sI[bI]);
        sI[NI + bI] = fmaf(aI, cur.y - sI[NI + bI], sI[NI + bI]);
        sI[2 * NI + bI] = fmaf(aI, cur.z - sI[2 * NI + bI], sI[2 * NI + bI]);
      }
      if (act && rD == r) {
        sD[bD] = fmaf(aD, tau - sD[bD], sD[bD]);
        sD[ND + bD] = fmaf(aD, tau2 - sD[ND + bD], sD[ND + bD]);
      }
      wave_sync();
      if (ballot(rmax > r) == 0ull) break;
    }
  };
  // pilot reuse (Sec. 4.4): the probe's 8 pilot samples first, in octant
  // order, each into the texels of its own direction
  if (reuse) apply(prec, pbins, lane < 8);
  float4 nxt = rec0;
  uint32_t nbin = bins0;
  float2 nuv = uv0;
  if (n == 0u) at_last_chunk();
  const RayStrata strata(CHAIN ? 0u : n);
  uint32_t m = first_step_size<CHAIN>(n), step = 0;
  for (uint32_t c0 = 0; c0 < n; c0 += m, m = CHAIN ? min(64u, n - c0) : strata.size(++step)) {
    const float4 cur = nxt;
    uint32_t cbin = nbin;
    const float2 cuv = nuv;
    const uint32_t c1 = c0 + m;  // the next step's first sample
    if (c1 < n) {
      const uint32_t m1 = CHAIN ? min(64u, n - c1) : strata.size(step + 1u);
      if ((uint32_t)lane < m1) load_sample<CHAIN>(v, off, c1 + lane, nxt, nbin, nuv);
    } else {
      at_last_chunk();
    }
    const bool act = (uint32_t)lane < m;
    if (CHAIN && act) {
      // sample k: irradiance texel of d(uv_k), depth texel of -d
      const uint32_t j = c0 + (uint32_t)lane;
      const float3 d = oct_decode_dir(cuv);
      const uint32_t bI = oct_bin(oct_encode(d), RI);
      const uint32_t bD = oct_bin(oct_encode(make_float3(-d.x, -d.y, -d.z)), RD);
      cbin = bI | (bD << 16);
      if (fp.debug) {
        v.dbg_ibin[2 * (size_t)(off + j)] = (uint16_t)bI;
        v.dbg_dbin[2 * (size_t)(off + j) + 1] = (uint16_t)bD;
      }
    }
    apply(cur, cbin, act);
  }
  if (CHAIN && fp.dyn_chains > 0) {
    // dynamic updates after the static samples (Sec. 4.9): every texel of a
    // marked octant of the probe's proxy takes its texel-centre ray once,
    // with the dynamic step floor
    const int x = i % v.dx, y = (i / v.dx) % v.dy, z = i / (v.dx * v.dy);
    const uint8_t* mk = v.dyn_mark + 8 * (x / 3 + v.pdx * (y / 3 + v.pdy * (z / 3)));
    const DynTables& tb = *v.dyn_tab;
    uint32_t pre[8], acc = 2u * v.offsets[v.P] + v.dyn_off[i];
#pragma unroll
    for (int oc = 0; oc < 8; ++oc) {
      pre[oc] = acc;
      if (mk[oc]) acc += (uint32_t)(tb.start_i[oc + 1] - tb.start_i[oc]) + (uint32_t)(tb.start_d[oc + 1] - tb.start_d[oc]);
    }
    for (int k = lane; k < NI; k += 64) {
      const int oc = tb.oct_i[k];
      if (mk[oc]) plane_rgb<NI>(sI, k, v.rec[pre[oc] + tb.rank_i[k]], alpha_dyn);
    }
    for (int k = lane; k < ND; k += 64) {
      const int oc = tb.oct_d[k];
      if (mk[oc]) {
        const uint32_t ni_oc = (uint32_t)(tb.start_i[oc + 1] - tb.start_i[oc]);
        const float tau = fminf(v.rec[pre[oc] + ni_oc + tb.rank_d[k]].w * inv_s, tmax);
        plane_tau<ND>(sD, k, tau, tau * tau, alpha_dyn);
      }
    }
    wave_sync();
  }
}

// Both tiles of probe i with the border fold, and the counts, from the LDS
// planes (tab: the fold table of the planar layout).
template <int RI, int RD, bool HALF>
__device__ __forceinline__ void store_probe(const BlendIO& io, int i, const uint8_t* wbase, const uint16_t* tab) {
  using S = Store<HALF>;
  using T = typename S::T;
  using W = WaveTile<RI, RD>;
  constexpr int NI = W::NI, ND = W::ND, GI = W::GI, GD = W::GD;
  const int lane = threadIdx.x & 63;
  const float* sI = (const float*)(wbase + W::kStI);
  const float* sD = (const float*)(wbase + W::kStD);
  if constexpr (HALF) {
    // two halves per 32-bit store
    uint32_t* irr_w = (uint32_t*)io.irr_out + (size_t)i * (GI * GI * 3 / 2);
    uint32_t* dep_w = (uint32_t*)io.dep_out + (size_t)i * GD * GD;
    for (int w = lane; w < GI * GI * 3 / 2; w += 64)
      irr_w[w] = half_word(sI[tab[2 * w]], sI[tab[2 * w + 1]]);
    for (int w = lane; w < GD * GD; w += 64)
      dep_w[w] = half_word(sD[tab[GI * GI * 3 + 2 * w]], sD[tab[GI * GI * 3 + 2 * w + 1]]);
  } else {
    T* irr_out = (T*)io.irr_out + (size_t)i * GI * GI * 3;
    T* dep_out = (T*)io.dep_out + (size_t)i * GD * GD * 2;
    for (int f = lane; f < GI * GI * 3; f += 64) S::store(irr_out + f, sI[tab[f]]);
    for (int f = lane; f < GD * GD * 2; f += 64) S::store(dep_out + f, sD[tab[GI * GI * 3 + f]]);
  }
  uint32_t* ni_out = (uint32_t*)(io.irr_n_out + (size_t)i * NI);
  uint32_t* nd_out = (uint32_t*)(io.dep_n_out + (size_t)i * ND);
  const uint32_t* nI = (const uint32_t*)(sI + 3 * NI);
  const uint32_t* nD = (const uint32_t*)(sD + 2 * ND);
  for (int w = lane; w < NI / 4; w += 64)
    ni_out[w] = nI[4 * w] | (nI[4 * w + 1] << 8) | (nI[4 * w + 2] << 16) | (nI[4 * w + 3] << 24);
  for (int w = lane; w < ND / 4; w += 64)
    nd_out[w] = nD[4 * w] | (nD[4 * w + 1] << 8) | (nD[4 * w + 2] << 16) | (nD[4 * w + 3] << 24);
}

// One wave per probe, probes taken round-robin over all waves of the grid in
// the allocation's order (most chunks first). A wave first reads the probe
// index and ray range of each of its probes (up to 64 at a time, one per
// lane: two memory round trips for all of them), then takes them from its
// lanes' registers, so each probe waits on memory once, for its texels,
// counts and first records. (Also loading the next probe's texels while
// the current one is applied measured no faster and held 18 more registers.)
// order and offsets are passed apart as restrict pointers (no store of the
// kernel aliases them).
template <int RI, int RD, bool HALF, bool CHAIN>
__global__ __launch_bounds__(256) void blend_wave_kernel(VolumeView v, BlendIO io,
                                                         const int32_t* __restrict__ order,
                                                         const uint32_t* __restrict__ offsets) {
  using W = WaveTile<RI, RD>;
  using G = ProbeRegs<RI, RD, HALF, CHAIN>;
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  uint16_t* tab = (uint16_t*)(smem + 4 * W::kWaveBytes);  // planar layout
  float* alpha = (float*)(smem + 4 * W::kWaveBytes + W::kTabBytes);
  float* alpha_dyn = alpha + 256;
  build_fold_tables<RI, RD, true>(tab);
  // step weight of Alg. MovingAvgUpdate by sample count N (static and dynamic)
  for (int k = threadIdx.x; k < 256; k += blockDim.x) {
    alpha[k] = fmaxf(1.0f / (float)(k + 1), v.one_minus_h);
    if (CHAIN) alpha_dyn[k] = fmaxf(1.0f / (float)(k + 1), v.fp->dyn_one_minus_h);
  }
  __syncthreads();
  const uint32_t waves = gridDim.x * (blockDim.x >> 6);
  uint8_t* wbase = smem + (size_t)(threadIdx.x >> 6) * W::kWaveBytes;
  const uint32_t P = (uint32_t)v.P;
  const int lane = threadIdx.x & 63;
  for (int k = lane; k < W::NI + W::ND; k += 64) ((uint64_t*)(wbase + W::kMaskI))[k] = 0ull;
  wave_sync();
  const uint32_t first = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  if (first >= P) return;
  const uint32_t nq = (P - first + waves - 1u) / waves;  // this wave's probes
  // read once: a load in the loop would wait behind the probe's loads
  const bool reuse = v.fp->pilot_reuse != 0;
  for (uint32_t base = 0; base < nq; base += 64u) {
    const uint32_t k = base + (uint32_t)lane;
    int ik = 0;
    uint32_t ok = 0u, ek = 0u;
    if (k < nq) {
      ik = order[first + k * waves];
      ok = offsets[ik];
      ek = offsets[ik + 1];
    }
    const uint32_t cnt = min(64u, nq - base);
    G g;
    {
      const uint32_t off = __builtin_amdgcn_readlane(ok, 0);
      load_probe<RI, RD, HALF, CHAIN>(v, io, __builtin_amdgcn_readlane(ik, 0), off,
                                      __builtin_amdgcn_readlane(ek, 0) - off, reuse, g);
    }
    for (uint32_t kk = 0; kk < cnt; ++kk) {
      const int i = __builtin_amdgcn_readlane(ik, kk);
      const uint32_t off = __builtin_amdgcn_readlane(ok, kk);
      const uint32_t n = __builtin_amdgcn_readlane(ek, kk) - off;
      stage_probe<RI, RD, HALF, CHAIN>(g, wbase);
      wave_sync();
      blend_probe_samples<RI, RD, HALF, CHAIN>(v, i, off, n, g.rec, g.bins, g.uv, reuse, g.prec, g.pbins,
                                               wbase, alpha, alpha_dyn, []() {});
      // the next probe's loads go out before this probe's stores: a wave
      // waits for its loads in issue order, so loads behind the stores would
      // also wait for the stores to complete
      if (kk + 1u < cnt) {
        const uint32_t off1 = __builtin_amdgcn_readlane(ok, kk + 1u);
        load_probe<RI, RD, HALF, CHAIN>(v, io, __builtin_amdgcn_readlane(ik, kk + 1u), off1,
                                        __builtin_amdgcn_readlane(ek, kk + 1u) - off1, reuse, g);
      }
      store_probe<RI, RD, HALF>(io, i, wbase, tab);
      wave_sync();
    }
  }
}

// ---------------------------------------------------------------------------
// DDGI's cosine-weighted gather (Majercik et al. 2019; the update Sec. 3.1
// describes), a measured alternative to the per-sample update: every texel
// takes all of the probe's rays of the frame, weighted by max(0, c.d) with c
// its centre direction (depth: that cosine to the 50th power, the DDGI
// sharpness), and the weighted mean enters the texel with
// a = max(1/(N+1), 1-h), N counting the frames in which the texel had weight.
// One wave per probe, its texels in registers; per step of 64 rays the
// directions (recomputed from the ray index), radiance and tau are staged in
// LDS and every lane runs over them for each texel it owns.
__device__ __forceinline__ float pow50(float c) {
  const float c2 = c * c, c4 = c2 * c2, c8 = c4 * c4, c16 = c8 * c8, c32 = c16 * c16;
  return c32 * c16 * c2;
}

template <int RI, int RD, bool HALF>
__device__ void gather_probe_wave(const VolumeView& v, const BlendIO& io, int i, uint8_t* wbase,
                                  const uint16_t* tab, const float* alpha) {
  using S = Store<HALF>;
  using T = typename S::T;
  using W = WaveTile<RI, RD>;
  constexpr int NI = W::NI, ND = W::ND, SI = W::SI, SD = W::SD, GI = W::GI, GD = W::GD;
  static_assert(64 * 32 <= W::kWaveBytes, "ray staging does not fit the wave's LDS");
  const int lane = threadIdx.x & 63;
  float4* st_dir = (float4*)wbase;        // (d.x, d.y, d.z, tau)
  float4* st_rgb = st_dir + 64;           // (r, g, b, -)
  const FrameParams& fp = *v.fp;
  const T* irr_in = (const T*)io.irr_in + (size_t)i * GI * GI * 3;
  const T* dep_in = (const T*)io.dep_in + (size_t)i * GD * GD * 2;
  float3 ci[SI], cd[SD];
  float ai[SI][4], ad[SD][3];
#pragma unroll
  for (int s = 0; s < SI; ++s) {
    const int k = lane + 64 * s;
    ci[s] = k < NI ? texel_centre_dir((uint32_t)k, RI) : make_float3(0.f, 0.f, 0.f);
    ai[s][0] = ai[s][1] = ai[s][2] = ai[s][3] = 0.f;
  }
#pragma unroll
  for (int s = 0; s < SD; ++s) {
    const int k = lane + 64 * s;
    cd[s] = k < ND ? texel_centre_dir((uint32_t)k, RD) : make_float3(0.f, 0.f, 0.f);
    ad[s][0] = ad[s][1] = ad[s][2] = 0.f;
  }
  const uint32_t off = v.offsets[i];
  const uint32_t n = v.offsets[i + 1] - off;
  const float inv_s = 1.0f / v.s_diag;
  for (uint32_t c0 = 0; c0 < n; c0 += 64u) {
    const uint32_t m = min(64u, n - c0);
    if ((uint32_t)lane < m) {
      const float3 d = sf_direction(sf_point_of_ray(c0 + (uint32_t)lane, n), n, fp.R);
      const float4 r = v.rec[off + c0 + (uint32_t)lane];
      st_dir[lane] = make_float4(d.x, d.y, d.z, fminf(r.w * inv_s, v.tau_max));
      st_rgb[lane] = r;
    }
    wave_sync();
    for (uint32_t j = 0; j < m; ++j) {
      const float4 dt = st_dir[j];
      const float4 rgb = st_rgb[j];
#pragma unroll
      for (int s = 0; s < SI; ++s) {
        const float w = fmaxf(0.0f, ci[s].x * dt.x + ci[s].y * dt.y + ci[s].z * dt.z);
        ai[s][0] += w;
        ai[s][1] = fmaf(w, rgb.x, ai[s][1]);
        ai[s][2] = fmaf(w, rgb.y, ai[s][2]);
        ai[s][3] = fmaf(w, rgb.z, ai[s][3]);
      }
#pragma unroll
      for (int s = 0; s < SD; ++s) {
        const float w = pow50(fmaxf(0.0f, cd[s].x * dt.x + cd[s].y * dt.y + cd[s].z * dt.z));
        ad[s][0] += w;
        ad[s][1] = fmaf(w, dt.w, ad[s][1]);
        ad[s][2] = fmaf(w, dt.w * dt.w, ad[s][2]);
      }
    }
    wave_sync();
  }
  float* stI = (float*)wbase;
  float* stD = stI + 3 * NI;
  uint8_t* stN = (uint8_t*)(stD + 2 * ND);
#pragma unroll
  for (int s = 0; s < SI; ++s) {
    const int k = lane + 64 * s;
    if (k < NI) {
      const int iy = k / RI, ix = k - iy * RI;
      const T* p = irr_in + ((iy + 1) * GI + ix + 1) * 3;
      float V[3] = {S::load(p), S::load(p + 1), S::load(p + 2)};
      uint32_t N = io.irr_n_in[(size_t)i * NI + k];
      if (ai[s][0] > 0.0f) {
        const float inv = 1.0f / ai[s][0];
        blend_rgb(V, N, make_float4(ai[s][1] * inv, ai[s][2] * inv, ai[s][3] * inv, 0.f), alpha);
      }
      stI[3 * k] = V[0];
      stI[3 * k + 1] = V[1];
      stI[3 * k + 2] = V[2];
      stN[k] = (uint8_t)N;
    }
  }
#pragma unroll
  for (int s = 0; s < SD; ++s) {
    const int k = lane + 64 * s;
    if (k < ND) {
      const int iy = k / RD, ix = k - iy * RD;
      const T* p = dep_in + ((iy + 1) * GD + ix + 1) * 2;
      float V[2] = {S::load(p), S::load(p + 1)};
      uint32_t N = io.dep_n_in[(size_t)i * ND + k];
      if (ad[s][0] > 0.0f) {
        const float inv = 1.0f / ad[s][0], al = alpha[N];
        V[0] = fmaf(al, ad[s][1] * inv - V[0], V[0]);
        V[1] = fmaf(al, ad[s][2] * inv - V[1], V[1]);
        N = min(N + 1u, 255u);
      }
      stD[2 * k] = V[0];
      stD[2 * k + 1] = V[1];
      stN[NI + k] = (uint8_t)N;
    }
  }
  wave_sync();
  write_tiles<RI, RD, HALF>(v, io, i, stI, stD, stN, tab, lane, 64);
  wave_sync();
}

template <int RI, int RD, bool HALF>
__global__ __launch_bounds__(256) void blend_gather_kernel(VolumeView v, BlendIO io) {
  using W = WaveTile<RI, RD>;
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  uint16_t* tab = (uint16_t*)(smem + 4 * W::kWaveBytes);
  float* alpha = (float*)(smem + 4 * W::kWaveBytes + W::kTabBytes);
  build_fold_tables<RI, RD>(tab);
  for (int k = threadIdx.x; k < 256; k += blockDim.x) alpha[k] = fmaxf(1.0f / (float)(k + 1), v.one_minus_h);
  __syncthreads();
  const uint32_t waves = gridDim.x * (blockDim.x >> 6);
  uint8_t* wbase = smem + (size_t)(threadIdx.x >> 6) * W::kWaveBytes;
  for (uint32_t q = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); q < (uint32_t)v.P; q += waves)
    gather_probe_wave<RI, RD, HALF>(v, io, v.order[q], wbase, tab, alpha);
}

// ---------------------------------------------------------------------------
// Packed 32-bit texels (eq. rgbEnc, App. B): one wave per probe as in the
// binary32 kernel, the probe's interior words staged in LDS and each chunk's
// samples applied in rounds by rank. A sample decodes its texel's word,
// applies the moving average in binary32 with the step of the word's count
// and re-encodes it (the per-sample update of Alg. AtomicMovingAvg; a probe
// belongs to one wave, so no compare-and-swap is needed). Counts saturate at
// 63 (6 bits). The decoded value of every code (68.6 KB, exact values rounded
// once, built on the host) and its rounding direction sit in LDS, so one
// workgroup of kPkWaves waves holds a CU.
constexpr int kPkWaves = 16;

template <int RI, int RD>
struct PackedTile {
  static constexpr int NI = RI * RI, ND = RD * RD, NT = NI + ND, GI = RI + 2, GD = RD + 2;
  // per wave: the interior words (irradiance, then depth), then one 64-bit
  // lane mask per interior texel
  static constexpr size_t kMasks = (4 * (size_t)NT + 7) & ~(size_t)7;
  static constexpr size_t kWaveBytes = kMasks + 8 * (size_t)NT;
  static constexpr size_t kTabBytes = (2 * (GI * GI * 3 + GD * GD * 2) + 15) & ~(size_t)15;
  static constexpr size_t kBlockBytes =
      kPkWaves * kWaveBytes + kTabBytes + 64 * 4 + 4 * (size_t)kPkDecSize + 4 * (size_t)kPkUpWords;
};

template <int RI, int RD>
__device__ __forceinline__ void packed_probe(const VolumeView& v, const BlendIO& io, int i, uint32_t off,
                                             uint32_t n, uint8_t* wbase, const uint16_t* tab, const float* alpha,
                                             const float* dec, const uint32_t* up, float inv_s, float tmax) {
  using PT = PackedTile<RI, RD>;
  constexpr int NI = PT::NI, ND = PT::ND, GI = PT::GI, GD = PT::GD;
  constexpr int SI = (NI + 63) / 64, SD = (ND + 63) / 64;
  const int lane = threadIdx.x & 63;
  uint32_t* words = (uint32_t*)wbase;
  uint64_t* mk = (uint64_t*)(wbase + PT::kMasks);
  const uint32_t* irr_in = (const uint32_t*)io.irr_in + (size_t)i * GI * GI;
  const uint32_t* dep_in = (const uint32_t*)io.dep_in + (size_t)i * GD * GD;
  uint32_t wi[SI], wd[SD];
#pragma unroll
  for (int s = 0; s < SI; ++s) {
    const int k = lane + 64 * s;
    if (k < NI) {
      const int iy = k / RI, ix = k - iy * RI;
      wi[s] = irr_in[(iy + 1) * GI + ix + 1];
    }
  }
#pragma unroll
  for (int s = 0; s < SD; ++s) {
    const int k = lane + 64 * s;
    if (k < ND) {
      const int iy = k / RD, ix = k - iy * RD;
      wd[s] = dep_in[(iy + 1) * GD + ix + 1];
    }
  }
  float4 nxt = make_float4(0.f, 0.f, 0.f, 0.f);
  uint32_t nbin = 0u;
  const RayStrata strata(n);  // one stratum of rays per step
  if ((uint32_t)lane < strata.size(0u)) {
    nxt = v.rec[off + lane];
    nbin = v.ray_bins[off + lane];
  }
#pragma unroll
  for (int s = 0; s < SI; ++s)
    if (lane + 64 * s < NI) words[lane + 64 * s] = wi[s];
#pragma unroll
  for (int s = 0; s < SD; ++s)
    if (lane + 64 * s < ND) words[NI + lane + 64 * s] = wd[s];
  wave_sync();
  uint32_t m = strata.size(0u), step = 0;
  for (uint32_t c0 = 0; c0 < n; c0 += m, m = strata.size(++step)) {
    const float4 cur = nxt;
    const uint32_t cbin = nbin;
    const uint32_t c1 = c0 + m;
    if (c1 < n && (uint32_t)lane < strata.size(step + 1u)) {
      nxt = v.rec[off + c1 + lane];
      nbin = v.ray_bins[off + c1 + lane];
    }
    const bool act = (uint32_t)lane < m;
    const uint32_t bI = cbin & 0xFFFFu, bD = NI + (cbin >> 16);
    // the chunk's lanes in this lane's texels (as in the binary32 kernel)
    uint64_t mI = 0ull, mD = 0ull;
    if (act) {
      atomicOr((unsigned long long*)&mk[bI], 1ull << lane);
      atomicOr((unsigned long long*)&mk[bD], 1ull << lane);
    }
    wave_sync();
    if (act) {
      mI = mk[bI];
      mD = mk[bD];
    }
    wave_sync();
    if (act) {
      mk[bI] = 0ull;
      mk[bD] = 0ull;
    }
    const uint32_t rI = lanes_below(mI), rD = lanes_below(mD);
    const uint32_t rmax = act ? max(rI, rD) : 0u;
    const float tau = fminf(cur.w * inv_s, tmax);
    const float tau2 = tau * tau;
    for (uint32_t r = 0;; ++r) {
      if (act && rI == r) {
        const uint32_t w = words[bI];
        const uint32_t N = w >> 26;
        const float al = alpha[N];
        const float o0 = dec[kPkDecIrr9 + (w & 0x1FFu)];
        const float o1 = dec[kPkDecIrr9 + ((w >> 9) & 0x1FFu)];
        const float o2 = dec[kPkDecIrr8 + ((w >> 18) & 0xFFu)];
        const uint32_t q0 = pk_encode<9>(fmaf(al, cur.x - o0, o0), 5.0f, 15.0f, dec, up, kPkDecIrr9);
        const uint32_t q1 = pk_encode<9>(fmaf(al, cur.y - o1, o1), 5.0f, 15.0f, dec, up, kPkDecIrr9);
        const uint32_t q2 = pk_encode<8>(fmaf(al, cur.z - o2, o2), 5.0f, 15.0f, dec, up, kPkDecIrr8);
        words[bI] = q0 | (q1 << 9) | (q2 << 18) | (min(N + 1u, 63u) << 26);
      }
      if (act && rD == r) {
        const uint32_t w = words[bD];
        const uint32_t N = w >> 26;
        const float al = alpha[N];
        const float p0 = dec[kPkDecTau + (w & 0x1FFFu)];
        const float p1 = dec[kPkDecTau2 + ((w >> 13) & 0x1FFFu)];
        const uint32_t d0 = pk_encode<13>(fmaf(al, tau - p0, p0), 5.0f, 15.0f, dec, up, kPkDecTau);
        const uint32_t d1 = pk_encode<13>(fmaf(al, tau2 - p1, p1), 8.0f, 20.0f, dec, up, kPkDecTau2);
        words[bD] = d0 | (d1 << 13) | (min(N + 1u, 63u) << 26);
      }
      wave_sync();
      if (ballot(rmax > r) == 0ull) break;
    }
  }
  // both tiles with the border fold (channel 0 of a tile texel names its
  // interior texel)
  uint32_t* irr_out = (uint32_t*)io.irr_out + (size_t)i * GI * GI;
  uint32_t* dep_out = (uint32_t*)io.dep_out + (size_t)i * GD * GD;
  for (int f = lane; f < GI * GI; f += 64) irr_out[f] = words[tab[3 * f] / 3];
  for (int f = lane; f < GD * GD; f += 64) dep_out[f] = words[NI + tab[GI * GI * 3 + 2 * f] / 2];
  wave_sync();
}

template <int RI, int RD>
__global__ __launch_bounds__(kPkWaves * 64) void blend_packed_kernel(VolumeView v, BlendIO io,
                                                                    const int32_t* __restrict__ order,
                                                                    const uint32_t* __restrict__ offsets) {
  using PT = PackedTile<RI, RD>;
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  uint16_t* tab = (uint16_t*)(smem + kPkWaves * PT::kWaveBytes);
  float* alpha = (float*)(smem + kPkWaves * PT::kWaveBytes + PT::kTabBytes);
  float* dec = alpha + 64;
  uint32_t* up = (uint32_t*)(dec + kPkDecSize);
  build_fold_tables<RI, RD>(tab);
  // step weight of Alg. MovingAvgUpdate by the word's count N <= 63
  for (int k = threadIdx.x; k < 64; k += blockDim.x) alpha[k] = fmaxf(1.0f / (float)(k + 1), v.one_minus_h);
  for (int k = threadIdx.x; k < kPkDecSize; k += blockDim.x) dec[k] = v.pk_dec[k];
  for (int k = threadIdx.x; k < kPkUpWords; k += blockDim.x) up[k] = v.pk_up[k];
  uint8_t* wbase = smem + (size_t)(threadIdx.x >> 6) * PT::kWaveBytes;
  const int lane = threadIdx.x & 63;
  for (int k = lane; k < PT::NT; k += 64) ((uint64_t*)(wbase + PT::kMasks))[k] = 0ull;
  __syncthreads();
  const uint32_t waves = gridDim.x * (blockDim.x >> 6);
  const uint32_t P = (uint32_t)v.P;
  const uint32_t first = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  if (first >= P) return;
  const uint32_t nq = (P - first + waves - 1u) / waves;
  const float inv_s = 1.0f / v.s_diag;
  const float tmax = v.tau_max;
  for (uint32_t base = 0; base < nq; base += 64u) {
    const uint32_t k = base + (uint32_t)lane;
    int ik = 0;
    uint32_t ok = 0u, ek = 0u;
    if (k < nq) {
      ik = order[first + k * waves];
      ok = offsets[ik];
      ek = offsets[ik + 1];
    }
    const uint32_t cnt = min(64u, nq - base);
    for (uint32_t kk = 0; kk < cnt; ++kk) {
      const uint32_t off = __builtin_amdgcn_readlane(ok, kk);
      packed_probe<RI, RD>(v, io, __builtin_amdgcn_readlane(ik, kk), off, __builtin_amdgcn_readlane(ek, kk) - off,
                           wbase, tab, alpha, dec, up, inv_s, tmax);
    }
  }
}

// Round trip of n binary32 values through one packed channel with the
// blend's encoder and tables: the code of each value and the value it
// decodes to.
__global__ void pack_channel_kernel(const float* __restrict__ x, int64_t n, int channel,
                                    const float* __restrict__ dec, const uint32_t* __restrict__ up,
                                    uint32_t* __restrict__ codes, float* __restrict__ decoded) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float v = x[i];
  uint32_t q;
  int base;
  if (channel == 0) {
    q = pk_encode<9>(v, 5.0f, 15.0f, dec, up, kPkDecIrr9);
    base = kPkDecIrr9;
  } else if (channel == 1) {
    q = pk_encode<8>(v, 5.0f, 15.0f, dec, up, kPkDecIrr8);
    base = kPkDecIrr8;
  } else if (channel == 2) {
    q = pk_encode<13>(v, 5.0f, 15.0f, dec, up, kPkDecTau);
    base = kPkDecTau;
  } else {
    q = pk_encode<13>(v, 8.0f, 20.0f, dec, up, kPkDecTau2);
    base = kPkDecTau2;
  }
  if (codes) codes[i] = q;
  if (decoded) decoded[i] = dec[base + q];
}

hipError_t launch_pack_channel(const float* x, int64_t n, int channel, const float* dec, const uint32_t* up,
                               uint32_t* codes, float* decoded, hipStream_t s) {
  const int64_t g = (n + 255) / 256;
  hipLaunchKernelGGL(pack_channel_kernel, dim3((uint32_t)g), dim3(256), 0, s, x, n, channel, dec, up, codes, decoded);
  return hipGetLastError();
}

bool blend_wave_supported(const VolumeView& v) {
  return (v.irr_res == 8 && v.dep_res == 16) || (v.irr_res == 16 && v.dep_res == 16);
}

size_t blend_lds_bytes(const VolumeView& v, int chunk) {
  return blend_layout(v.irr_res, v.dep_res, chunk, nullptr, nullptr);
}

template <int RI, int RD>
static void launch_sched(const VolumeView& v, const BlendIO& io, hipStream_t s, int storage, int grid,
                         bool chain, bool gather) {
  using W = WaveTile<RI, RD>;
  const size_t lds = W::kBlockBytes, lds_pk = PackedTile<RI, RD>::kBlockBytes;
  if (gather && storage == ADGI_FP16)
    hipLaunchKernelGGL((blend_gather_kernel<RI, RD, true>), dim3(grid), dim3(256), lds, s, v, io);
  else if (gather)
    hipLaunchKernelGGL((blend_gather_kernel<RI, RD, false>), dim3(grid), dim3(256), lds, s, v, io);
  else if (chain && storage == ADGI_FP16)
    hipLaunchKernelGGL((blend_wave_kernel<RI, RD, true, true>), dim3(grid), dim3(256), lds, s, v, io, v.order, v.offsets);
  else if (chain)
    hipLaunchKernelGGL((blend_wave_kernel<RI, RD, false, true>), dim3(grid), dim3(256), lds, s, v, io, v.order, v.offsets);
  else if (storage == ADGI_PACKED)
    hipLaunchKernelGGL((blend_packed_kernel<RI, RD>), dim3(grid), dim3(kPkWaves * 64), lds_pk, s, v, io, v.order,
                       v.offsets);
  else if (storage == ADGI_FP16)
    hipLaunchKernelGGL((blend_wave_kernel<RI, RD, true, false>), dim3(grid), dim3(256), lds, s, v, io, v.order, v.offsets);
  else
    hipLaunchKernelGGL((blend_wave_kernel<RI, RD, false, false>), dim3(grid), dim3(256), lds, s, v, io, v.order, v.offsets);
}

// The packed kernel's workgroup takes more LDS than the default dynamic
// limit: raised once per tile shape, before any launch (and outside graph
// capture).
hipError_t blend_prepare(int irr_res, int dep_res, int storage) {
  if (storage != ADGI_PACKED) return hipSuccess;
  if (irr_res == 8 && dep_res == 16)
    return hipFuncSetAttribute((const void*)blend_packed_kernel<6, 14>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)PackedTile<6, 14>::kBlockBytes);
  if (irr_res == 16 && dep_res == 16)
    return hipFuncSetAttribute((const void*)blend_packed_kernel<14, 14>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)PackedTile<14, 14>::kBlockBytes);
  return hipErrorInvalidValue;
}

hipError_t launch_blend(const VolumeView& v, const BlendIO& io, hipStream_t s, int storage, int chunk,
                        int grid, bool chain, bool gather) {
  if (chunk == 0 || storage == ADGI_PACKED || chain || gather) {  // wave-per-probe kernels, most-rays-first order
    if (v.irr_res == 8 && v.dep_res == 16) launch_sched<6, 14>(v, io, s, storage, grid, chain, gather);
    else if (v.irr_res == 16 && v.dep_res == 16) launch_sched<14, 14>(v, io, s, storage, grid, chain, gather);
    else return hipErrorInvalidValue;
    return hipGetLastError();
  }
  const bool fp16 = storage == ADGI_FP16;
  size_t lds = blend_lds_bytes(v, chunk);
  if (fp16)
    hipLaunchKernelGGL(blend_kernel<true>, dim3(v.P), dim3(256), lds, s, v, io, chunk);
  else
    hipLaunchKernelGGL(blend_kernel<false>, dim3(v.P), dim3(256), lds, s, v, io, chunk);
  return hipGetLastError();
}

}  // namespace adgi
