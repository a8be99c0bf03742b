// query.hip - irradiance at shading points from the probe volume (the
// deferred-shading lookup of Sec. 3.1: the 8 probes of the grid cell around
// the point, interpolated, with DDGI's weights).
//
// Per probe: trilinear weight x smooth backface term (((dir.n + 1)/2)^2 + 0.2,
// dir from the point to the probe) x one-sided Chebyshev visibility (when the
// point is farther from the probe than the mean of the probe's depth moments
// towards it: (var / (var + (r - mean)^2))^3), floored at 1e-6 before the
// trilinear factor; the result is the weighted mean of the probes'
// irradiance in the normal's direction. Texels are read bilinearly from the
// bordered tiles. One thread per point, FP32 arithmetic.
#include <hip/hip_fp16.h>

#include "adgi_internal.hpp"

namespace adgi {

template <bool HALF>
__device__ __forceinline__ float tex_load(const void* base, size_t i) {
  if (HALF) return __half2float(((const __half*)base)[i]);
  return ((const float*)base)[i];
}

// Bilinear read of C channels of the bordered r x r map of `tile` (element
// offset) at the direction d.
template <bool HALF, int C>
__device__ __forceinline__ void tile_bilinear(const void* tex, size_t tile, int r, float3 d, float* out) {
  const float2 uv = oct_encode(d);
  const float fx = fmaf((uv.x + 1.0f) * 0.5f, (float)r, -0.5f), fy = fmaf((uv.y + 1.0f) * 0.5f, (float)r, -0.5f);
  const float x0 = fminf(fmaxf(floorf(fx), -1.0f), (float)(r - 1));
  const float y0 = fminf(fmaxf(floorf(fy), -1.0f), (float)(r - 1));
  const float ax = fx - x0, ay = fy - y0;
  const int X = (int)x0 + 1, Y = (int)y0 + 1, g = r + 2;
  const size_t e00 = tile + (size_t)(Y * g + X) * C, e10 = tile + (size_t)((Y + 1) * g + X) * C;
#pragma unroll
  for (int k = 0; k < C; ++k) {
    const float v00 = tex_load<HALF>(tex, e00 + k), v01 = tex_load<HALF>(tex, e00 + C + k);
    const float v10 = tex_load<HALF>(tex, e10 + k), v11 = tex_load<HALF>(tex, e10 + C + k);
    out[k] = fmaf(ay, fmaf(ax, v11 - v10, v10) - fmaf(ax, v01 - v00, v00), fmaf(ax, v01 - v00, v00));
  }
}

template <bool HALF>
__global__ void query_kernel(VolumeView v, const void* irr, const void* dep, const float* __restrict__ pts,
                             const float* __restrict__ nrm, float* __restrict__ out, int64_t count) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= count) return;
  const float x[3] = {pts[3 * q], pts[3 * q + 1], pts[3 * q + 2]};
  const float3 n = make_float3(nrm[3 * q], nrm[3 * q + 1], nrm[3 * q + 2]);
  const float o[3] = {v.ox, v.oy, v.oz}, s[3] = {v.sx, v.sy, v.sz};
  const int dims[3] = {v.dx, v.dy, v.dz};
  int base[3];
  float al[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (dims[a] == 1) {
      base[a] = 0;
      al[a] = 0.0f;
      continue;
    }
    const float f = (x[a] - o[a]) / s[a];
    const float b = fminf(fmaxf(floorf(f), 0.0f), (float)(dims[a] - 2));
    base[a] = (int)b;
    al[a] = fminf(fmaxf(f - b, 0.0f), 1.0f);
  }
  const int ri = v.irr_res - 2, rd = v.dep_res - 2;
  const float inv_s = 1.0f / v.s_diag;
  float sum[3] = {0.f, 0.f, 0.f}, wsum = 0.f;
  for (int corner = 0; corner < 8; ++corner) {
    int idx[3];
    float tri = 1.0f;
    bool skip = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int oc = (corner >> a) & 1;
      skip = skip || (oc && dims[a] == 1);
      idx[a] = base[a] + oc;
      tri *= oc ? al[a] : 1.0f - al[a];
    }
    if (skip) continue;
    const int pr = idx[0] + v.dx * (idx[1] + v.dy * idx[2]);
    const float3 p = make_float3(fmaf((float)idx[0], v.sx, v.ox), fmaf((float)idx[1], v.sy, v.oy),
                                 fmaf((float)idx[2], v.sz, v.oz));
    float3 dir = make_float3(p.x - x[0], p.y - x[1], p.z - x[2]);
    const float len = sqrtf(dir.x * dir.x + dir.y * dir.y + dir.z * dir.z);
    float w = 1.0f;
    if (len > 0.0f) {
      const float il = 1.0f / len;
      dir = make_float3(dir.x * il, dir.y * il, dir.z * il);
      const float c = (dir.x * n.x + dir.y * n.y + dir.z * n.z + 1.0f) * 0.5f;
      w *= fmaf(c, c, 0.2f);
      float m[2];
      tile_bilinear<HALF, 2>(dep, (size_t)pr * (rd + 2) * (rd + 2) * 2, rd, make_float3(-dir.x, -dir.y, -dir.z), m);
      const float rr = len * inv_s;
      if (rr > m[0]) {
        const float var = fabsf(m[1] - m[0] * m[0]);
        const float dd = rr - m[0];
        const float cheb = var / (var + dd * dd);
        w *= cheb * cheb * cheb;
      }
    }
    w = fmaxf(w, 1e-6f) * tri;
    float e[3];
    tile_bilinear<HALF, 3>(irr, (size_t)pr * (ri + 2) * (ri + 2) * 3, ri, n, e);
#pragma unroll
    for (int k = 0; k < 3; ++k) sum[k] = fmaf(w, e[k], sum[k]);
    wsum += w;
  }
  const float inv = wsum > 0.0f ? 1.0f / wsum : 0.0f;
#pragma unroll
  for (int k = 0; k < 3; ++k) out[3 * q + k] = sum[k] * inv;
}

hipError_t launch_query(const VolumeView& v, bool fp16, const void* irr, const void* dep, const float* pts,
                        const float* nrm, float* out, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const dim3 grid((unsigned)((count + 255) / 256));
  if (fp16)
    hipLaunchKernelGGL(query_kernel<true>, grid, dim3(256), 0, s, v, irr, dep, pts, nrm, out, count);
  else
    hipLaunchKernelGGL(query_kernel<false>, grid, dim3(256), 0, s, v, irr, dep, pts, nrm, out, count);
  return hipGetLastError();
}

}  // namespace adgi
