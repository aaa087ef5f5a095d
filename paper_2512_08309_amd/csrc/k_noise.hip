// Seed noise G(seed, x, y, c, step) for J_T (formal appendix, "Seeds and
// initial noise": J_T is a deterministic function of seed and pixel).
//
// Specification (shared with any other implementation, bit for bit):
//  * Philox4x32-10 (Salmon et al., SC'11): key (lo32(seed), hi32(seed)),
//    counter (u32 x, u32 y, step, c/4); outputs r0..r3.  Channels 4q, 4q+1
//    take (r0, r1), channels 4q+2, 4q+3 take (r2, r3).
//  * u = (2*(r >> 9) + 1) * 2^-24 (exact).
//  * Box-Muller in binary32, every operation a single IEEE operation, no
//    contraction: rho = sqrt(-2 ln ua), angle 2 pi ub; even channel
//    rho*cos, odd channel rho*sin.
//  * ln by the atanh series on m in [sqrt(1/2), sqrt(2)) (6 terms, Horner),
//    sin / cos by quadrant reduction v = 4 ub, q = rint(v), theta =
//    (v - q) * pi/2, Taylor to theta^11 / theta^10 (Horner).
// The HBM-bound part is the store: one Philox block feeds four channels.
#include "td_internal.h"

namespace td {
namespace {

#pragma clang fp contract(off)

__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint32_t hi0 = __umulhi(M0, c[0]), lo0 = M0 * c[0];
    uint32_t hi1 = __umulhi(M1, c[2]), lo1 = M1 * c[2];
    uint32_t n0 = hi1 ^ c[1] ^ k0;
    uint32_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    k0 += W0; k1 += W1;
  }
}

__device__ __forceinline__ float word_to_uniform(uint32_t r) {
  float k = (float)((r >> 9) * 2u + 1u);       // < 2^24, exact
  return k * 0x1p-24f;
}

__device__ __forceinline__ float series_ln(float u) {
  uint32_t bits = __float_as_uint(u);
  int e = (int)(bits >> 23) - 127;
  float m = __uint_as_float((bits & 0x7FFFFFu) | 0x3F800000u);
  if (m >= 0x1.6a09e6p+0f) {                   // sqrt(2) rounded
    m = m * 0.5f;
    e += 1;
  }
  float s = (m - 1.0f) / (m + 1.0f);
  float s2 = s * s;
  float p = 0x1.745d18p-4f;                    // 1/11
  p = p * s2; p = p + 0x1.c71c72p-4f;          // 1/9
  p = p * s2; p = p + 0x1.24924ap-3f;          // 1/7
  p = p * s2; p = p + 0x1.99999ap-3f;          // 1/5
  p = p * s2; p = p + 0x1.555556p-2f;          // 1/3
  p = p * s2; p = p + 1.0f;
  float t = s * p;
  float lnm = t + t;
  float el = (float)e * 0x1.62e430p-1f;        // ln 2 rounded
  return el + lnm;
}

__device__ __forceinline__ void sincos_turn(float ub, float* sn_out, float* cs_out) {
  float v = ub * 4.0f;
  float q = __builtin_rintf(v);
  float a = v - q;
  float th = a * 0x1.921fb6p+0f;               // pi/2 rounded
  float t2 = th * th;
  float ps = -0x1.ae6456p-26f;                 // -1/11!
  ps = ps * t2; ps = ps + 0x1.71de3ap-19f;     //  1/9!
  ps = ps * t2; ps = ps + -0x1.a01a02p-13f;    // -1/7!
  ps = ps * t2; ps = ps + 0x1.111112p-7f;      //  1/5!
  ps = ps * t2; ps = ps + -0x1.555556p-3f;     // -1/3!
  ps = ps * t2; ps = ps + 1.0f;
  float sn = ps * th;
  float pc = -0x1.27e4fcp-22f;                 // -1/10!
  pc = pc * t2; pc = pc + 0x1.a01a02p-16f;     //  1/8!
  pc = pc * t2; pc = pc + -0x1.6c16c2p-10f;    // -1/6!
  pc = pc * t2; pc = pc + 0x1.555556p-5f;      //  1/4!
  pc = pc * t2; pc = pc + -0.5f;               // -1/2!
  pc = pc * t2; pc = pc + 1.0f;
  float cs = pc;
  int quad = ((int)q) & 3;
  float s_out, c_out;
  if (quad == 0) { s_out = sn; c_out = cs; }
  else if (quad == 1) { s_out = cs; c_out = -sn; }
  else if (quad == 2) { s_out = -sn; c_out = -cs; }
  else { s_out = -cs; c_out = sn; }
  *sn_out = s_out;
  *cs_out = c_out;
}

__device__ __forceinline__ void box_muller(uint32_t ra, uint32_t rb, float* ev, float* od) {
  float ua = word_to_uniform(ra);
  float ub = word_to_uniform(rb);
  float l = series_ln(ua);
  float rho = __builtin_sqrtf(-2.0f * l);
  float sn, cs;
  sincos_turn(ub, &sn, &cs);
  *ev = rho * cs;
  *od = rho * sn;
}

__global__ __launch_bounds__(256) void noise_kernel(uint32_t k0, uint32_t k1, int64_t x0, int64_t y0,
                                                    int w, int h, int C, uint32_t step, float scale,
                                                    int layout, int accumulate, float* __restrict__ out) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)w * h) return;
  int ry = (int)(idx / w), rx = (int)(idx - (int64_t)ry * w);
  uint32_t ux = (uint32_t)(uint64_t)(x0 + rx);
  uint32_t uy = (uint32_t)(uint64_t)(y0 + ry);
  for (int cq = 0; cq < C; cq += 4) {
    uint32_t c[4] = {ux, uy, step, (uint32_t)(cq >> 2)};
    philox4x32_10(c, k0, k1);
    float z[4];
    box_muller(c[0], c[1], &z[0], &z[1]);
    box_muller(c[2], c[3], &z[2], &z[3]);
    int nc = C - cq < 4 ? C - cq : 4;
    if (accumulate) {
      for (int j = 0; j < nc; ++j) {
        float* o = layout == 0 ? out + idx * C + cq + j : out + (int64_t)(cq + j) * w * h + idx;
        *o = *o + z[j] * scale;
      }
    } else if (layout == 0) {
      float* o = out + idx * C + cq;
      if (nc == 4 && (C & 3) == 0) {
        *reinterpret_cast<float4*>(o) = make_float4(z[0] * scale, z[1] * scale, z[2] * scale, z[3] * scale);
      } else {
        for (int j = 0; j < nc; ++j) o[j] = z[j] * scale;
      }
    } else {
      for (int j = 0; j < nc; ++j) out[(int64_t)(cq + j) * w * h + idx] = z[j] * scale;
    }
  }
}

__global__ void fill_kernel(float* p, size_t n, float v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

void launch_noise(hipStream_t st, uint64_t seed, int64_t x0, int64_t y0, int w, int h, int C,
                  uint32_t step, float scale, int layout, float* out, int accumulate) {
  int64_t n = (int64_t)w * h;
  if (n == 0) return;
  int blocks = (int)((n + 255) / 256);
  prof_begin(st);
  hipLaunchKernelGGL(noise_kernel, dim3(blocks), dim3(256), 0, st, (uint32_t)(seed & 0xFFFFFFFFu),
                     (uint32_t)(seed >> 32), x0, y0, w, h, C, step, scale, layout, accumulate, out);
  TD_LAUNCHED();
  prof_end(st, K_NOISE, 0.0, (accumulate ? 8.0 : 4.0) * n * C);
}

void launch_fill(hipStream_t st, float* p, size_t n, float v) {
  if (!n) return;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  TD_LAUNCHED();
}

}  // namespace td
