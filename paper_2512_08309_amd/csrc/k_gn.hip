// GroupNorm statistics per (window, group), turned into a per-channel
// affine (scale = gamma * rstd, shift = beta - mean * scale) that the
// consuming convolution applies while staging its input.
//
// Input is the same virtual tensor the convolution reads: concat of src0
// (optionally stored at half resolution and nearest-upsampled; its pixels
// then count four times, which leaves mean and biased variance unchanged)
// and src1.  Sums and sums of squares are accumulated in FP64 in a fixed
// order (per thread, then per channel over threads, then per group, then
// over pixel chunks), so the statistics are deterministic and free of the
// cancellation that FP32 E[x^2] - E[x]^2 would suffer.  The pass reads the
// tensor once: HBM-bound.
#include "td_internal.h"

namespace td {
namespace {

constexpr int kMaxCin = 1024;
constexpr int kWinMaxCin = 512;
constexpr int kWinMaxElems = 32768;   // 16 pixels x 8 channels per thread

__host__ __device__ inline int gn_nchunk(int lh, int lw, int cin, int up0) {
  long hw = 1L << (lh + lw);
  int n = 1;
  while (n < 16 && hw * cin / (2L * n) >= 32768 && hw / (2L * n) >= (up0 ? 4 : 1)) n *= 2;
  return n;
}

__global__ __launch_bounds__(256) void gn_partial_kernel(GnArgs a, int nchunk) {
  __shared__ double ls[256 * 4];
  __shared__ double lq[256 * 4];
  __shared__ double cs[kMaxCin];
  __shared__ double cq[kMaxCin];
  const int tid = threadIdx.x;
  const int b = blockIdx.y, chunk = blockIdx.x;
  const int hw = 1 << (a.lh + a.lw);
  const int cin = a.c0 + a.c1;
  for (int seg = 0; seg < 2; ++seg) {
    const int Cs = seg == 0 ? a.c0 : a.c1;
    if (Cs == 0) continue;
    const float* src = seg == 0 ? a.src0 : a.src1;
    const int up = (seg == 0 && a.up0) ? 1 : 0;
    const int npix_img = up ? hw >> 2 : hw;
    const int per = npix_img / nchunk;
    const int p0 = chunk * per;
    const int nq = Cs / 4, npl = 256 / nq;
    const int q = tid % nq, pl = tid / nq;
    double s[4] = {0, 0, 0, 0}, sq[4] = {0, 0, 0, 0};
    const float* base = src + ((size_t)b * npix_img + p0) * Cs + 4 * q;
    // unrolled so that several loads are in flight; every sum still takes
    // its terms in pixel order
#pragma unroll 8
    for (int p = pl; p < per; p += npl) {
      float4 v = *reinterpret_cast<const float4*>(base + (size_t)p * Cs);
      double d0 = v.x, d1 = v.y, d2 = v.z, d3 = v.w;
      s[0] += d0; s[1] += d1; s[2] += d2; s[3] += d3;
      sq[0] += d0 * d0; sq[1] += d1 * d1; sq[2] += d2 * d2; sq[3] += d3 * d3;
    }
    for (int j = 0; j < 4; ++j) {
      ls[tid * 4 + j] = s[j];
      lq[tid * 4 + j] = sq[j];
    }
    __syncthreads();
    const double wgt = up ? 4.0 : 1.0;
    for (int c = tid; c < Cs; c += 256) {
      double ts = 0, tq = 0;
      for (int l = 0; l < npl; ++l) {
        ts += ls[(l * nq + c / 4) * 4 + (c & 3)];
        tq += lq[(l * nq + c / 4) * 4 + (c & 3)];
      }
      const int cg = (seg == 0 ? 0 : a.c0) + c;
      cs[cg] = ts * wgt;
      cq[cg] = tq * wgt;
    }
    __syncthreads();
  }
  const int cgp = cin / a.groups;
  for (int g = tid; g < a.groups; g += 256) {
    double ts = 0, tq = 0;
    for (int c = g * cgp; c < (g + 1) * cgp; ++c) {
      ts += cs[c];
      tq += cq[c];
    }
    double* o = a.partial + (((size_t)b * nchunk + chunk) * a.groups + g) * 2;
    o[0] = ts;
    o[1] = tq;
  }
}

__global__ __launch_bounds__(256) void gn_finalize_kernel(GnArgs a, int nchunk) {
  const int b = blockIdx.x;
  const int cin = a.c0 + a.c1;
  const int cgp = cin / a.groups;
  const double n = (double)(1L << (a.lh + a.lw)) * cgp;
  for (int c = threadIdx.x; c < cin; c += blockDim.x) {
    const int g = c / cgp;
    double ts = 0, tq = 0;
    for (int k = 0; k < nchunk; ++k) {
      const double* p = a.partial + (((size_t)b * nchunk + k) * a.groups + g) * 2;
      ts += p[0];
      tq += p[1];
    }
    double mean = ts / n;
    double var = tq / n - mean * mean;
    if (var < 0) var = 0;
    double rstd = 1.0 / sqrt(var + (double)a.eps);
    if (a.mean && c % cgp == 0) {
      a.mean[(size_t)b * a.groups + g] = (float)mean;
      a.rstd[(size_t)b * a.groups + g] = (float)rstd;
    }
    double sc = (double)a.gamma[c] * rstd;
    a.scale[(size_t)b * cin + c] = (float)sc;
    a.shift[(size_t)b * cin + c] = (float)((double)a.beta[c] - mean * sc);
  }
}

// The affine of a GroupNorm over concat(src0 (optionally upsampled), src1)
// from per-channel sums written by the producers of src0 and src1
// ([nb][slots][C][2], one slot per tile of the window): per window, each
// group's sums over its channels (channel order), each channel's over its
// slots (slot order), an upsampled source's terms weighted by 4 (its pixels
// count four times); then the same affine as gn_finalize_kernel.
__global__ __launch_bounds__(256) void gn_finalize_ch_kernel(GnArgs a, const double* ch0, int slots0,
                                                             const double* ch1, int slots1) {
  __shared__ double gs1[kMaxCin], gs2[kMaxCin];
  const int b = blockIdx.x;
  const int cin = a.c0 + a.c1;
  const int cgp = cin / a.groups;
  for (int g = threadIdx.x; g < a.groups; g += blockDim.x) {
    double ts = 0, tq = 0;
    for (int c = g * cgp; c < (g + 1) * cgp; ++c) {
      const bool first = c < a.c0;
      const int C = first ? a.c0 : a.c1, slots = first ? slots0 : slots1;
      const double* p = (first ? ch0 : ch1) + ((size_t)b * slots * C + (first ? c : c - a.c0)) * 2;
      double cs = 0, cq = 0;
      for (int k = 0; k < slots; ++k) {
        cs += p[(size_t)k * C * 2];
        cq += p[(size_t)k * C * 2 + 1];
      }
      const double w = (first && a.up0) ? 4.0 : 1.0;
      ts += cs * w;
      tq += cq * w;
    }
    gs1[g] = ts;
    gs2[g] = tq;
  }
  __syncthreads();
  const double n = (double)(1L << (a.lh + a.lw)) * cgp;
  for (int c = threadIdx.x; c < cin; c += blockDim.x) {
    const int g = c / cgp;
    const double mean = gs1[g] / n;
    double var = gs2[g] / n - mean * mean;
    if (var < 0) var = 0;
    const double rstd = 1.0 / sqrt(var + (double)a.eps);
    if (a.mean && c % cgp == 0) {
      a.mean[(size_t)b * a.groups + g] = (float)mean;
      a.rstd[(size_t)b * a.groups + g] = (float)rstd;
    }
    const double sc = (double)a.gamma[c] * rstd;
    a.scale[(size_t)b * cin + c] = (float)sc;
    a.shift[(size_t)b * cin + c] = (float)((double)a.beta[c] - mean * sc);
  }
}

__device__ __forceinline__ float silu_f(float v) { return v * __builtin_amdgcn_rcpf(1.0f + __expf(-v)); }

__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
  typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
  bf2 p = {(__bf16)lo, (__bf16)hi};
  return __builtin_bit_cast(uint32_t, p);
}

// One thread per (pixel, 8 channels): reads the virtual conv input in FP32,
// applies the GroupNorm affine (and SiLU), writes 16 bytes of BF16 or 32
// bytes of FP32; with a.raw also the input itself as BF16 (the operand of a
// residual block's 1x1 skip convolution), from the same read.
template <bool F32>
__global__ __launch_bounds__(256) void apply_kernel(ApplyArgs a) {
  const int cin = a.c0 + a.c1, q8 = cin / 8;
  const int lhw = a.lh + a.lw;
  const size_t n = ((size_t)a.nb << lhw) * q8;
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const int q = (int)(e % q8);
  const size_t p = e / q8;
  const int b = (int)(p >> lhw);
  const int y = (int)((p >> a.lw) & ((1 << a.lh) - 1)), x = (int)(p & ((1 << a.lw) - 1));
  const int c = 8 * q;
  const float* s;
  if (c < a.c0) {
    if (a.up0)
      s = a.src0 + ((((size_t)b << (lhw - 2)) + ((size_t)(y >> 1) << (a.lw - 1)) + (x >> 1)) * a.c0 + c);
    else
      s = a.src0 + (p * a.c0 + c);
  } else {
    s = a.src1 + (p * a.c1 + (c - a.c0));
  }
  float4 v0 = *reinterpret_cast<const float4*>(s);
  float4 v1 = *reinterpret_cast<const float4*>(s + 4);
  float v[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
  if (!F32 && a.raw) {
    const uint4 r = {pack_bf16(v[0], v[1]), pack_bf16(v[2], v[3]), pack_bf16(v[4], v[5]), pack_bf16(v[6], v[7])};
    *reinterpret_cast<uint4*>(a.raw + p * cin + c) = r;
  }
  if (a.act) {
    const float* sc = a.scale + (size_t)b * cin + c;
    const float* sh = a.shift + (size_t)b * cin + c;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      v[j] = v[j] * sc[j] + sh[j];
      if (a.act == 2) v[j] = silu_f(v[j]);
    }
  }
  if constexpr (F32) {
    float4* o = reinterpret_cast<float4*>(a.out32 + p * cin + c);
    o[0] = make_float4(v[0], v[1], v[2], v[3]);
    o[1] = make_float4(v[4], v[5], v[6], v[7]);
  } else {
    uint4 o = {pack_bf16(v[0], v[1]), pack_bf16(v[2], v[3]), pack_bf16(v[4], v[5]), pack_bf16(v[6], v[7])};
    *reinterpret_cast<uint4*>(a.out + p * cin + c) = o;
  }
}

// act(x * scale + shift) of a BF16 tensor into BF16: a thread takes 8
// channels of 4 consecutive pixels of one window, so that each scale / shift
// pair is loaded once per 4 pixels.
__global__ __launch_bounds__(256) void apply_bf16_kernel(const uint4* __restrict__ src, int C, const float* scale,
                                                         const float* shift, int act, int lhw, size_t n4,
                                                         uint4* __restrict__ out) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n4) return;
  const int q8 = C / 8;
  const int q = (int)(e % q8);
  const size_t p0 = 4 * (e / q8);   // first of the thread's pixels
  const int c = 8 * q;
  const int b = (int)(p0 >> lhw);
  uint4 u[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) u[i] = src[(p0 + i) * q8 + q];
  float sc[8], sh[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    sc[k] = scale[(size_t)b * C + c + k];
    sh[k] = shift[(size_t)b * C + c + k];
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t w[4] = {u[i].x, u[i].y, u[i].z, u[i].w};
    uint32_t o[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      float v0 = __uint_as_float(w[k] << 16), v1 = __uint_as_float(w[k] & 0xffff0000u);
      v0 = v0 * sc[2 * k] + sh[2 * k];
      v1 = v1 * sc[2 * k + 1] + sh[2 * k + 1];
      if (act == 2) {
        v0 = silu_f(v0);
        v1 = silu_f(v1);
      }
      o[k] = pack_bf16(v0, v1);
    }
    out[(p0 + i) * q8 + q] = uint4{o[0], o[1], o[2], o[3]};
  }
}

// GroupNorm of whole windows in one pass, for windows whose virtual input
// (h * w * C_in elements) fits in the registers of one workgroup: the
// workgroup of window b loads it once, reduces per-channel sums and sums of
// squares in FP64 (per thread over its pixels, then over threads in a fixed
// order, then over the group's channels), forms the same affine as
// gn_finalize_kernel and writes act(x * scale + shift) as BF16 or FP32.
// One launch and one read instead of statistics, finalize and apply.
template <int NS, bool F32>
__global__ __launch_bounds__(256) void gn_apply_window_kernel(GnArgs g, int act, uint16_t* out, float* out32) {
  __shared__ double ls[256 * 8];
  __shared__ double lq[256 * 8];
  __shared__ double cs[kWinMaxCin];
  __shared__ double cq[kWinMaxCin];
  __shared__ double gmean[kWinMaxCin], grstd[kWinMaxCin];
  __shared__ float scl[kWinMaxCin], shf[kWinMaxCin];
  const int tid = threadIdx.x, b = blockIdx.x;
  const int cin = g.c0 + g.c1, q8 = cin / 8;
  const int lhw = g.lh + g.lw, hw = 1 << lhw;
  const int q = tid % q8, c = 8 * q, pstep = 256 / q8;
  const int ns = hw / pstep;   // pixels per thread (<= NS)
  float v[NS][8];
  double s[8] = {0, 0, 0, 0, 0, 0, 0, 0}, sq[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    if (k < ns) {
    const int p = tid / q8 + k * pstep;
    const int y = p >> g.lw, x = p & ((1 << g.lw) - 1);
    const float* src;
    if (c < g.c0) {
      if (g.up0)
        src = g.src0 + ((((size_t)b << (lhw - 2)) + ((size_t)(y >> 1) << (g.lw - 1)) + (x >> 1)) * g.c0 + c);
      else
        src = g.src0 + (((size_t)b << lhw) + p) * g.c0 + c;
    } else {
      src = g.src1 + (((size_t)b << lhw) + p) * g.c1 + (c - g.c0);
    }
    const float4 v0 = *reinterpret_cast<const float4*>(src);
    const float4 v1 = *reinterpret_cast<const float4*>(src + 4);
    v[k][0] = v0.x; v[k][1] = v0.y; v[k][2] = v0.z; v[k][3] = v0.w;
    v[k][4] = v1.x; v[k][5] = v1.y; v[k][6] = v1.z; v[k][7] = v1.w;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const double d = v[k][j];
      s[j] += d;
      sq[j] += d * d;
    }
    }
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    ls[tid * 8 + j] = s[j];
    lq[tid * 8 + j] = sq[j];
  }
  __syncthreads();
  for (int ch = tid; ch < cin; ch += 256) {
    const int qq = ch / 8, jj = ch % 8;
    double ts = 0, tq = 0;
    for (int l = 0; l < pstep; ++l) {
      ts += ls[(qq + l * q8) * 8 + jj];
      tq += lq[(qq + l * q8) * 8 + jj];
    }
    cs[ch] = ts;
    cq[ch] = tq;
  }
  __syncthreads();
  const int cgp = cin / g.groups;
  const double n = (double)hw * cgp;
  for (int gr = tid; gr < g.groups; gr += 256) {
    double ts = 0, tq = 0;
    for (int ch = gr * cgp; ch < (gr + 1) * cgp; ++ch) {
      ts += cs[ch];
      tq += cq[ch];
    }
    const double mean = ts / n;
    double var = tq / n - mean * mean;
    if (var < 0) var = 0;
    gmean[gr] = mean;
    grstd[gr] = 1.0 / sqrt(var + (double)g.eps);
  }
  __syncthreads();
  for (int ch = tid; ch < cin; ch += 256) {
    const int gr = ch / cgp;
    const double sc = (double)g.gamma[ch] * grstd[gr];
    scl[ch] = (float)sc;
    shf[ch] = (float)((double)g.beta[ch] - gmean[gr] * sc);
  }
  __syncthreads();
  float sc8[8], sh8[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    sc8[j] = scl[c + j];
    sh8[j] = shf[c + j];
  }
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    if (k >= ns) continue;
    const int p = tid / q8 + k * pstep;
    float o[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      o[j] = v[k][j];
      if (act) {
        o[j] = o[j] * sc8[j] + sh8[j];
        if (act == 2) o[j] = silu_f(o[j]);
      }
    }
    const size_t off = (((size_t)b << lhw) + p) * cin + c;
    if constexpr (F32) {
      float4* d = reinterpret_cast<float4*>(out32 + off);
      d[0] = make_float4(o[0], o[1], o[2], o[3]);
      d[1] = make_float4(o[4], o[5], o[6], o[7]);
    } else {
      uint4 u = {pack_bf16(o[0], o[1]), pack_bf16(o[2], o[3]), pack_bf16(o[4], o[5]), pack_bf16(o[6], o[7])};
      *reinterpret_cast<uint4*>(out + off) = u;
    }
  }
}

template <int NS>
void launch_gaw(hipStream_t st, const GnArgs& g, int act, uint16_t* out, float* out32) {
  if (out32)
    hipLaunchKernelGGL((gn_apply_window_kernel<NS, true>), dim3(g.nb), dim3(256), 0, st, g, act, out, out32);
  else
    hipLaunchKernelGGL((gn_apply_window_kernel<NS, false>), dim3(g.nb), dim3(256), 0, st, g, act, out, out32);
  TD_LAUNCHED();
}

}  // namespace

void launch_apply(hipStream_t st, const ApplyArgs& a) {
  const int cin = a.c0 + a.c1;
  TD_CHECK(cin % 8 == 0 && a.c0 % 8 == 0, -5, "apply: channels must be multiples of 8");
  const size_t n = ((size_t)a.nb << (a.lh + a.lw)) * (cin / 8);
  if (!n) return;
  prof_begin(st);
  TD_CHECK((a.out != nullptr) != (a.out32 != nullptr), -5, "apply: exactly one of the BF16 and FP32 outputs");
  TD_CHECK(!a.raw || a.out, -5, "apply: the raw BF16 copy goes with the BF16 output");
  if (a.out32)
    hipLaunchKernelGGL(apply_kernel<true>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(apply_kernel<false>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a);
  TD_LAUNCHED();
  const double el = 8.0 * n;
  prof_end(st, a.out32 ? K_APPLY32 : K_APPLY, 4.0 * el,
           el * ((a.out32 ? 4.0 : 2.0) + (a.raw ? 2.0 : 0.0) + (a.up0 ? 4.0 * a.c1 / cin + 1.0 * a.c0 / cin : 4.0)));
}

void launch_apply_bf16(hipStream_t st, const uint16_t* src, int C, const float* scale, const float* shift, int act,
                       int nb, int lh, int lw, uint16_t* out) {
  TD_CHECK(C % 8 == 0 && act >= 1 && act <= 2, -5, "apply_bf16: channels must be multiples of 8");
  TD_CHECK(lh + lw >= 2, -5, "apply_bf16: windows of at least 4 pixels");
  const size_t n = ((size_t)nb << (lh + lw)) * (C / 8);
  if (!n) return;
  prof_begin(st);
  hipLaunchKernelGGL(apply_bf16_kernel, dim3((unsigned)((n / 4 + 255) / 256)), dim3(256), 0, st,
                     reinterpret_cast<const uint4*>(src), C, scale, shift, act, lh + lw, n / 4,
                     reinterpret_cast<uint4*>(out));
  TD_LAUNCHED();
  prof_end(st, K_APPLY, 32.0 * n, 32.0 * n);
}

void launch_gn_finalize_ch(hipStream_t st, const GnArgs& a, const double* ch0, int slots0, const double* ch1,
                           int slots1) {
  const int cin = a.c0 + a.c1;
  TD_CHECK(cin >= 1 && cin <= kMaxCin && a.groups >= 1 && a.groups <= kMaxCin && cin % a.groups == 0, -5,
           "groupnorm finalize: bad channels or groups");
  TD_CHECK(ch0 && slots0 >= 1 && (a.c1 == 0 || (ch1 && slots1 >= 1)), -5, "groupnorm finalize: missing sums");
  TD_CHECK(!a.up0 || a.lh + a.lw >= 2, -5, "groupnorm finalize: upsampled source needs h, w >= 2");
  if (!a.nb) return;
  hipLaunchKernelGGL(gn_finalize_ch_kernel, dim3(a.nb), dim3(256), 0, st, a, ch0, slots0, ch1, slots1);
  TD_LAUNCHED();
}

void launch_gn_finalize(hipStream_t st, const GnArgs& a, int nchunk) {
  TD_CHECK(nchunk >= 1 && nchunk <= 32 && (a.c0 + a.c1) % a.groups == 0, -5, "groupnorm finalize: bad partials");
  if (!a.nb) return;
  hipLaunchKernelGGL(gn_finalize_kernel, dim3(a.nb), dim3(256), 0, st, a, nchunk);
  TD_LAUNCHED();
}

bool gn_apply_window_fits(int lh, int lw, int c0, int c1, int up0, int groups) {
  const int cin = c0 + c1;
  const long elems = (1L << (lh + lw)) * cin;
  if (cin % 8 || c0 % 8 || c1 % 8 || cin > kWinMaxCin || cin % groups) return false;
  if (up0 && (lh < 1 || lw < 1)) return false;
  const int q8 = cin / 8;
  if (256 % q8 || (1L << (lh + lw)) % (256 / q8)) return false;   // whole pixels per thread
  return elems <= kWinMaxElems && elems >= 2048;
}

void launch_gn_apply_window(hipStream_t st, const GnArgs& g, int act, uint16_t* out, float* out32) {
  TD_CHECK(gn_apply_window_fits(g.lh, g.lw, g.c0, g.c1, g.up0, g.groups), -5, "gn_apply_window: window does not fit");
  TD_CHECK((out != nullptr) != (out32 != nullptr), -5, "gn_apply_window: exactly one of the BF16 and FP32 outputs");
  if (!g.nb) return;
  const int cin = g.c0 + g.c1;
  const int ns = (int)((1L << (g.lh + g.lw)) / (256 / (cin / 8)));
  prof_begin(st);
  if (ns <= 4) launch_gaw<4>(st, g, act, out, out32);
  else if (ns <= 8) launch_gaw<8>(st, g, act, out, out32);
  else launch_gaw<16>(st, g, act, out, out32);
  const double el = (double)g.nb * (1L << (g.lh + g.lw)) * cin;
  prof_end(st, out32 ? K_APPLY32 : K_APPLY, 4.0 * el,
           el * ((out32 ? 4.0 : 2.0) + (g.up0 ? 4.0 * g.c1 / cin + 1.0 * g.c0 / cin : 4.0)));
}

size_t gn_partial_doubles(int nb, int lh, int lw, int cin, int groups) {
  return (size_t)nb * 32 * groups * 2;   // up to 32 partials per window (convolution epilogues)
}

void launch_gn(hipStream_t st, const GnArgs& a) {
  const int cin = a.c0 + a.c1;
  TD_CHECK(cin <= kMaxCin && cin % a.groups == 0, -5, "groupnorm: bad channel/group count");
  for (int cs : {a.c0, a.c1}) {
    if (!cs) continue;
    TD_CHECK(cs % 4 == 0 && 256 % (cs / 4) == 0, -5, "groupnorm: segment channels must divide 1024 in quads");
  }
  if (!a.nb) return;
  const int nchunk = gn_nchunk(a.lh, a.lw, cin, a.up0);
  const double hw = (double)(1 << (a.lh + a.lw));
  prof_begin(st);
  hipLaunchKernelGGL(gn_partial_kernel, dim3(nchunk, a.nb), dim3(256), 0, st, a, nchunk);
  TD_LAUNCHED();
  hipLaunchKernelGGL(gn_finalize_kernel, dim3(a.nb), dim3(256), 0, st, a, nchunk);
  TD_LAUNCHED();
  const double elems = a.nb * hw * ((a.up0 ? a.c0 / 4.0 : a.c0) + a.c1);
  prof_end(st, K_GN, 3.0 * elems, 4.0 * elems + 8.0 * a.nb * cin);
}

}  // namespace td
