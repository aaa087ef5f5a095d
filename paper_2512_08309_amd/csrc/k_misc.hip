// The thin layers of the window denoiser, which do not map onto matrix
// cores: the 3x3 input conv (4 or 1 input channels, K = 36 or 9) with the
// window gather and EDM input scaling fused in; the 3x3 output conv (4 or 1
// output channels) fused with GroupNorm + SiLU on its input, the EDM output
// preconditioning, the Euler step and the window weighting; 2x2 average
// pooling; the noise-level embedding MLP; and 64-token window attention.
// Together they are well under 1% of the denoiser's FLOPs.
#include "td_internal.h"

namespace td {
namespace {

__device__ __forceinline__ float silu_f(float v) { return __fdividef(v, 1.0f + __expf(-v)); }

// ---------------------------------------------------------------- conv_in
// One workgroup per (window, 16x16 output tile).  LDS holds the (16+2)^2 x
// (CI + CC) inputs: c_in-scaled latent channels, then the conditioning
// channels, zero outside the window (the network pads with zeros).  A
// thread owns one pair of output channels (its 2 x 9 x (CI + CC) weights
// live in VGPRs) and walks the tile's pixels; the c0 / 2 lanes that share a
// pixel read the same halo values (LDS broadcast).  Needs 256 % (c0 / 2) == 0.
template <int CI, int CC>
__global__ __launch_bounds__(256) void conv_in_kernel(const float* __restrict__ canvas, int canvas_w,
                                                      const int* __restrict__ origins,
                                                      const float* __restrict__ cond, int H, int c0,
                                                      float c_in, const float* __restrict__ wt,
                                                      const float* __restrict__ bias, float* __restrict__ out) {
  constexpr int CT = CI + CC;
  constexpr int NH = 18 * 18 * CT;
  __shared__ float halo[NH];
  const int b = blockIdx.y;
  const int tiles_x = H / 16;
  const int tx0 = (blockIdx.x % tiles_x) * 16, ty0 = (blockIdx.x / tiles_x) * 16;
  const int ox = origins[2 * b], oy = origins[2 * b + 1];
#pragma unroll
  for (int j = 0; j < (NH + 255) / 256; ++j) {
    const int e = threadIdx.x + 256 * j;
    if (e < NH) {
      const int c = e % CT, p = e / CT;
      const int y = ty0 + p / 18 - 1, x = tx0 + p % 18 - 1;
      float v = 0.f;
      if (y >= 0 && y < H && x >= 0 && x < H) {
        if (c < CI) v = c_in * canvas[((size_t)(oy + y) * canvas_w + ox + x) * CI + c];
        else v = cond[(((size_t)b * H + y) * H + x) * CC + (c - CI)];
      }
      halo[e] = v;
    }
  }
  const int npair = c0 >> 1;
  const int co = 2 * (threadIdx.x % npair);
  float w0[9 * CT], w1[9 * CT];
#pragma unroll
  for (int k = 0; k < 9 * CT; ++k) {
    w0[k] = wt[(size_t)k * c0 + co];
    w1[k] = wt[(size_t)k * c0 + co + 1];
  }
  const float b0 = bias[co], b1 = bias[co + 1];
  __syncthreads();
  for (int p = threadIdx.x / npair; p < 256; p += 256 / npair) {
    const int py = p / 16, px = p % 16;
    float a0 = b0, a1 = b1;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const float* hp = halo + ((py + t / 3) * 18 + px + t % 3) * CT;
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const float v = hp[c];
        a0 += v * w0[t * CT + c];
        a1 += v * w1[t * CT + c];
      }
    }
    *reinterpret_cast<float2*>(out + (((size_t)b * H + ty0 + py) * H + tx0 + px) * c0 + co) = make_float2(a0, a1);
  }
}

// ---------------------------------------------------------------- conv_out
// One workgroup per (window, 16x16 output tile), one output pixel per
// thread.  The input channels go through LDS in chunks of CK: each chunk's
// (16+2)^2 x CK halo is read as 16-byte segments (a thread keeps the same
// 4-channel segment for every pixel it loads, so its GroupNorm scale and
// shift are one float4 each), normalised and SiLU-activated, zero outside
// the window.  The next chunk's segments are loaded into registers while the
// current chunk is being multiplied, so a chunk costs one memory latency,
// not one per element.  Halo rows are CK + 4 floats (16-byte aligned; eight
// consecutive lanes of a 16-byte read cover all 32 banks once); the weights
// are the same for every lane and are read with uniform addresses straight
// from global memory, so the products touch LDS once per 4 channels.
template <int CO, int CK>
__global__ __launch_bounds__(256) void conv_out_kernel(OutArgs a) {
  constexpr int C4 = CK / 4;                    // 16-byte segments per halo pixel
  constexpr int NSEG = 18 * 18 * C4;            // segments per chunk
  constexpr int PT = (NSEG + 255) / 256;        // per thread
  static_assert(256 % C4 == 0, "a thread's segment index must be the same for every pixel it loads");
  constexpr int LD = CK + 4;
  __shared__ __attribute__((aligned(16))) float halo[18 * 18 * LD];
  const int b = blockIdx.y;
  const int H = a.H, c0 = a.c0;
  const int tiles_x = H / 16;
  const int tx0 = (blockIdx.x % tiles_x) * 16, ty0 = (blockIdx.x / tiles_x) * 16;
  const int py = threadIdx.x / 16, px = threadIdx.x % 16;
  float acc[CO];
#pragma unroll
  for (int o = 0; o < CO; ++o) acc[o] = 0.f;
  const float* hb = a.h + (size_t)b * H * H * c0;
  const float* sc = a.gn_scale + (size_t)b * c0;
  const float* sh = a.gn_shift + (size_t)b * c0;
  const int q4 = 4 * (threadIdx.x % C4);        // first channel of this thread's segment
  int hoff[PT];                                 // LDS offset of the segment (-1: none)
  int goff[PT];                                 // float offset in the window (-1: outside)
#pragma unroll
  for (int j = 0; j < PT; ++j) {
    const int e = threadIdx.x + 256 * j;
    const int p = e / C4, hy = p / 18, hx = p % 18;
    const int y = ty0 + hy - 1, x = tx0 + hx - 1;
    hoff[j] = e < NSEG ? p * LD + q4 : -1;
    goff[j] = (e < NSEG && y >= 0 && y < H && x >= 0 && x < H) ? (y * H + x) * c0 + q4 : -1;
  }
  const float4 z4 = {0.f, 0.f, 0.f, 0.f};
  float4 r[PT];
  // unconditional 16-byte loads (pixels outside the window read the
  // window's first segment and are zeroed when stored to LDS)
  auto load = [&](int ci0) {
#pragma unroll
    for (int j = 0; j < PT; ++j) r[j] = *reinterpret_cast<const float4*>(hb + (goff[j] < 0 ? 0 : goff[j]) + ci0);
  };
  load(0);
  for (int ci0 = 0; ci0 < c0; ci0 += CK) {
    __syncthreads();                            // every thread is done with the last chunk
    const float4 s4 = *reinterpret_cast<const float4*>(sc + ci0 + q4);
    const float4 h4 = *reinterpret_cast<const float4*>(sh + ci0 + q4);
#pragma unroll
    for (int j = 0; j < PT; ++j) {
      if (hoff[j] < 0) continue;
      float4 v = z4;
      if (goff[j] >= 0) {
        v.x = silu_f(r[j].x * s4.x + h4.x);
        v.y = silu_f(r[j].y * s4.y + h4.y);
        v.z = silu_f(r[j].z * s4.z + h4.z);
        v.w = silu_f(r[j].w * s4.w + h4.w);
      }
      *reinterpret_cast<float4*>(halo + hoff[j]) = v;
    }
    __syncthreads();
    if (ci0 + CK < c0) load(ci0 + CK);          // in flight during the products below
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const float* hp = halo + ((py + t / 3) * 18 + px + t % 3) * LD;
      const float* wp = a.wt + ((size_t)t * c0 + ci0) * CO;   // [c][o] of this tap and chunk
#pragma unroll 2
      for (int c4 = 0; c4 < CK / 4; ++c4) {
        const float4 v4 = *reinterpret_cast<const float4*>(hp + 4 * c4);
        const float v[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int o = 0; o < CO; ++o) acc[o] += v[q] * wp[(4 * c4 + q) * CO + o];
      }
    }
  }
  const int u = tx0 + px, v = ty0 + py;
  const int ox = a.origins[2 * b], oy = a.origins[2 * b + 1];
  const float* xin = a.canvas + ((size_t)(oy + v) * a.canvas_w + ox + u) * CO;
  const float wuv = a.mode == 0 ? a.w1d[u] * a.w1d[v] : 0.f;   // window weight: contributions only
#pragma unroll
  for (int o = 0; o < CO; ++o) {
    float x = xin[o];
    float F = acc[o] + a.bias[o];
    float d = a.c_skip * x + a.c_out * F;
    if (a.mode == 1) {
      a.dout[(((size_t)b * H + v) * H + u) * CO + o] = d;
    } else {
      float phi = a.direct ? d : x + a.c_euler * (x - d);
      if (a.mode == 2) a.dout[(((size_t)b * H + v) * H + u) * CO + o] = phi;
      else a.slots[b][((size_t)v * H + u) * CO + o] = wuv * phi;
    }
  }
}

// ---------------------------------------------------------------- avgpool
__global__ __launch_bounds__(256) void avgpool_kernel(const float* __restrict__ in, float* __restrict__ out,
                                                      int nb, int h, int w, int C) {
  const int ho = h / 2, wo = w / 2, cq = C / 4;
  size_t n = (size_t)nb * ho * wo * cq;
  size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  int q = (int)(e % cq);
  size_t p = e / cq;
  int x = (int)(p % wo);
  size_t r = p / wo;
  int y = (int)(r % ho);
  size_t b = r / ho;
  const float* s = in + (((b * h + 2 * y) * w + 2 * x) * C) + 4 * q;
  float4 a0 = *reinterpret_cast<const float4*>(s);
  float4 a1 = *reinterpret_cast<const float4*>(s + C);
  float4 a2 = *reinterpret_cast<const float4*>(s + (size_t)w * C);
  float4 a3 = *reinterpret_cast<const float4*>(s + (size_t)w * C + C);
  float4 o;
  o.x = 0.25f * ((a0.x + a1.x) + (a2.x + a3.x));
  o.y = 0.25f * ((a0.y + a1.y) + (a2.y + a3.y));
  o.z = 0.25f * ((a0.z + a1.z) + (a2.z + a3.z));
  o.w = 0.25f * ((a0.w + a1.w) + (a2.w + a3.w));
  *reinterpret_cast<float4*>(out + p * C + 4 * q) = o;
}

// ---------------------------------------------------------------- embedding
__global__ void gemv_kernel(const float* __restrict__ W, const float* __restrict__ b,
                            const float* __restrict__ add, const float* __restrict__ in,
                            float* __restrict__ out, int nk, int nin, int nout, int act) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nk * nout) return;
  int k = e / nout, o = e % nout;
  float acc = 0.f;
  for (int i = 0; i < nin; ++i) acc += W[(size_t)o * nin + i] * in[(size_t)k * nin + i];
  acc += b[o];
  if (add) acc += add[o];
  if (act) acc = acc / (1.0f + expf(-acc));
  out[e] = acc;
}

__global__ void pos_emb_kernel(const float* __restrict__ cn, int nk, int dim, float log_period,
                               float* __restrict__ out) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nk * dim) return;
  int k = e / dim, j = e % dim, half = dim / 2;
  int jj = j < half ? j : j - half;
  float f = expf(-log_period * (float)jj / (float)half);
  float arg = cn[k] * f;
  out[e] = j < half ? cosf(arg) : sinf(arg);
}

// ---------------------------------------------------------------- attention
// One workgroup per (window, head); T <= 64 tokens, head dim d <= 64, both
// zero-padded to 64 in LDS.  FP32 MFMA (v_mfma_f32_16x16x4_f32): wave w owns
// query rows 16w..16w+15.  S = Q K^T for its rows (4 column tiles x 16
// k-steps), scaled; the row softmax (masked to the T valid keys) reduces
// across the 16 lanes that hold a row with xor shuffles; P goes through LDS
// into the A-operand layout and O = P V (4 tiles x 16 k-steps).  A lane of
// an MFMA holds D[4 (lane / 16) + v][lane % 16] of a tile.
typedef float f4v_a __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void attention_kernel(const float* __restrict__ qkv, float* __restrict__ out,
                                                        int T, int C, int heads) {
  constexpr int LD = 65;
  __shared__ float Q[64 * LD], Kt[64 * LD], V[64 * LD], P[64 * LD];
  const int b = blockIdx.x, h = blockIdx.y;
  const int d = C / heads;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int g = lane >> 4, r16 = lane & 15;
  const float* base = qkv + (size_t)b * T * 3 * C;
  for (int e = tid; e < 64 * 64; e += 256) {
    const int t = e >> 6, i = e & 63;
    float q = 0.f, k = 0.f, v = 0.f;
    if (t < T && i < d) {
      const float* row = base + (size_t)t * 3 * C + h * d + i;
      q = row[0];
      k = row[C];
      v = row[2 * C];
    }
    Q[t * LD + i] = q;
    Kt[t * LD + i] = k;
    V[t * LD + i] = v;
  }
  __syncthreads();
  const int r0 = 16 * w;
  f4v_a s[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) s[j] = (f4v_a){0.f, 0.f, 0.f, 0.f};
  for (int kk = 0; kk < 16; ++kk) {
    const int k = 4 * kk + g;
    const float a = Q[(r0 + r16) * LD + k];
#pragma unroll
    for (int j = 0; j < 4; ++j) s[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, Kt[(16 * j + r16) * LD + k], s[j], 0, 0, 0);
  }
  const float scale = 1.0f / sqrtf((float)d);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    float mx = -3.0e38f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      s[j][v] = (16 * j + r16 < T) ? s[j][v] * scale : -3.0e38f;
      mx = fmaxf(mx, s[j][v]);
    }
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    float sum = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float ev = (16 * j + r16 < T) ? expf(s[j][v] - mx) : 0.f;
      s[j][v] = ev;
      sum += ev;
    }
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) sum += __shfl_xor(sum, o);
    const float inv = 1.0f / sum;
#pragma unroll
    for (int j = 0; j < 4; ++j) P[(r0 + 4 * g + v) * LD + 16 * j + r16] = s[j][v] * inv;
  }
  __syncthreads();
  f4v_a o[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) o[t] = (f4v_a){0.f, 0.f, 0.f, 0.f};
  for (int kk = 0; kk < 16; ++kk) {
    const int j = 4 * kk + g;
    const float a = P[(r0 + r16) * LD + j];
#pragma unroll
    for (int t = 0; t < 4; ++t) o[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, V[j * LD + 16 * t + r16], o[t], 0, 0, 0);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = r0 + 4 * g + v, f = 16 * t + r16;
      if (i < T && f < d) out[((size_t)b * T + i) * C + h * d + f] = o[t][v];
    }
}

}  // namespace

void launch_conv_in(hipStream_t st, const float* canvas, int canvas_w, const int* origins, int nwin, int H,
                    int cimg, const float* cond, int ccond, int c0, float c_in, const float* wt, const float* bias,
                    float* out) {
  if (!nwin) return;
  TD_CHECK(H % 16 == 0, -5, "conv_in: window size must be a multiple of 16");
  TD_CHECK(ccond == 0 || cond, -5, "conv_in: conditioning channels without conditioning input");
  const int ct = cimg + ccond;
  dim3 grid((H / 16) * (H / 16), nwin);
  // a pixel's c0 / 2 channel-pair lanes must tile the 256-thread workgroup
  TD_CHECK(c0 % 2 == 0 && c0 <= 512 && 256 % (c0 / 2) == 0, -5,
           "conv_in: the first level's width must be 2^k with 2 <= 2^k <= 512");
  prof_begin(st);
#define TD_CONV_IN(CI, CC)                                                                                   \
  hipLaunchKernelGGL((conv_in_kernel<CI, CC>), grid, dim3(256), 0, st, canvas, canvas_w, origins, cond, H, c0, \
                     c_in, wt, bias, out)
  if (cimg == 4 && ccond == 0) TD_CONV_IN(4, 0);
  else if (cimg == 1 && ccond == 0) TD_CONV_IN(1, 0);
  else if (cimg == 1 && ccond == 1) TD_CONV_IN(1, 1);
  else if (cimg == 4 && ccond == 1) TD_CONV_IN(4, 1);
  else if (cimg == 4 && ccond == 4) TD_CONV_IN(4, 4);
  else TD_CHECK(false, -5, "conv_in: supported (latent, conditioning) channels are (1|4, 0), (1|4, 1), (4, 4)");
#undef TD_CONV_IN
  TD_LAUNCHED();
  const double px = (double)nwin * H * H;
  prof_end(st, K_CONV_IN, 2.0 * px * c0 * 9 * ct, 4.0 * px * (ct + c0));
}

void launch_conv_out(hipStream_t st, const OutArgs& a) {
  if (!a.nb) return;
  TD_CHECK(a.H % 16 == 0, -5, "conv_out: window size must be a multiple of 16");
  TD_CHECK(a.mode == 0 ? (a.w1d && a.slots) : a.dout != nullptr, -5, "conv_out: output buffers missing for the mode");
  dim3 grid((a.H / 16) * (a.H / 16), a.nb);
  prof_begin(st);
  if (a.cimg == 4 && a.c0 % 32 == 0)
    hipLaunchKernelGGL((conv_out_kernel<4, 32>), grid, dim3(256), 0, st, a);
  else if (a.cimg == 4 && a.c0 % 16 == 0)
    hipLaunchKernelGGL((conv_out_kernel<4, 16>), grid, dim3(256), 0, st, a);
  else if (a.cimg == 1 && a.c0 % 16 == 0)
    hipLaunchKernelGGL((conv_out_kernel<1, 16>), grid, dim3(256), 0, st, a);
  else
    TD_CHECK(false, -5, "conv_out: unsupported channel counts");
  TD_LAUNCHED();
  const double px = (double)a.nb * a.H * a.H;
  prof_end(st, K_CONV_OUT, 2.0 * px * a.cimg * 9 * a.c0, 4.0 * px * (a.c0 + 2 * a.cimg));
}

void launch_avgpool(hipStream_t st, const float* in, float* out, int nb, int h, int w, int C) {
  TD_CHECK(C % 4 == 0, -5, "avgpool: channels must be a multiple of 4");
  size_t n = (size_t)nb * (h / 2) * (w / 2) * (C / 4);
  if (!n) return;
  prof_begin(st);
  hipLaunchKernelGGL(avgpool_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out, nb, h, w, C);
  TD_LAUNCHED();
  prof_end(st, K_POOL, 4.0 * n * 4, 4.0 * 4 * n * 5);
}

void launch_gemv(hipStream_t st, const float* W, const float* b, const float* add, const float* in, float* out,
                 int nk, int nin, int nout, int act_silu) {
  int n = nk * nout;
  if (!n) return;
  hipLaunchKernelGGL(gemv_kernel, dim3((n + 255) / 256), dim3(256), 0, st, W, b, add, in, out, nk, nin, nout,
                     act_silu);
  TD_LAUNCHED();
}

void launch_pos_emb(hipStream_t st, const float* c_noise, int nk, int dim, float max_period, float* out) {
  int n = nk * dim;
  if (!n) return;
  hipLaunchKernelGGL(pos_emb_kernel, dim3((n + 255) / 256), dim3(256), 0, st, c_noise, nk, dim,
                     logf(max_period), out);
  TD_LAUNCHED();
}

void launch_attention(hipStream_t st, const float* qkv, float* out, int nb, int T, int C, int heads) {
  TD_CHECK(T <= 64 && C / heads <= 64 && C % heads == 0, -5, "attention: at most 64 tokens and head dim 64");
  if (!nb) return;
  prof_begin(st);
  hipLaunchKernelGGL(attention_kernel, dim3(nb, heads), dim3(256), 0, st, qkv, out, T, C, heads);
  TD_LAUNCHED();
  prof_end(st, K_ATTN, 4.0 * nb * T * T * C, 4.0 * nb * T * 4 * C);
}

}  // namespace td
