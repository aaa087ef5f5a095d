// Kernels of student training (hand-written backward of the window UNet,
// distillation loss and AdamW).  The forward reuses the sampler's kernels;
// data gradients of the convolutions reuse the implicit-GEMM forward kernel
// with flipped, transposed weights.  What is here:
//  * weight relayouts ([co][ci][k][k] master -> forward / flipped layouts);
//  * materialising a conv input (virtual concat + nearest 2x upsample) and
//    its GroupNorm affine + activation;
//  * GroupNorm (+ SiLU) backward, one workgroup per (window, group);
//  * weight gradients of 3x3 / 1x1 convolutions, split over pixels with a
//    fixed-order reduction of the splits;
//  * column sums (bias gradients), window-attention backward, the
//    noise-embedding MLP backward, and small elementwise kernels;
//  * AdamW (decoupled weight decay) on the flat FP32 master parameters.
// Every reduction runs in a fixed order: gradients are deterministic.
#include "td_internal.h"

namespace td {
namespace {

__device__ __forceinline__ float sigm(float v) { return 1.0f / (1.0f + __expf(-v)); }

// w: [co][ci][kk] -> fwd [kk][ci][co]; flip (nullable) [kk][co_pad][ci] with
// tap kk-1-t (3x3 rotated by 180 degrees), rows co..co_pad-1 zero.
__global__ void relayout_kernel(const float* __restrict__ w, int co, int ci, int kk, int co_pad,
                                float* __restrict__ fwd, float* __restrict__ flip) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= co_pad * ci * kk) return;
  const int t = e % kk, i = (e / kk) % ci, o = e / (kk * ci);
  const float v = o < co ? w[e] : 0.f;
  if (o < co && fwd) fwd[((size_t)t * ci + i) * co + o] = v;
  if (flip) flip[((size_t)(kk - 1 - t) * co_pad + o) * ci + i] = v;
}

// BF16 weights for the reduced-precision convolution, [rows][kp] with
// K = tap * cols + col, zero-padded to kp.  flip = 0: the forward conv
// (rows = co, cols = ci, value w[o][i][t]); flip = 1: the data-gradient conv
// (rows = ci, cols = co, value w[o][i][kk-1-t]).
__global__ void lp_weights_kernel(const float* __restrict__ w, int co, int ci, int kk, int kp, int flip,
                                  __bf16* __restrict__ out) {
  const int rows = flip ? ci : co, cols = flip ? co : ci;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * kp) return;
  const int r = e / kp, k = e % kp;
  float v = 0.f;
  if (k < kk * cols) {
    const int t = k / cols, c = k % cols;
    v = flip ? w[((size_t)c * ci + r) * kk + (kk - 1 - t)] : w[((size_t)r * ci + c) * kk + t];
  }
  out[e] = (__bf16)v;
}

// out[b][y][x][c] = concat(up0 ? s0[b][y/2][x/2] : s0[b][y][x], s1[b][y][x])
__global__ void dense_in_kernel(const float* __restrict__ s0, int c0, int up0, const float* __restrict__ s1,
                                int c1, int lh, int lw, size_t n, float* __restrict__ out) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int cin = c0 + c1;
  const int c = (int)(e % cin);
  const size_t p = e / cin;
  const int lhw = lh + lw;
  const size_t b = p >> lhw;
  const int y = (int)((p >> lw) & ((1 << lh) - 1)), x = (int)(p & ((1 << lw) - 1));
  float v;
  if (c < c0) {
    if (up0) v = s0[(((b << (lhw - 2)) + ((size_t)(y >> 1) << (lw - 1)) + (x >> 1)) * c0) + c];
    else v = s0[p * c0 + c];
  } else {
    v = s1[p * c1 + (c - c0)];
  }
  out[e] = v;
}

// out = act(x * scale[b][c] + shift[b][c]); act 1 affine, 2 affine + SiLU
__global__ void act_kernel(const float* __restrict__ x, const float* __restrict__ scale,
                           const float* __restrict__ shift, int hw, int C, int act, size_t n,
                           float* __restrict__ out) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int c = (int)(e % C);
  const size_t b = e / ((size_t)hw * C);
  float v = x[e] * scale[b * C + c] + shift[b * C + c];
  if (act == 2) v = v * sigm(v);
  out[e] = v;
}

// GroupNorm (+ SiLU) backward for one (window b, group g).  With
// xh = (x - mean) rstd, y = xh gamma + beta, dy = dA (act' at y),
// gd = dy gamma: dx = rstd (gd - mean(gd) - xh mean(gd xh)).  Also per-
// channel partial sums of dy xh (dgamma) and dy (dbeta) for this window.
// Thread t < np cgp (np = 256 / cgp) handles channel t % cgp of the group
// and pixels t / cgp + k np; the remaining threads only join the reductions.
__global__ __launch_bounds__(256) void gn_bwd_kernel(const float* __restrict__ x, const float* __restrict__ mean,
                                                     const float* __restrict__ rstd, const float* __restrict__ gamma,
                                                     const float* __restrict__ beta, const float* __restrict__ dA,
                                                     int hw, int C, int groups, int act, int accumulate,
                                                     float* __restrict__ dx, float* __restrict__ dgam_part,
                                                     float* __restrict__ dbet_part) {
  __shared__ float r1[256], r2[256], r3[256], r4[256];
  const int b = blockIdx.x, g = blockIdx.y, tid = threadIdx.x;
  const int cgp = C / groups;
  const int np = 256 / cgp;
  const bool active = tid < np * cgp;
  const int cl = tid % cgp, pl = active ? tid / cgp : hw;
  const int c = g * cgp + cl;
  const float mu = mean[b * groups + g], rs = rstd[b * groups + g];
  const float ga = gamma[c], be = beta[c];
  const size_t base = (size_t)b * hw * C + c;
  float sg = 0.f, sgx = 0.f, sdy = 0.f, sdyx = 0.f;
  for (int p = pl; p < hw; p += np) {
    const size_t o = base + (size_t)p * C;
    const float xh = (x[o] - mu) * rs;
    float dy = dA[o];
    if (act == 2) {
      const float y = xh * ga + be;
      const float s = sigm(y);
      dy = dy * (s + y * s * (1.0f - s));
    }
    sdy += dy;
    sdyx += dy * xh;
    sg += dy * ga;
    sgx += dy * ga * xh;
  }
  r1[tid] = sg;
  r2[tid] = sgx;
  r3[tid] = sdy;
  r4[tid] = sdyx;
  __syncthreads();
  if (tid < cgp) {   // per-channel sums over the threads of this channel, in order
    float a = 0.f, bb = 0.f;
    for (int l = 0; l < np; ++l) {
      a += r3[l * cgp + tid];
      bb += r4[l * cgp + tid];
    }
    dbet_part[(size_t)b * C + g * cgp + tid] = a;
    dgam_part[(size_t)b * C + g * cgp + tid] = bb;
  }
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      r1[tid] += r1[tid + w];
      r2[tid] += r2[tid + w];
    }
    __syncthreads();
  }
  const float inv_n = 1.0f / (float)(hw * cgp);
  const float mg = r1[0] * inv_n, mgx = r2[0] * inv_n;
  for (int p = pl; p < hw; p += np) {
    const size_t o = base + (size_t)p * C;
    const float xh = (x[o] - mu) * rs;
    float dy = dA[o];
    if (act == 2) {
      const float y = xh * ga + be;
      const float s = sigm(y);
      dy = dy * (s + y * s * (1.0f - s));
    }
    const float v = rs * (dy * ga - mg - xh * mgx);
    dx[o] = accumulate ? dx[o] + v : v;
  }
}

// out[c] (+)= sum_r in[r][c], rows in order.
__global__ void sum_rows_kernel(const float* __restrict__ in, int rows, int C, int accumulate,
                                float* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  float s = 0.f;
  for (int r = 0; r < rows; ++r) s += in[(size_t)r * C + c];
  out[c] = accumulate ? out[c] + s : s;
}

// part[chunk][c] = sum of rows chunk*per .. of in[M][C].  A workgroup takes
// 64 columns; its 4 waves take rows r0 + w, r0 + w + 4, ... (a wave reads 64
// consecutive floats of a row), then the 4 partial sums are added in order.
__global__ __launch_bounds__(256) void colsum_part_kernel(const float* __restrict__ in, size_t M, int C, int per,
                                                          float* __restrict__ part) {
  __shared__ float red[4][64];
  const int chunk = blockIdx.y;
  const int cl = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + cl;
  const size_t r0 = (size_t)chunk * per;
  const size_t r1 = r0 + per < M ? r0 + per : M;
  float s = 0.f;
  if (c < C)
    for (size_t r = r0 + w; r < r1; r += 4) s += in[r * C + c];
  red[w][cl] = s;
  __syncthreads();
  if (w == 0 && c < C) part[(size_t)chunk * C + c] = ((red[0][cl] + red[1][cl]) + red[2][cl]) + red[3][cl];
}

// Weight gradient of a 3x3 (taps 9, zero padding) or 1x1 conv over the
// pixel range of split s: part[s][t][i][o] = sum_m A(t)[m][i] dY[m][o], a
// GEMM with the pixels as K.  Tile 64 (ci) x 64 (co) per workgroup; pixels
// staged WG_PIX at a time through LDS as [pixel][channel], which is the
// operand layout of v_mfma_f32_16x16x4_f32 (A = A(t)^T, B = dY, 4 pixels
// per step).  Wave w owns ci rows 16w..16w+15 and all 64 co columns.  The
// row stride of 80 floats puts the two rows a half-wave reads in disjoint
// LDS banks.
constexpr int WG_PIX = 32;
constexpr int WG_LD = 80;
typedef float wg_f4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void wgrad_kernel(const float* __restrict__ A, const float* __restrict__ dY,
                                                    int lh, int lw, int ci, int co, int taps, size_t M,
                                                    int per, float* __restrict__ part) {
  __shared__ float As[WG_PIX * WG_LD];
  __shared__ float Ds[WG_PIX * WG_LD];
  const int t = blockIdx.z % taps, s = blockIdx.z / taps;
  const int i0 = blockIdx.x * 64, o0 = blockIdx.y * 64;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int g = lane >> 4, r16 = lane & 15;
  const int W = 1 << lw, Hh = 1 << lh;
  int dy = 0, dx = 0;
  if (taps == 9) {
    dy = t / 3 - 1;
    dx = t % 3 - 1;
  }
  wg_f4 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = (wg_f4){0.f, 0.f, 0.f, 0.f};
  const size_t m0 = (size_t)s * per;
  const size_t m1 = m0 + per < M ? m0 + per : M;
  for (size_t mb = m0; mb < m1; mb += WG_PIX) {
    for (int e = tid; e < WG_PIX * 64; e += 256) {
      const int p = e / 64, k = e % 64;
      const size_t m = mb + p;
      float av = 0.f, dv = 0.f;
      if (m < m1) {
        if (i0 + k < ci) {
          const int y = (int)((m >> lw) & (Hh - 1)) + dy, x = (int)(m & (W - 1)) + dx;
          if (y >= 0 && y < Hh && x >= 0 && x < W) av = A[(m + (ptrdiff_t)dy * W + dx) * ci + i0 + k];
        }
        if (o0 + k < co) dv = dY[m * co + o0 + k];
      }
      As[p * WG_LD + k] = av;
      Ds[p * WG_LD + k] = dv;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < WG_PIX / 4; ++kk) {
      const int p = 4 * kk + g;
      const float a = As[p * WG_LD + 16 * w + r16];
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, Ds[p * WG_LD + 16 * j + r16], acc[j], 0, 0, 0);
    }
    __syncthreads();
  }
  // lane holds D[4g + v][r16] of tile (w, j): ci row i0 + 16w + 4g + v, co column o0 + 16j + r16
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + 16 * w + 4 * g + v, o = o0 + 16 * j + r16;
      if (i < ci && o < co) part[(((size_t)s * taps + t) * ci + i) * co + o] = acc[j][v];
    }
}

// grad[o][i][t] += sum_s part[s][t][i][o]
__global__ void wgrad_reduce_kernel(const float* __restrict__ part, int nsplit, int taps, int ci, int co,
                                    float* __restrict__ grad) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= co * ci * taps) return;
  const int t = e % taps, i = (e / taps) % ci, o = e / (taps * ci);
  float s = 0.f;
  for (int k = 0; k < nsplit; ++k) s += part[(((size_t)k * taps + t) * ci + i) * co + o];
  grad[e] += s;
}

// Window attention backward, one workgroup per (window, head): S = Q K^T / sqrt(d),
// P = softmax(S), O = P V.  Given dO: dV = P^T dO, dP = dO V^T,
// dS = P (dP - rowsum(dP P)), dQ = dS K / sqrt(d), dK = dS^T Q / sqrt(d).
__global__ __launch_bounds__(256) void attention_bwd_kernel(const float* __restrict__ qkv,
                                                            const float* __restrict__ dO, int T, int C,
                                                            int heads, float* __restrict__ dqkv) {
  __shared__ float Q[64 * 65], Kk[64 * 65], V[64 * 65], G[64 * 65], P[64 * 65], dS[64 * 65];
  const int b = blockIdx.x, h = blockIdx.y, tid = threadIdx.x;
  const int d = C / heads;
  const float scale = 1.0f / __builtin_sqrtf((float)d);
  const float* base = qkv + (size_t)b * T * 3 * C;
  for (int e = tid; e < T * d; e += 256) {
    const int i = e / d, k = e % d;
    Q[i * 65 + k] = base[(size_t)i * 3 * C + h * d + k];
    Kk[i * 65 + k] = base[(size_t)i * 3 * C + C + h * d + k];
    V[i * 65 + k] = base[(size_t)i * 3 * C + 2 * C + h * d + k];
    G[i * 65 + k] = dO[((size_t)b * T + i) * C + h * d + k];
  }
  __syncthreads();
  for (int e = tid; e < T * T; e += 256) {
    const int i = e / T, j = e % T;
    float s = 0.f, g = 0.f;
    for (int k = 0; k < d; ++k) {
      s += Q[i * 65 + k] * Kk[j * 65 + k];
      g += G[i * 65 + k] * V[j * 65 + k];
    }
    P[i * 65 + j] = s * scale;
    dS[i * 65 + j] = g;   // dP for now
  }
  __syncthreads();
  if (tid < T) {   // row softmax, then dS = P (dP - sum_j dP P)
    float mx = -3.0e38f;
    for (int j = 0; j < T; ++j) mx = fmaxf(mx, P[tid * 65 + j]);
    float sum = 0.f;
    for (int j = 0; j < T; ++j) {
      const float v = expf(P[tid * 65 + j] - mx);
      P[tid * 65 + j] = v;
      sum += v;
    }
    const float inv = 1.0f / sum;
    float r = 0.f;
    for (int j = 0; j < T; ++j) {
      P[tid * 65 + j] *= inv;
      r += dS[tid * 65 + j] * P[tid * 65 + j];
    }
    for (int j = 0; j < T; ++j) dS[tid * 65 + j] = P[tid * 65 + j] * (dS[tid * 65 + j] - r);
  }
  __syncthreads();
  float* out = dqkv + (size_t)b * T * 3 * C;
  for (int e = tid; e < T * d; e += 256) {
    const int i = e / d, k = e % d;
    float dv = 0.f, dq = 0.f, dk = 0.f;
    for (int j = 0; j < T; ++j) {
      dv += P[j * 65 + i] * G[j * 65 + k];
      dq += dS[i * 65 + j] * Kk[j * 65 + k];
      dk += dS[j * 65 + i] * Q[j * 65 + k];
    }
    out[(size_t)i * 3 * C + h * d + k] = dq * scale;
    out[(size_t)i * 3 * C + C + h * d + k] = dk * scale;
    out[(size_t)i * 3 * C + 2 * C + h * d + k] = dv;
  }
}

// Embedding MLP backward for one noise level: z1 = W1 pe + b1, e1 = SiLU(z1),
// z2 = W2 e1 + b2, e2 = SiLU(z2); given de2 accumulate dW1, db1, dW2, db2.
__global__ __launch_bounds__(256) void emb_bwd_kernel(float c_noise, int c0, int emb, float log_period,
                                                      const float* __restrict__ W1, const float* __restrict__ b1,
                                                      const float* __restrict__ W2, const float* __restrict__ b2,
                                                      const float* __restrict__ de2, float* __restrict__ dW1,
                                                      float* __restrict__ db1, float* __restrict__ dW2,
                                                      float* __restrict__ db2) {
  __shared__ float pe[1024], z1[1024], e1[1024], dz2[1024], dz1[1024];
  const int tid = threadIdx.x, half = c0 / 2;
  for (int j = tid; j < c0; j += 256) {
    const int jj = j < half ? j : j - half;
    const float f = expf(-log_period * (float)jj / (float)half);
    const float arg = c_noise * f;
    pe[j] = j < half ? cosf(arg) : sinf(arg);
  }
  __syncthreads();
  for (int o = tid; o < emb; o += 256) {
    float s = b1[o];
    for (int i = 0; i < c0; ++i) s += W1[(size_t)o * c0 + i] * pe[i];
    z1[o] = s;
    e1[o] = s * sigm(s);
  }
  __syncthreads();
  for (int o = tid; o < emb; o += 256) {
    float s = b2[o];
    for (int i = 0; i < emb; ++i) s += W2[(size_t)o * emb + i] * e1[i];
    const float sg = sigm(s);
    dz2[o] = de2[o] * (sg + s * sg * (1.0f - sg));
  }
  __syncthreads();
  for (int e = tid; e < emb * emb; e += 256) dW2[e] += dz2[e / emb] * e1[e % emb];
  for (int o = tid; o < emb; o += 256) db2[o] += dz2[o];
  for (int i = tid; i < emb; i += 256) {
    float s = 0.f;
    for (int o = 0; o < emb; ++o) s += W2[(size_t)o * emb + i] * dz2[o];
    const float sg = sigm(z1[i]);
    dz1[i] = s * (sg + z1[i] * sg * (1.0f - sg));
  }
  __syncthreads();
  for (int e = tid; e < emb * c0; e += 256) dW1[e] += dz1[e / c0] * pe[e % c0];
  for (int o = tid; o < emb; o += 256) db1[o] += dz1[o];
}

// Per ResBlock noise-level bias: bias = conv1.b + Wemb e2 + bemb.  Given its
// gradient db (= column sums of dh1): dWemb += db e2^T, dbemb += db,
// dconv1.b += db, de2 += Wemb^T db.
__global__ void emb_bias_bwd_kernel(const float* __restrict__ db, const float* __restrict__ e2,
                                    const float* __restrict__ Wemb, int cout, int emb, float* __restrict__ dWemb,
                                    float* __restrict__ dbemb, float* __restrict__ dcb, float* __restrict__ de2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < cout * emb) dWemb[e] += db[e / emb] * e2[e % emb];
  if (e < cout) {
    dbemb[e] += db[e];
    dcb[e] += db[e];
  }
  if (e < emb) {
    float s = 0.f;
    for (int o = 0; o < cout; ++o) s += Wemb[(size_t)o * emb + e] * db[o];
    de2[e] += s;
  }
}

// d = w * 2 (D - y) / n; part[block] = sum of (D - y)^2 over the block.
__global__ __launch_bounds__(256) void mse_kernel(const float* __restrict__ D, const float* __restrict__ y,
                                                  size_t n, float gscale, float* __restrict__ d,
                                                  float* __restrict__ part) {
  __shared__ float r[256];
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  float q = 0.f;
  if (e < n) {
    const float diff = D[e] - y[e];
    d[e] = gscale * diff;
    q = diff * diff;
  }
  r[threadIdx.x] = q;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) r[threadIdx.x] += r[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = r[0];
}

// out[i*cpad + c] = c < C ? s * in[i*C + c] : 0   (channel padding + scale)
__global__ void pad_scale_kernel(const float* __restrict__ in, size_t npix, int C, int cpad, float s,
                                 float* __restrict__ out) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= npix * cpad) return;
  const int c = (int)(e % cpad);
  const size_t p = e / cpad;
  out[e] = c < C ? s * in[p * C + c] : 0.f;
}

// a += b
__global__ void add_kernel(float* __restrict__ a, const float* __restrict__ b, size_t n) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) a[e] += b[e];
}

// dx (+)= avgpool backward: dx[b][y][x] = dy[b][y/2][x/2] / 4
__global__ void pool_bwd_kernel(const float* __restrict__ dy, int lh, int lw, int C, size_t n, int accumulate,
                                float* __restrict__ dx) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int c = (int)(e % C);
  const size_t p = e / C;
  const int lhw = lh + lw;
  const size_t b = p >> lhw;
  const int y = (int)((p >> lw) & ((1 << lh) - 1)), x = (int)(p & ((1 << lw) - 1));
  const float v = 0.25f * dy[(((b << (lhw - 2)) + ((size_t)(y >> 1) << (lw - 1)) + (x >> 1)) * C) + c];
  dx[e] = accumulate ? dx[e] + v : v;
}

// Split the gradient of a dense conv input (channels [0,c0) from src0, maybe
// upsampled, then [c0, c0+c1) from src1) back onto its sources:
// ds0 (+)= (up0 ? sum of the 2x2 children : dd[.., :c0]), ds1 += dd[.., c0:].
// One thread per element of ds0 (at its own resolution) and of ds1.
__global__ void split_bwd_kernel(const float* __restrict__ dd, int c0, int up0, int c1, int lh, int lw,
                                 size_t n0, size_t n1, int acc0, float* __restrict__ ds0, float* __restrict__ ds1) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int cin = c0 + c1;
  const int lhw = lh + lw;
  if (e < n0) {
    const int c = (int)(e % c0);
    const size_t p = e / c0;
    float v;
    if (up0) {
      const int slw = lw - 1, slh = lh - 1;
      const size_t b = p >> (slh + slw);
      const int y = (int)((p >> slw) & ((1 << slh) - 1)), x = (int)(p & ((1 << slw) - 1));
      v = 0.f;
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx)
          v += dd[(((b << lhw) + ((size_t)(2 * y + dy) << lw) + (2 * x + dx)) * cin) + c];
    } else {
      v = dd[p * cin + c];
    }
    ds0[e] = acc0 ? ds0[e] + v : v;
  } else if (e < n0 + n1) {
    const size_t f = e - n0;
    const int c = (int)(f % c1);
    const size_t p = f / c1;
    ds1[f] += dd[p * cin + c0 + c];
  }
}

// AdamW on the flat master parameters (bias-corrected moments, decoupled decay).
__global__ void adamw_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                             float* __restrict__ v, size_t n, float lr, float b1, float b2, float eps, float wd,
                             float c1, float c2) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gi = g[e];
  const float mi = b1 * m[e] + (1.0f - b1) * gi;
  const float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
  m[e] = mi;
  v[e] = vi;
  const float mh = mi / c1, vh = vi / c2;
  w[e] = w[e] - lr * (mh / (__builtin_sqrtf(vh) + eps) + wd * w[e]);
}

inline unsigned blocks(size_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

void tr_relayout(hipStream_t st, const float* w, int co, int ci, int kk, int co_pad, float* fwd, float* flip) {
  const int n = co_pad * ci * kk;
  hipLaunchKernelGGL(relayout_kernel, dim3(blocks(n)), dim3(256), 0, st, w, co, ci, kk, co_pad, fwd, flip);
  TD_LAUNCHED();
}

void tr_lp_weights(hipStream_t st, const float* w, int co, int ci, int kk, int kp, int flip, uint16_t* out) {
  const int n = (flip ? ci : co) * kp;
  hipLaunchKernelGGL(lp_weights_kernel, dim3(blocks(n)), dim3(256), 0, st, w, co, ci, kk, kp, flip,
                     reinterpret_cast<__bf16*>(out));
  TD_LAUNCHED();
}

void tr_dense_in(hipStream_t st, const float* s0, int c0, int up0, const float* s1, int c1, int nb, int lh, int lw,
                 float* out) {
  const size_t n = ((size_t)nb << (lh + lw)) * (c0 + c1);
  hipLaunchKernelGGL(dense_in_kernel, dim3(blocks(n)), dim3(256), 0, st, s0, c0, up0, s1, c1, lh, lw, n, out);
  TD_LAUNCHED();
}

void tr_act(hipStream_t st, const float* x, const float* scale, const float* shift, int nb, int hw, int C, int act,
            float* out) {
  const size_t n = (size_t)nb * hw * C;
  hipLaunchKernelGGL(act_kernel, dim3(blocks(n)), dim3(256), 0, st, x, scale, shift, hw, C, act, n, out);
  TD_LAUNCHED();
}

void tr_gn_bwd(hipStream_t st, const float* x, const float* mean, const float* rstd, const float* gamma,
               const float* beta, const float* dA, int nb, int hw, int C, int groups, int act, int accumulate,
               float* dx, float* dgam_part, float* dbet_part) {
  TD_CHECK(C % groups == 0 && C / groups <= 256, -5, "groupnorm backward: at most 256 channels per group");
  hipLaunchKernelGGL(gn_bwd_kernel, dim3(nb, groups), dim3(256), 0, st, x, mean, rstd, gamma, beta, dA, hw, C,
                     groups, act, accumulate, dx, dgam_part, dbet_part);
  TD_LAUNCHED();
}

void tr_sum_rows(hipStream_t st, const float* in, int rows, int C, int accumulate, float* out) {
  hipLaunchKernelGGL(sum_rows_kernel, dim3(blocks(C)), dim3(256), 0, st, in, rows, C, accumulate, out);
  TD_LAUNCHED();
}

void tr_colsum(hipStream_t st, const float* in, size_t M, int C, float* part, int nchunk, int accumulate,
               float* out) {
  const int per = (int)((M + nchunk - 1) / nchunk);
  hipLaunchKernelGGL(colsum_part_kernel, dim3((C + 63) / 64, nchunk), dim3(256), 0, st, in, M, C, per, part);
  TD_LAUNCHED();
  tr_sum_rows(st, part, nchunk, C, accumulate, out);
}

void tr_wgrad(hipStream_t st, const float* A, const float* dY, int nb, int lh, int lw, int ci, int co, int taps,
              float* part, int nsplit, float* grad) {
  const size_t M = (size_t)nb << (lh + lw);
  int per = (int)((M + nsplit - 1) / nsplit);
  per = (per + WG_PIX - 1) / WG_PIX * WG_PIX;
  const int ns = (int)((M + per - 1) / per);
  dim3 grid((ci + 63) / 64, (co + 63) / 64, taps * ns);
  prof_begin(st);
  hipLaunchKernelGGL(wgrad_kernel, grid, dim3(256), 0, st, A, dY, lh, lw, ci, co, taps, M, per, part);
  TD_LAUNCHED();
  const int n = co * ci * taps;
  hipLaunchKernelGGL(wgrad_reduce_kernel, dim3(blocks(n)), dim3(256), 0, st, part, ns, taps, ci, co, grad);
  TD_LAUNCHED();
  prof_end(st, K_WGRAD, 2.0 * M * ci * co * taps, 4.0 * M * (ci + co) * taps);
}

void tr_attention_bwd(hipStream_t st, const float* qkv, const float* dO, int nb, int T, int C, int heads,
                      float* dqkv) {
  TD_CHECK(T <= 64 && C % heads == 0 && C / heads <= 64, -5, "attention backward: at most 64 tokens, head dim 64");
  hipLaunchKernelGGL(attention_bwd_kernel, dim3(nb, heads), dim3(256), 0, st, qkv, dO, T, C, heads, dqkv);
  TD_LAUNCHED();
}

void tr_emb_bwd(hipStream_t st, float c_noise, int c0, int emb, float max_period, const float* W1, const float* b1,
                const float* W2, const float* b2, const float* de2, float* dW1, float* db1, float* dW2, float* db2) {
  TD_CHECK(c0 <= 1024 && emb <= 1024, -5, "embedding backward: widths up to 1024");
  hipLaunchKernelGGL(emb_bwd_kernel, dim3(1), dim3(256), 0, st, c_noise, c0, emb, logf(max_period), W1, b1, W2, b2,
                     de2, dW1, db1, dW2, db2);
  TD_LAUNCHED();
}

void tr_emb_bias_bwd(hipStream_t st, const float* db, const float* e2, const float* Wemb, int cout, int emb,
                     float* dWemb, float* dbemb, float* dcb, float* de2) {
  const int n = cout * emb > emb ? cout * emb : emb;
  hipLaunchKernelGGL(emb_bias_bwd_kernel, dim3(blocks(n)), dim3(256), 0, st, db, e2, Wemb, cout, emb, dWemb, dbemb,
                     dcb, de2);
  TD_LAUNCHED();
}

void tr_mse(hipStream_t st, const float* D, const float* y, size_t n, float gscale, float* d, float* part) {
  hipLaunchKernelGGL(mse_kernel, dim3(blocks(n)), dim3(256), 0, st, D, y, n, gscale, d, part);
  TD_LAUNCHED();
}

void tr_pad_scale(hipStream_t st, const float* in, size_t npix, int C, int cpad, float s, float* out) {
  hipLaunchKernelGGL(pad_scale_kernel, dim3(blocks(npix * cpad)), dim3(256), 0, st, in, npix, C, cpad, s, out);
  TD_LAUNCHED();
}

void tr_add(hipStream_t st, float* a, const float* b, size_t n) {
  if (!n) return;
  hipLaunchKernelGGL(add_kernel, dim3(blocks(n)), dim3(256), 0, st, a, b, n);
  TD_LAUNCHED();
}

void tr_pool_bwd(hipStream_t st, const float* dy, int nb, int lh, int lw, int C, int accumulate, float* dx) {
  const size_t n = ((size_t)nb << (lh + lw)) * C;
  hipLaunchKernelGGL(pool_bwd_kernel, dim3(blocks(n)), dim3(256), 0, st, dy, lh, lw, C, n, accumulate, dx);
  TD_LAUNCHED();
}

void tr_split_bwd(hipStream_t st, const float* dd, int c0, int up0, int c1, int nb, int lh, int lw, int acc0,
                  float* ds0, float* ds1) {
  const size_t n0 = ((size_t)nb << (lh + lw - (up0 ? 2 : 0))) * c0;
  const size_t n1 = ((size_t)nb << (lh + lw)) * c1;
  hipLaunchKernelGGL(split_bwd_kernel, dim3(blocks(n0 + n1)), dim3(256), 0, st, dd, c0, up0, c1, lh, lw, n0, n1,
                     acc0, ds0, ds1);
  TD_LAUNCHED();
}

void tr_adamw(hipStream_t st, float* w, const float* g, float* m, float* v, size_t n, float lr, float b1, float b2,
              float eps, float wd, int step) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(adamw_kernel, dim3(blocks(n)), dim3(256), 0, st, w, g, m, v, n, lr, b1, b2, eps, wd, c1, c2);
  TD_LAUNCHED();
}

}  // namespace td
