// Laplacian decode of a terrain latent (Sec. 5.2) with the signed-sqrt
// inverse (signed-sqrt appendix), and the encode that builds such a latent
// from elevation (at the end of the file).
//
//   L = sigma_low * J0[.., 0]                   low band (signed-sqrt metres)
//   Hres(X, Y) = sum_k sigma_res * J0[Y/8, X/8, k] * beta_k(X mod 8, Y mod 8)
//                (orthonormal 8x8 DCT-II atoms (1,0), (0,1), (1,1); k = 1..3)
//   P = up8(L) + Hres,  L_hat = G5 * down8(P),  z = up8(L_hat) + Hres,
//   elevation = sign(z) z^2
// up8 is bilinear with half-pixel centres (xi = (X + 0.5)/8 - 0.5), down8 the
// 8x8 block mean, G5 the separable sigma = 5 Gaussian (radius 15) at latent
// resolution.  There is no padding: the latent covers a 17-pixel apron.
//
// Stages: (1) down8(P) per latent block as a 3x3 stencil on the latent;
// (2) vertical then (3) horizontal 31-tap blur at latent resolution -- one
// LDS-tiled launch for blur radii up to 24, two beyond; (4) the
// full-resolution pass, 8 x 1024-pixel tiles with their inputs staged in
// LDS, which is the HBM-bound one (4 B written per pixel, the latent read
// once).
#include "td_internal.h"

#include <mutex>

namespace td {
namespace {

struct Span {
  int64_t xl, xh, yl, yh;   // latent range of L_hat read by up8
};

__host__ __device__ inline int64_t floordiv(int64_t a, int64_t b) {
  int64_t q = a / b;
  return (q * b > a) ? q - 1 : q;
}

inline Span span_of(const DecodeArgs& a) {
  Span s;
  s.xl = floordiv(2 * a.X0 - 7, 16);
  s.xh = floordiv(2 * (a.X0 + a.W - 1) - 7, 16) + 1;
  s.yl = floordiv(2 * a.Y0 - 7, 16);
  s.yh = floordiv(2 * (a.Y0 + a.H - 1) - 7, 16) + 1;
  return s;
}

// (1) D(bx, by) = mean of P over latent block (bx, by).  Bilinear
// half-pixel up8 followed by the 8x8 block mean is exactly the separable
// stencil [1, 6, 1]/8 on the latent grid; the residual contributes
// sum_k r_k * mean(beta_k) (the atom means are zero up to rounding of the
// table).  Block origin relative to the latent origin: (bx0 + i, by0 + j).
__device__ __forceinline__ float down_p_at(const float* __restrict__ lat, int lw, int C, float sl, float sr,
                                           const float* __restrict__ atom_mean, int x, int y) {
  const float* r0 = lat + ((size_t)(y - 1) * lw + x - 1) * C;
  const float* r1 = r0 + (size_t)lw * C;
  const float* r2 = r1 + (size_t)lw * C;
  float a = (r0[0] + 6.f * r0[C] + r0[2 * C]) * 0.125f;
  float b = (r1[0] + 6.f * r1[C] + r1[2 * C]) * 0.125f;
  float c = (r2[0] + 6.f * r2[C] + r2[2 * C]) * 0.125f;
  float d = sl * ((a + 6.f * b + c) * 0.125f);
  int nk = C - 1 < 3 ? C - 1 : 3;
  float h = 0.f;
  for (int k = 0; k < nk; ++k) h += r1[C + 1 + k] * atom_mean[k];
  return d + sr * h;
}

__global__ __launch_bounds__(256) void down_p_kernel(const float* __restrict__ lat, int lw, int C, float sl,
                                                     float sr, const float* __restrict__ atom_mean, int bx0,
                                                     int by0, int nx, int ny, float* __restrict__ D) {
  int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= nx * ny) return;
  int j = e / nx, i = e % nx;
  D[e] = down_p_at(lat, lw, C, sl, sr, atom_mean, bx0 + i, by0 + j);
}

// (2) vertical blur: out[j][i] = sum_t g[t] in[j + t][i], out rows ny_out
__global__ __launch_bounds__(256) void blur_v_kernel(const float* __restrict__ in, int nx, int ny_out,
                                                     const float* __restrict__ g, int R, float* __restrict__ out) {
  int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= nx * ny_out) return;
  int j = e / nx, i = e % nx;
  float s = 0.f;
  for (int t = 0; t <= 2 * R; ++t) s += g[t] * in[(size_t)(j + t) * nx + i];
  out[e] = s;
}

// (3) horizontal blur: out[j][i] = sum_t g[t] in[j][i + t], in width nx_in
__global__ __launch_bounds__(256) void blur_h_kernel(const float* __restrict__ in, int nx_in, int nx_out, int ny,
                                                     const float* __restrict__ g, int R, float* __restrict__ out) {
  int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= nx_out * ny) return;
  int j = e / nx_out, i = e % nx_out;
  float s = 0.f;
  for (int t = 0; t <= 2 * R; ++t) s += g[t] * in[(size_t)j * nx_in + i + t];
  out[e] = s;
}

// (2) and (3) in one launch for blur radii up to kFusedR: a workgroup makes
// a kBx x kBy tile of the blurred grid.  Its input patch of the D grid
// [nyD][nxD] (the tile plus the 2R apron) goes to LDS, the vertical pass
// into a second LDS array, then the horizontal pass to out [ny][nx], every
// sum taking its taps in the order of blur_v_kernel and blur_h_kernel (the
// results are the two kernels' bit for bit).  nxD = nx + 2R, nyD = ny + 2R.
constexpr int kBx = 64, kBy = 32, kFusedR = 24;
__global__ __launch_bounds__(256) void blur2d_kernel(const float* __restrict__ src, int nxD, int nyD,
                                                     const float* __restrict__ g, int R, int nx, int ny,
                                                     float* __restrict__ out) {
  extern __shared__ float sm[];
  const int TXR = kBx + 2 * R, TYR = kBy + 2 * R;
  float* in = sm;                      // [TYR][TXR]
  float* V = sm + TYR * TXR;           // [kBy][TXR]
  const int x0 = blockIdx.x * kBx, y0 = blockIdx.y * kBy;
  // U patch elements per thread in flight; positions past the grid are
  // clamped into it (their values feed only outputs past nx, ny, which are
  // not written), so every load is unconditional
  constexpr int U = 8;
  const int n_in = TYR * TXR;
  for (int e0 = threadIdx.x; e0 < n_in; e0 += 256 * U) {
    float v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = min(e0 + 256 * u, n_in - 1);
      const int r = e / TXR, c = e - r * TXR;
      const int i = min(x0 + c, nxD - 1), j = min(y0 + r, nyD - 1);
      v[u] = src[(size_t)j * nxD + i];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (e0 + 256 * u < n_in) in[e0 + 256 * u] = v[u];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kBy * TXR; e += 256) {
    const int r = e / TXR, c = e - r * TXR;
    float acc = 0.f;
    for (int t = 0; t <= 2 * R; ++t) acc += g[t] * in[(r + t) * TXR + c];
    V[e] = acc;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kBy * kBx; e += 256) {
    const int r = e / kBx, c = e - r * kBx;
    const int i = x0 + c, j = y0 + r;
    if (i >= nx || j >= ny) continue;
    float acc = 0.f;
    for (int t = 0; t <= 2 * R; ++t) acc += g[t] * V[r * TXR + c + t];
    out[(size_t)j * nx + i] = acc;
  }
}

size_t blur2d_lds_bytes(int R) { return sizeof(float) * (size_t)(kBx + 2 * R) * (kBy + 2 * R + kBy); }

// (4) full resolution: z = up8(L_hat) + Hres, elevation = sign(z) z^2.
// A workgroup writes a tile of 8 rows x 1024 columns; the L_hat rows and
// columns, the residual latents of the (at most 2 x 130) blocks it covers
// and the atom table are staged in LDS once, so each output pixel costs LDS
// reads and its share of one 16-byte store.
constexpr int kTileW = 1024, kTileH = 8;
__global__ __launch_bounds__(256) void decode_out_kernel(const float* __restrict__ lat, int lw, int lh, int C, float sr,
                                                         const float* __restrict__ atoms,
                                                         const float* __restrict__ lhat, int nlx, int nly, int hx0,
                                                         int hy0, int xo, int yo, int W, int H,
                                                         float* __restrict__ out) {
  __shared__ float sl[3][kTileW / 8 + 4];        // L_hat rows iy0..iy0+2, columns ix0..
  __shared__ float sres[2][kTileW / 8 + 2][3];   // residual latents of blocks by0.., bx0..
  __shared__ float sat[3 * 64];
  const int tid = threadIdx.x;
  const int X0 = blockIdx.x * kTileW, Y0 = blockIdx.y * kTileH;
  const int Xa = xo + X0, Ya = yo + Y0;                   // relative full-res coordinates (>= 8)
  const int ix0 = ((2 * Xa - 7) >> 4) - hx0, iy0 = ((2 * Ya - 7) >> 4) - hy0;
  const int bx0 = Xa >> 3, by0 = Ya >> 3;
  const int nk = C - 1 < 3 ? C - 1 : 3;
  for (int e = tid; e < 3 * (kTileW / 8 + 4); e += 256) {
    const int r = e / (kTileW / 8 + 4), c = e % (kTileW / 8 + 4);
    const int gy = iy0 + r, gx = ix0 + c;
    sl[r][c] = (gy < nly && gx < nlx) ? lhat[(size_t)gy * nlx + gx] : 0.f;
  }
  for (int e = tid; e < 2 * (kTileW / 8 + 2) * 3; e += 256) {
    const int k = e % 3, c = (e / 3) % (kTileW / 8 + 2), r = e / (3 * (kTileW / 8 + 2));
    const int gy = by0 + r, gx = bx0 + c;
    float v = 0.f;
    if (k < nk && gx < lw && gy < lh) v = lat[((size_t)gy * lw + gx) * C + 1 + k];
    sres[r][c][k] = v;
  }
  for (int e = tid; e < 3 * 64; e += 256) sat[e] = e < nk * 64 ? atoms[e] : 0.f;
  __syncthreads();
  const int X = X0 + 4 * tid;
  if (X >= W) return;
  for (int yy = 0; yy < kTileH; ++yy) {
    const int Y = Y0 + yy;
    if (Y >= H) break;
    const int Yr = yo + Y;
    const int ty = (2 * Yr - 7) >> 4;
    const int ry = ty - hy0 - iy0;
    const float fy = (float)((2 * Yr - 7) - 16 * ty) * 0.0625f;
    const int rb = (Yr >> 3) - by0;
    float v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int Xr = xo + X + q;
      const int tx = (2 * Xr - 7) >> 4;
      const int cx = tx - hx0 - ix0;
      const float fx = (float)((2 * Xr - 7) - 16 * tx) * 0.0625f;
      const float a0 = (1.f - fy) * sl[ry][cx] + fy * sl[ry + 1][cx];
      const float a1 = (1.f - fy) * sl[ry][cx + 1] + fy * sl[ry + 1][cx + 1];
      const int a = (Yr & 7) * 8 + (Xr & 7);
      const float* rr = sres[rb][(Xr >> 3) - bx0];
      const float h = sr * ((rr[0] * sat[a] + rr[1] * sat[64 + a]) + rr[2] * sat[128 + a]);
      const float z = (1.f - fx) * a0 + fx * a1 + (C < 2 ? 0.f : h);
      v[q] = (z < 0.f ? -z : z) * z;
    }
    float* o = out + (size_t)Y * W + X;
    if (X + 3 < W && (((uintptr_t)o) & 15) == 0) {
      *reinterpret_cast<float4*>(o) = make_float4(v[0], v[1], v[2], v[3]);
    } else {
      for (int q = 0; q < 4 && X + q < W; ++q) o[q] = v[q];
    }
  }
}

// ---------------------------------------------------------------- encode
// Elevation -> latent on an 8-aligned full-resolution region: z = sign(h)
// sqrt|h|; D = down8(z); L = G5 * D (valid: the region shrinks by R blocks a
// side); for each output block (one more block in, for up8) the low band
// L / sigma_low and the residual coefficients <z - up8(L), beta_k> /
// sigma_res of the 8 x 8 block.  Heights are read twice (stages e1 and e3).
__device__ __forceinline__ float ssqrt(float h) { return copysignf(sqrtf(fabsf(h)), h); }

// (e1) D(bx, by) = mean over block (bx, by) of sign(h) sqrt|h|
__global__ __launch_bounds__(256) void enc_down_kernel(const float* __restrict__ h, int W, int nbx, int nby,
                                                       float* __restrict__ D) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= nbx * nby) return;
  const int by = e / nbx, bx = e % nbx;
  const float* p = h + (size_t)(8 * by) * W + 8 * bx;
  float s = 0.f;
  for (int r = 0; r < 8; ++r) {
    const float4 a = *reinterpret_cast<const float4*>(p + (size_t)r * W);
    const float4 b = *reinterpret_cast<const float4*>(p + (size_t)r * W + 4);
    s += ((ssqrt(a.x) + ssqrt(a.y)) + (ssqrt(a.z) + ssqrt(a.w))) + ((ssqrt(b.x) + ssqrt(b.y)) + (ssqrt(b.z) + ssqrt(b.w)));
  }
  D[e] = s * (1.f / 64.f);
}

// (e3) output block (R + 1 + i, R + 1 + j) of the region: L is [nly][nlx]
// at block offset R; writes lat[j][i][0..C)
__global__ __launch_bounds__(256) void enc_res_kernel(const float* __restrict__ h, int W, const float* __restrict__ L,
                                                      int nlx, int ow, int oh, int R, int C, float inv_sl,
                                                      float inv_sr, const float* __restrict__ atoms,
                                                      float* __restrict__ lat) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= ow * oh) return;
  const int j = e / ow, i = e % ow;
  const int bx = R + 1 + i, by = R + 1 + j;             // block in the region
  const int lx = bx - R, ly = by - R;                   // the same block in L
  float l3[3][3];
  for (int dy = 0; dy < 3; ++dy)
    for (int dx = 0; dx < 3; ++dx) l3[dy][dx] = L[(size_t)(ly - 1 + dy) * nlx + (lx - 1 + dx)];
  const int nk = C - 1 < 3 ? C - 1 : 3;
  float r[3] = {0.f, 0.f, 0.f};
  const float* p = h + (size_t)(8 * by) * W + 8 * bx;
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const int ty = v < 4 ? 0 : 1;                        // rows (ly - 1 + ty, ly + ty) of L
    const float fy = (float)(v < 4 ? 2 * v + 9 : 2 * v - 7) * 0.0625f;
    const float4 q0 = *reinterpret_cast<const float4*>(p + (size_t)v * W);
    const float4 q1 = *reinterpret_cast<const float4*>(p + (size_t)v * W + 4);
    const float hv[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int tx = u < 4 ? 0 : 1;
      const float fx = (float)(u < 4 ? 2 * u + 9 : 2 * u - 7) * 0.0625f;
      const float a0 = (1.f - fy) * l3[ty][tx] + fy * l3[ty + 1][tx];
      const float a1 = (1.f - fy) * l3[ty][tx + 1] + fy * l3[ty + 1][tx + 1];
      const float res = ssqrt(hv[u]) - ((1.f - fx) * a0 + fx * a1);
      for (int k = 0; k < nk; ++k) r[k] += res * atoms[k * 64 + v * 8 + u];
    }
  }
  float* o = lat + (size_t)e * C;
  o[0] = l3[1][1] * inv_sl;
  for (int k = 1; k < C; ++k) o[k] = k <= nk ? r[k - 1] * inv_sr : 0.f;
}

}  // namespace

// Fixed decode scratch for callers that cannot allocate device memory
// (td_lap_decode_noalloc): one array per GPU, whose device address is looked
// up once per device.  In host code the array's name is not a device
// address; only the looked-up pointer is passed to kernels.
static __device__ __align__(256) float scratch[kDecodeScratchFloats];

namespace {
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

void init_decode_scratch(int device) {
  TD_CHECK(device >= 0 && device < kMaxDevices, -1, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void* p = nullptr;
  TD_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));   // the current device's copy
  TD_CHECK(p, -3, "decode scratch has no device address");
  g_scratch_ptr[device] = static_cast<float*>(p);
}

float* decode_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

size_t decode_work_floats(const DecodeArgs& a) {
  Span s = span_of(a);
  size_t nx = (size_t)(s.xh - s.xl + 1 + 2 * a.radius), ny = (size_t)(s.yh - s.yl + 1 + 2 * a.radius);
  return nx * ny;
}

void launch_decode(hipStream_t st, const DecodeArgs& a) {
  Span s = span_of(a);
  const int R = a.radius;
  // latent needed: [xl - R - 1, xh + R + 1] (bilinear inside P) and blocks of the output
  TD_CHECK(s.xl - R - 1 >= a.lx0 && s.yl - R - 1 >= a.ly0 && s.xh + R + 1 < a.lx0 + a.lw &&
               s.yh + R + 1 < a.ly0 + a.lh,
           -1, "decode: latent does not cover the 17-pixel apron");
  const int nxD = (int)(s.xh - s.xl + 1 + 2 * R), nyD = (int)(s.yh - s.yl + 1 + 2 * R);
  const int nx = (int)(s.xh - s.xl + 1), ny = (int)(s.yh - s.yl + 1);
  const int bx0 = (int)(s.xl - R - a.lx0), by0 = (int)(s.yl - R - a.ly0);
  prof_begin(st);
  const float* lhat = a.work0;
  if (R <= kFusedR) {
    // D into work0, then both blur passes in one launch into work1
    hipLaunchKernelGGL(down_p_kernel, dim3((nxD * nyD + 255) / 256), dim3(256), 0, st, a.latent, a.lw, a.C,
                       a.sigma_low, a.sigma_res, a.atoms + 3 * 64, bx0, by0, nxD, nyD, a.work0);
    TD_LAUNCHED();
    hipLaunchKernelGGL(blur2d_kernel, dim3((nx + kBx - 1) / kBx, (ny + kBy - 1) / kBy), dim3(256),
                       blur2d_lds_bytes(R), st, a.work0, nxD, nyD, a.taps, R, nx, ny, a.work1);
    TD_LAUNCHED();
    lhat = a.work1;
  } else {
    hipLaunchKernelGGL(down_p_kernel, dim3((nxD * nyD + 255) / 256), dim3(256), 0, st, a.latent, a.lw, a.C,
                       a.sigma_low, a.sigma_res, a.atoms + 3 * 64, bx0, by0, nxD, nyD, a.work0);
    TD_LAUNCHED();
    hipLaunchKernelGGL(blur_v_kernel, dim3((nxD * ny + 255) / 256), dim3(256), 0, st, a.work0, nxD, ny, a.taps, R,
                       a.work1);
    TD_LAUNCHED();
    hipLaunchKernelGGL(blur_h_kernel, dim3((nx * ny + 255) / 256), dim3(256), 0, st, a.work1, nxD, nx, ny, a.taps, R,
                       a.work0);
    TD_LAUNCHED();
  }
  const int xo = (int)(a.X0 - 8 * a.lx0), yo = (int)(a.Y0 - 8 * a.ly0);
  hipLaunchKernelGGL(decode_out_kernel, dim3((a.W + kTileW - 1) / kTileW, (a.H + kTileH - 1) / kTileH), dim3(256), 0,
                     st, a.latent, a.lw, a.lh, a.C, a.sigma_res, a.atoms, lhat, nx, ny, (int)(s.xl - a.lx0),
                     (int)(s.yl - a.ly0), xo, yo, a.W, a.H, a.out);
  TD_LAUNCHED();
  prof_end(st, K_DECODE, 20.0 * a.W * a.H, 4.0 * (double)a.W * a.H + 4.0 * (double)nxD * nyD * a.C);
}

void launch_encode(hipStream_t st, const EncodeArgs& a) {
  const int R = a.radius;
  TD_CHECK(a.W % 8 == 0 && a.H % 8 == 0, -1, "encode: region sides must be multiples of 8");
  const int nbx = a.W / 8, nby = a.H / 8;
  const int nlx = nbx - 2 * R, nly = nby - 2 * R, ow = nlx - 2, oh = nly - 2;
  TD_CHECK(ow >= 1 && oh >= 1, -1, "encode: region too small for the blur and up8 aprons");
  prof_begin(st);
  hipLaunchKernelGGL(enc_down_kernel, dim3((nbx * nby + 255) / 256), dim3(256), 0, st, a.height, a.W, nbx, nby,
                     a.work0);
  TD_LAUNCHED();
  const float* L = a.work0;
  if (R <= kFusedR) {
    // L into work1 in one launch
    hipLaunchKernelGGL(blur2d_kernel, dim3((nlx + kBx - 1) / kBx, (nly + kBy - 1) / kBy), dim3(256),
                       blur2d_lds_bytes(R), st, a.work0, nbx, nby, a.taps, R, nlx, nly, a.work1);
    TD_LAUNCHED();
    L = a.work1;
  } else {
    hipLaunchKernelGGL(blur_v_kernel, dim3((nbx * nly + 255) / 256), dim3(256), 0, st, a.work0, nbx, nly, a.taps, R,
                       a.work1);
    TD_LAUNCHED();
    hipLaunchKernelGGL(blur_h_kernel, dim3((nlx * nly + 255) / 256), dim3(256), 0, st, a.work1, nbx, nlx, nly,
                       a.taps, R, a.work0);
    TD_LAUNCHED();
  }
  hipLaunchKernelGGL(enc_res_kernel, dim3((ow * oh + 255) / 256), dim3(256), 0, st, a.height, a.W, L, nlx, ow, oh, R,
                     a.C, 1.f / a.sigma_low, 1.f / a.sigma_res, a.atoms, a.latent);
  TD_LAUNCHED();
  prof_end(st, K_ENCODE, 12.0 * a.W * a.H, 8.0 * (double)a.W * a.H + 4.0 * (double)ow * oh * a.C);
}

}  // namespace td
