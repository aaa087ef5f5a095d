// Overlap blend of window contributions (InfiniteDiffusion update, Eq. 2):
//   J_t(p) = sum_{i in kappa(p)} V_i(p - o_i) / sum_{i in kappa(p)} W(p - o_i),
// V_i = W (x) Phi_i stored per window (Sec. 3.3), 0/0 := 0 (formal appendix).
// The denominator is recomputed from the separable weight table instead of
// being stored.  Windows are summed in canonical order (iy, then ix
// ascending), so a pixel's value does not depend on the region it was
// queried with.  One thread per pixel; all channels of a contribution pixel
// are contiguous, so threads along x read consecutive addresses of the
// same window.  HBM-bound: (H/s)^2 contribution reads + one write per value.
//
// Also here: the analytic linear-Gaussian window step (posterior mean of a
// Gaussian prior, Euler step, weighting), used to check the sampler
// machinery against a closed form.
#include "td_internal.h"

namespace td {
namespace {

__device__ __forceinline__ int ceil_div_i(int a, int s) { return a >= 0 ? (a + s - 1) / s : -((-a) / s); }
__device__ __forceinline__ int floor_div_i(int a, int s) { return a >= 0 ? a / s : -((-a + s - 1) / s); }

template <int CC>
__global__ __launch_bounds__(256) void blend_kernel(int H, int S, int C, int rx0, int ry0, int w, int h,
                                                    int nx, int ny, const float* const* __restrict__ ptrs,
                                                    const float* __restrict__ w1d, int layout,
                                                    float* __restrict__ out) {
  const int nc = CC > 0 ? CC : C;
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= w * h) return;
  int ry = idx / w, rx = idx - ry * w;
  int px = rx0 + rx, py = ry0 + ry;
  int xlo = max(0, ceil_div_i(px - H + 1, S)), xhi = min(nx - 1, floor_div_i(px, S));
  int ylo = max(0, ceil_div_i(py - H + 1, S)), yhi = min(ny - 1, floor_div_i(py, S));
  float acc[CC > 0 ? CC : 4];
  float bsum = 0.f;
  if (CC > 0) {
#pragma unroll
    for (int c = 0; c < (CC > 0 ? CC : 4); ++c) acc[c] = 0.f;
  }
  for (int c = 0; CC == 0 && c < 4; ++c) acc[c] = 0.f;
  for (int iy = ylo; iy <= yhi; ++iy) {
    int v = py - iy * S;
    float wv = w1d[v];
    for (int ix = xlo; ix <= xhi; ++ix) {
      int u = px - ix * S;
      bsum += w1d[u] * wv;
      const float* p = ptrs[iy * nx + ix] + ((size_t)v * H + u) * nc;
      if (CC == 4) {
        float4 q = *reinterpret_cast<const float4*>(p);
        acc[0] += q.x; acc[1] += q.y; acc[2] += q.z; acc[3] += q.w;
      } else if (CC == 1) {
        acc[0] += p[0];
      }
    }
  }
  if (CC > 0) {
#pragma unroll
    for (int c = 0; c < (CC > 0 ? CC : 4); ++c) {
      float r = bsum > 0.f ? acc[c] / bsum : 0.f;
      if (layout == 0) out[(size_t)idx * nc + c] = r;
      else out[(size_t)c * w * h + idx] = r;
    }
  }
}

// Generic channel count: one pass per channel (C not 1 or 4).
__global__ __launch_bounds__(256) void blend_generic(int H, int S, int C, int rx0, int ry0, int w, int h,
                                                     int nx, int ny, const float* const* __restrict__ ptrs,
                                                     const float* __restrict__ w1d, int layout,
                                                     float* __restrict__ out) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= w * h) return;
  int ry = idx / w, rx = idx - ry * w;
  int px = rx0 + rx, py = ry0 + ry;
  int xlo = max(0, ceil_div_i(px - H + 1, S)), xhi = min(nx - 1, floor_div_i(px, S));
  int ylo = max(0, ceil_div_i(py - H + 1, S)), yhi = min(ny - 1, floor_div_i(py, S));
  for (int c = 0; c < C; ++c) {
    float acc = 0.f, bsum = 0.f;
    for (int iy = ylo; iy <= yhi; ++iy) {
      int v = py - iy * S;
      for (int ix = xlo; ix <= xhi; ++ix) {
        int u = px - ix * S;
        bsum += w1d[u] * w1d[v];
        acc += ptrs[iy * nx + ix][((size_t)v * H + u) * C + c];
      }
    }
    float r = bsum > 0.f ? acc / bsum : 0.f;
    if (layout == 0) out[(size_t)idx * C + c] = r;
    else out[(size_t)c * w * h + idx] = r;
  }
}

__device__ __forceinline__ int floor_mod(int a, int m) {
  int r = a % m;
  return r < 0 ? r + m : r;
}

__global__ __launch_bounds__(256) void lg_step_kernel(int H, int C, const float* __restrict__ canvas,
                                                      int canvas_w, const int* __restrict__ origins,
                                                      const int* __restrict__ widx,
                                                      const float* __restrict__ cond, int cc, float a_post,
                                                      float c_euler, int direct, const float* __restrict__ w1d,
                                                      float* const* __restrict__ slots, int mode,
                                                      float* __restrict__ dout) {
  int b = blockIdx.y;
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= H * H * C) return;
  int c = idx % C;
  int pix = idx / C;
  int v = pix / H, u = pix - v * H;
  int ox = origins[2 * b], oy = origins[2 * b + 1];
  float x = canvas[((size_t)(oy + v) * canvas_w + ox + u) * C + c];
  int ix = widx[2 * b], iy = widx[2 * b + 1];
  float mu = 0.1f * (float)(floor_mod(ix, 7) - 3) - 0.05f * (float)(floor_mod(iy, 5) - 2) + 0.01f * (float)c;
  if (cc) mu += cond[((size_t)b * H * H + pix) * cc + c % cc];
  float d = mu + a_post * (x - mu);
  if (mode == 1) {
    dout[(size_t)b * H * H * C + idx] = d;
    return;
  }
  float phi = direct ? d : x + c_euler * (x - d);
  if (mode == 2) dout[(size_t)b * H * H * C + idx] = phi;
  else slots[b][idx] = (w1d[u] * w1d[v]) * phi;
}

// Window gather: out[b][v][u][c] = src[b][(v * pitch[b] + u) * C + c].
__global__ __launch_bounds__(256) void gather_kernel(const float* const* __restrict__ src,
                                                     const int* __restrict__ pitch, int H, int C,
                                                     float* __restrict__ out) {
  const int b = blockIdx.y;
  const int per = H * H * C;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= per) return;
  const int c = e % C, p = e / C;
  const int v = p / H, u = p - v * H;
  out[(size_t)b * per + e] = src[b][((size_t)v * pitch[b] + u) * C + c];
}

// Conditioning windows: nearest upsampling of a parent-resolution canvas.
__global__ __launch_bounds__(256) void cond_gather_kernel(const CondSrc* __restrict__ src, int H, int cc,
                                                          int factor, float* __restrict__ out) {
  const int b = blockIdx.y;
  const int per = H * H * cc;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= per) return;
  const int c = e % cc, p = e / cc;
  const int v = p / H, u = p - v * H;
  const CondSrc s = src[b];
  const int py = (s.offy + v) / factor, px = (s.offx + u) / factor;
  out[(size_t)b * per + e] = s.base[((size_t)py * s.pitch + px) * cc + c];
}

// Judge: one workgroup per window.  Fixed-order reduction (thread-strided
// partial sums, then a fixed tree), so the decision does not depend on the
// batch a window is in.  flags[b] = 1 where the RMS of ds - dt over the
// window exceeds thr.
__global__ __launch_bounds__(256) void judge_kernel(const float* __restrict__ ds, const float* __restrict__ dt,
                                                    int H, int C, float thr, int* __restrict__ flags,
                                                    unsigned long long* __restrict__ counter) {
  __shared__ float red[256];
  const int b = blockIdx.x;
  const int n = H * H * C;
  const float* s = ds + (size_t)b * n;
  const float* t = dt + (size_t)b * n;
  float acc = 0.f;
  for (int e = threadIdx.x; e < n; e += 256) {
    const float q = s[e] - t[e];
    acc += q * q;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const bool fall = __builtin_sqrtf(red[0] / (float)n) > thr;
    flags[b] = fall ? 1 : 0;
    if (fall && counter) atomicAdd(counter, 1ull);
  }
}

// slots[b] = W (x) (pos[b] < 0 ? ds[b] : fb[pos[b]])
__global__ __launch_bounds__(256) void select_kernel(const float* __restrict__ ds, const float* __restrict__ fb,
                                                     const int* __restrict__ pos, int H, int C,
                                                     const float* __restrict__ w1d, float* const* __restrict__ slots) {
  const int b = blockIdx.y;
  const int per = H * H * C;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= per) return;
  const int p = e / C;
  const int v = p / H, u = p - v * H;
  const int k = pos[b];
  const float x = k < 0 ? ds[(size_t)b * per + e] : fb[(size_t)k * per + e];
  slots[b][e] = (w1d[u] * w1d[v]) * x;
}

}  // namespace

void launch_judge(hipStream_t st, const float* ds, const float* dt, int nwin, int H, int C, float thr, int* flags,
                  unsigned long long* counter) {
  if (!nwin) return;
  prof_begin(st);
  hipLaunchKernelGGL(judge_kernel, dim3(nwin), dim3(256), 0, st, ds, dt, H, C, thr, flags, counter);
  TD_LAUNCHED();
  const double n = (double)nwin * H * H * C;
  prof_end(st, K_BLEND, 3.0 * n, 8.0 * n);
}

void launch_select(hipStream_t st, const float* ds, const float* fb, const int* pos, int nwin, int H, int C,
                   const float* w1d, float* const* slots) {
  if (!nwin) return;
  const int per = H * H * C;
  hipLaunchKernelGGL(select_kernel, dim3((per + 255) / 256, nwin), dim3(256), 0, st, ds, fb, pos, H, C, w1d, slots);
  TD_LAUNCHED();
}

void launch_cond_gather(hipStream_t st, const CondSrc* src, int nb, int H, int cc, int factor, float* out) {
  if (!nb) return;
  TD_CHECK(cc >= 1 && factor >= 1, -5, "conditioning gather: bad channels or factor");
  const int per = H * H * cc;
  prof_begin(st);
  hipLaunchKernelGGL(cond_gather_kernel, dim3((per + 255) / 256, nb), dim3(256), 0, st, src, H, cc, factor, out);
  TD_LAUNCHED();
  prof_end(st, K_GATHER, 0.0, 8.0 * per * nb);
}

void launch_gather(hipStream_t st, const float* const* src, const int* pitch, int nb, int H, int C, float* out) {
  if (!nb) return;
  const int per = H * H * C;
  prof_begin(st);
  hipLaunchKernelGGL(gather_kernel, dim3((per + 255) / 256, nb), dim3(256), 0, st, src, pitch, H, C, out);
  TD_LAUNCHED();
  prof_end(st, K_GATHER, 0.0, 8.0 * per * nb);
}

void launch_blend(hipStream_t st, const WinGeom& g, int rx0, int ry0, int w, int h, int nx, int ny,
                  const float* const* ptrs, const float* w1d, int layout, float* out) {
  int n = w * h;
  if (!n) return;
  dim3 grid((n + 255) / 256);
  prof_begin(st);
  if (g.channels == 4)
    hipLaunchKernelGGL(blend_kernel<4>, grid, dim3(256), 0, st, g.size, g.stride, 4, rx0, ry0, w, h, nx,
                       ny, ptrs, w1d, layout, out);
  else if (g.channels == 1)
    hipLaunchKernelGGL(blend_kernel<1>, grid, dim3(256), 0, st, g.size, g.stride, 1, rx0, ry0, w, h, nx,
                       ny, ptrs, w1d, layout, out);
  else
    hipLaunchKernelGGL(blend_generic, grid, dim3(256), 0, st, g.size, g.stride, g.channels, rx0, ry0, w,
                       h, nx, ny, ptrs, w1d, layout, out);
  TD_LAUNCHED();
  const double cov = (double)((g.size + g.stride - 1) / g.stride) * ((g.size + g.stride - 1) / g.stride);
  prof_end(st, K_BLEND, (double)n * g.channels * (cov + 1), 4.0 * n * g.channels * (cov + 1));
}

void launch_lg_step(hipStream_t st, const WinGeom& g, const float* canvas, int canvas_w,
                    const int* origins, const int* widx, const float* cond, int cc, int nwin,
                    double prior_std, double sigma,
                    float c_euler, int direct, const float* w1d, float* const* slots, int mode, float* dout) {
  if (!nwin) return;
  TD_CHECK(cc == 0 || cond, -5, "conditioned denoiser run without conditioning");
  int per = g.size * g.size * g.channels;
  double s2 = prior_std * prior_std;
  float a_post = (float)(s2 / (s2 + sigma * sigma));
  prof_begin(st);
  hipLaunchKernelGGL(lg_step_kernel, dim3((per + 255) / 256, nwin), dim3(256), 0, st, g.size, g.channels,
                     canvas, canvas_w, origins, widx, cond, cc, a_post, c_euler, direct, w1d, slots, mode, dout);
  TD_LAUNCHED();
  prof_end(st, K_LG, 6.0 * per * nwin, 8.0 * per * nwin);
}

}  // namespace td
