// Kernel micro-benchmark driver for profiler runs: launches one library
// convolution kernel at a given layer shape (random operands) after a plain
// copy kernel of known size, the reference that scales hardware byte
// counters.  Not part of the C-ABI; built beside the library.
//
//   kbench f32  L CIN COUT NB RES      3x3 FP32 (launch_conv), RES = 1 adds a residual input
//   kbench bf16 L CIN COUT NB TAPS OUT BF16 halo-staged (launch_conv_lp), TAPS 9 or 1,
//                                      OUT 0 = FP32 output, 1 = BF16 output + GroupNorm sums,
//                                      2 = FP32 output + a residual input
//
// Square images of side 2^L, NB windows; one warm-up and one timed launch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "td_internal.h"

using namespace td;

namespace {

#define KB_CHECK(x)                                                                     \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess) {                                                             \
      std::fprintf(stderr, "kbench: %s failed: %s\n", #x, hipGetErrorString(e_));       \
      std::exit(1);                                                                     \
    }                                                                                   \
  } while (0)

__global__ void copy_kernel(const float4* __restrict__ a, float4* __restrict__ b, size_t n) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) b[i] = a[i];
}

uint16_t bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

template <class T>
T* upload(const std::vector<T>& v) {
  T* p = nullptr;
  KB_CHECK(hipMalloc(&p, v.size() * sizeof(T)));
  KB_CHECK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return p;
}

// 256 MiB read and 256 MiB written.
void copy_reference() {
  const size_t n = (size_t)16 << 20;   // float4 elements
  float4 *a = nullptr, *b = nullptr;
  KB_CHECK(hipMalloc(&a, n * sizeof(float4)));
  KB_CHECK(hipMalloc(&b, n * sizeof(float4)));
  KB_CHECK(hipMemset(a, 0, n * sizeof(float4)));
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, 0, a, b, n);
  KB_CHECK(hipGetLastError());
  KB_CHECK(hipDeviceSynchronize());
  KB_CHECK(hipFree(a));
  KB_CHECK(hipFree(b));
}

template <class F>
float time_once(F&& launch) {
  hipEvent_t e0, e1;
  KB_CHECK(hipEventCreate(&e0));
  KB_CHECK(hipEventCreate(&e1));
  launch();
  KB_CHECK(hipDeviceSynchronize());
  KB_CHECK(hipEventRecord(e0));
  launch();
  KB_CHECK(hipEventRecord(e1));
  KB_CHECK(hipEventSynchronize(e1));
  float ms = 0.f;
  KB_CHECK(hipEventElapsedTime(&ms, e0, e1));
  return ms;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc < 7) {
    std::fprintf(stderr, "usage: kbench f32 L CIN COUT NB RES | kbench bf16 L CIN COUT NB TAPS OUT\n");
    return 2;
  }
  const bool f32 = !std::strcmp(argv[1], "f32");
  const int L = std::atoi(argv[2]), cin = std::atoi(argv[3]), cout = std::atoi(argv[4]), nb = std::atoi(argv[5]);
  const int opt = std::atoi(argv[6]);
  const int taps = f32 ? 9 : opt;
  const int out_mode = (!f32 && argc > 7) ? std::atoi(argv[7]) : 0;
  if (L < 3 || L > 6 || cin < 32 || cout < 128 || nb < 1 || (taps != 9 && taps != 1) || out_mode < 0 || out_mode > 2) {
    std::fprintf(stderr, "kbench: shape out of range\n");
    return 2;
  }
  const size_t M = (size_t)nb << (2 * L);
  std::mt19937 rng(1);
  std::normal_distribution<float> nd(0.f, 1.f);
  copy_reference();
  double bytes = 0;
  float ms = 0.f;
  try {
    if (f32) {
      std::vector<float> x(M * cin), w((size_t)9 * cin * cout), b(cout);
      for (auto& v : x) v = nd(rng);
      for (auto& v : w) v = nd(rng) / std::sqrt(9.f * cin);
      for (auto& v : b) v = 0.1f * nd(rng);
      float* dx = upload(x);
      float* dw = upload(w);
      float* db = upload(b);
      float *dr = nullptr, *dout = nullptr;
      KB_CHECK(hipMalloc(&dout, M * cout * sizeof(float)));
      if (opt) {
        KB_CHECK(hipMalloc(&dr, M * cout * sizeof(float)));
        KB_CHECK(hipMemset(dr, 0, M * cout * sizeof(float)));
      }
      ConvArgs a{};
      a.src0 = dx;
      a.c0 = cin;
      a.nb = nb;
      a.lh = L;
      a.lw = L;
      a.cout = cout;
      a.taps = 9;
      a.wt = dw;
      a.bias = db;
      a.res = dr;
      a.out = dout;
      ms = time_once([&] { launch_conv(nullptr, a); });
      bytes = 4.0 * M * cin + 4.0 * 9 * cin * cout + 4.0 * M * cout * (opt ? 2 : 1);
    } else {
      std::vector<uint16_t> x(M * cin), wf((size_t)taps * cin * cout), wl((size_t)cout * conv_lp_kp(taps, cin), 0);
      std::vector<float> b(cout);
      for (auto& v : x) v = bf16_bits(nd(rng));
      const int K = taps * cin;
      for (int o = 0; o < cout; ++o)
        for (int k = 0; k < K; ++k) {
          const uint16_t v = bf16_bits(nd(rng) / std::sqrt((float)K));
          wf[conv_lp_frag_index(o, k, K)] = v;
          wl[(size_t)o * conv_lp_kp(taps, cin) + k] = v;
        }
      for (auto& v : b) v = 0.1f * nd(rng);
      uint16_t* dx = upload(x);
      uint16_t* dwf = upload(wf);
      uint16_t* dwl = upload(wl);
      float* db = upload(b);
      ConvLpArgs a{};
      a.act = dx;
      a.cin = cin;
      a.nb = nb;
      a.lh = L;
      a.lw = L;
      a.cout = cout;
      a.taps = taps;
      a.kp = conv_lp_kp(taps, cin);
      a.wt = dwl;
      a.wfrag = dwf;
      a.bias = db;
      if (out_mode == 1) {
        KB_CHECK(hipMalloc(&a.out16, M * cout * sizeof(uint16_t)));
        KB_CHECK(hipMalloc(&a.stats, (size_t)nb * 16 * 32 * 2 * sizeof(double)));
        a.groups = 32;
      } else {
        KB_CHECK(hipMalloc(&a.out, M * cout * sizeof(float)));
      }
      if (out_mode == 2) {
        float* dr = nullptr;
        KB_CHECK(hipMalloc(&dr, M * cout * sizeof(float)));
        KB_CHECK(hipMemset(dr, 0, M * cout * sizeof(float)));
        a.res = dr;
      }
      ms = time_once([&] { launch_conv_lp(nullptr, a); });
      bytes = 2.0 * M * cin + 2.0 * K * cout + (out_mode == 1 ? 2.0 : 4.0) * M * cout + (out_mode == 2 ? 4.0 * M * cout : 0.0);
    }
  } catch (const Error& e) {
    std::fprintf(stderr, "kbench: %s\n", e.msg.c_str());
    return 1;
  }
  const double flops = 2.0 * M * cout * (double)taps * cin;
  std::printf("kbench %s L=%d cin=%d cout=%d nb=%d taps=%d opt=%d: %.3f ms, %.1f TFLOP/s, algorithmic %.3e B (%.0f GB/s)\n",
              argv[1], L, cin, cout, nb, taps, f32 ? opt : out_mode, ms, flops / ms / 1e9, bytes, bytes / ms / 1e6);
  return 0;
}
