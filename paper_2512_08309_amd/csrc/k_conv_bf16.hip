// Reduced-precision implicit-GEMM convolution: BF16 operands on CDNA4
// matrix cores (v_mfma_f32_16x16x32_bf16), FP32 accumulation, FP32 output
// with bias and residual added in FP32.
//
// Operands are prepared outside: activations by the GroupNorm-apply kernel
// (NHWC BF16, the virtual concat / upsample / GN / SiLU already applied),
// weights at load time as [C_out][Kp] BF16 with K = tap * C_in + c_in
// flattened and zero-padded to a multiple of the stage depth.  With no
// per-element transform left, staging is plain 16-byte copies: one
// (pixel, 8-channel) segment per load.
//
// Tile 128 x 128 per 256-thread workgroup (4 waves, 2 x 2, 64 x 64 each),
// K advances BK = 32 per stage through double-buffered LDS (32 KB, so four
// workgroups share a CU).  LDS rows hold BK BF16 values of one pixel (A) or
// one output channel (B); the 16-byte segments of a row are XOR-swizzled by
// the row index so that the MFMA operand reads (16 consecutive rows, same
// segment) are bank-conflict free.
// A K-group g of an MFMA lane pairs the same 8 K indices for A and B, so
// the product is the plain dot product whatever order the hardware sums
// the 32 terms in; that order is fixed, keeping results batch-invariant.
//
// Weights may instead be OCP FP8 e4m3 with a per-output-channel FP32 scale
// (applied in the epilogue); they are widened to BF16 while staging, which
// is exact.
//
// FAST (C_in a multiple of BK): a stage never straddles a tap, so the
// shifted pixel address is computed once per tap.  Otherwise every segment
// resolves its own (tap, channel).
#include <type_traits>

#include "td_internal.h"

namespace td {
namespace {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));
typedef unsigned u2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));

// 4 OCP e4m3 bytes -> 4 BF16 (exact: every e4m3 value is a BF16 value).
__device__ __forceinline__ u2v fp8x4_to_bf16x4(unsigned w) {
  f2v lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, false);
  f2v hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, true);
  bf2v a = {(__bf16)lo.x, (__bf16)lo.y}, b = {(__bf16)hi.x, (__bf16)hi.y};
  return (u2v){__builtin_bit_cast(unsigned, a), __builtin_bit_cast(unsigned, b)};
}

// 4 segments of 16 bytes per 64-byte row; rows 2r and 2r+1 share a 128-byte
// bank line, so the swizzle changes every second row.
__device__ __forceinline__ int swz(int row, int seg) { return seg ^ ((row >> 1) & 3); }

template <int TAPS, bool FAST, bool W8, int BN, int WM, int WN>
__global__ __launch_bounds__(256, 4) void conv_bf16_kernel(ConvLpArgs a, int n_tiles_n) {
  constexpr int BM = 128;
  constexpr int BK = 32;
  constexpr int SEGS = BK / 8;             // 16-byte segments per row
  constexpr int AL = BM * SEGS / 256;      // A segment loads per thread
  constexpr int BL = (BN * SEGS + 255) / 256;
  constexpr int KS = BK / 32;              // MFMA k-steps per stage
  constexpr int TM = BM / WM / 16, TN = BN / WN / 16;
  __shared__ __attribute__((aligned(16))) u4v As[2][BM * SEGS];
  __shared__ __attribute__((aligned(16))) u4v Bs[2][BN * SEGS];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int bid = blockIdx.x, nblk = gridDim.x;
  const int tile = ((nblk & 7) == 0) ? (bid & 7) * (nblk >> 3) + (bid >> 3) : bid;
  const int tn = tile % n_tiles_n, tm = tile / n_tiles_n;
  const int m0 = tm * BM, n0 = tn * BN;
  const int lw = a.lw, lh = a.lh, W = 1 << lw, H = 1 << lh, lhw = lw + lh;
  const int M = a.nb << lhw;
  const int cin = a.cin, Kp = a.kp, K = TAPS * cin;
  const __bf16* act = reinterpret_cast<const __bf16*>(a.act);
  const __bf16* wts = reinterpret_cast<const __bf16*>(a.wt);
  const unsigned char* wts8 = reinterpret_cast<const unsigned char*>(a.wt);

  // Staging map: consecutive lanes take consecutive 16-byte segments of one
  // LDS row, so a wave's load instruction reads SEGS-lane runs of contiguous
  // bytes (64-byte row halves of a 128-byte line) instead of one segment from 64
  // different lines.  Thread tid owns segment sg of rows r0 + RSTEP * j.
  constexpr int RSTEP = 256 / SEGS;
  const int sg = tid % SEGS, r0 = tid / SEGS;
  int mpix[AL];
  bool mval[AL];
#pragma unroll
  for (int j = 0; j < AL; ++j) {
    const int m = m0 + r0 + RSTEP * j;
    mval[j] = m < M;
    mpix[j] = mval[j] ? m : 0;
  }

  u4v ra[AL];
  typedef typename std::conditional<W8, u2v, u4v>::type wreg;
  wreg rb[BL];
  const u4v zero = {0u, 0u, 0u, 0u};
  const __bf16* pix[AL];   // shifted pixel + segment base (FAST)
  bool pok[AL];
  auto set_tap = [&](int tap) {
    int dy = 0, dx = 0;
    if (TAPS == 9) { dy = tap / 3 - 1; dx = tap % 3 - 1; }
#pragma unroll
    for (int j = 0; j < AL; ++j) {
      const int yy = ((mpix[j] >> lw) & (H - 1)) + dy, xx = (mpix[j] & (W - 1)) + dx;
      pok[j] = mval[j] && yy >= 0 && yy < H && xx >= 0 && xx < W;
      const int p = pok[j] ? mpix[j] + dy * W + dx : 0;
      pix[j] = act + ((size_t)p * cin + 8 * sg);
    }
  };
  auto load_stage = [&](int k0, int ci0) {
#pragma unroll
    for (int j = 0; j < AL; ++j) {
      if (FAST) {
        u4v v = *reinterpret_cast<const u4v*>(pix[j] + ci0);
        ra[j] = pok[j] ? v : zero;
      } else {
        const int k = k0 + 8 * sg;
        const int t = k / cin, ci = k - t * cin;
        int dy = 0, dx = 0;
        if (TAPS == 9) { dy = t / 3 - 1; dx = t % 3 - 1; }
        const int yy = ((mpix[j] >> lw) & (H - 1)) + dy, xx = (mpix[j] & (W - 1)) + dx;
        const bool ok = mval[j] && k < K && yy >= 0 && yy < H && xx >= 0 && xx < W;
        const int p = ok ? mpix[j] + dy * W + dx : 0;
        u4v v = *reinterpret_cast<const u4v*>(act + ((size_t)p * cin + (ok ? ci : 0)));
        ra[j] = ok ? v : zero;
      }
    }
#pragma unroll
    for (int j = 0; j < BL; ++j) {
      const int e = tid + 256 * j;
      if (e < BN * SEGS) {
        const int n = e / SEGS;
        if (W8) rb[j] = *reinterpret_cast<const wreg*>(wts8 + (size_t)(n0 + n) * Kp + k0 + 8 * sg);
        else rb[j] = *reinterpret_cast<const wreg*>(wts + (size_t)(n0 + n) * Kp + k0 + 8 * sg);
      }
    }
  };
  auto store_stage = [&](int buf) {
#pragma unroll
    for (int j = 0; j < AL; ++j) {
      const int row = r0 + RSTEP * j;
      As[buf][row * SEGS + swz(row, sg)] = ra[j];
    }
#pragma unroll
    for (int j = 0; j < BL; ++j) {
      const int e = tid + 256 * j;
      if (e < BN * SEGS) {
        const int n = e / SEGS;
        if constexpr (W8) {
          u2v lo = fp8x4_to_bf16x4(rb[j].x), hi = fp8x4_to_bf16x4(rb[j].y);
          Bs[buf][n * SEGS + swz(n, sg)] = (u4v){lo.x, lo.y, hi.x, hi.y};
        } else {
          Bs[buf][n * SEGS + swz(n, sg)] = rb[j];
        }
      }
    }
  };

  f4v acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = (f4v){0.f, 0.f, 0.f, 0.f};

  const int nst = Kp / BK;
  int tap = 0, ci = 0;
  if (FAST) set_tap(0);
  load_stage(0, 0);
  store_stage(0);
  __syncthreads();

  const int g = lane >> 4, r16 = lane & 15;
  for (int st = 0; st < nst; ++st) {
    const int buf = st & 1;
    const bool more = st + 1 < nst;
    if (more) {
      if (FAST) {
        ci += BK;
        if (ci == cin) {
          ci = 0;
          ++tap;
          set_tap(tap);
        }
      }
      load_stage((st + 1) * BK, ci);
    }
    bf8v av[KS][TM], bv[KS][TN];
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      const int seg = 4 * kk + g;
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int row = wm * (BM / WM) + 16 * i + r16;
        u4v u = As[buf][row * SEGS + swz(row, seg)];
        av[kk][i] = __builtin_bit_cast(bf8v, u);
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int col = wn * (BN / WN) + 16 * j + r16;
        u4v w = Bs[buf][col * SEGS + swz(col, seg)];
        bv[kk][j] = __builtin_bit_cast(bf8v, w);
      }
    }
#pragma unroll
    for (int kk = 0; kk < KS; ++kk)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[kk][i], bv[kk][j], acc[i][j], 0, 0, 0);
    if (more) store_stage(buf ^ 1);
    __syncthreads();
  }

  // Epilogue: tile (i, j), lane holds rows 4g+v, column r16.
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int n = n0 + wn * (BN / WN) + 16 * j + r16;
    const float bias = a.bias ? a.bias[n] : 0.f;
    const float scl = a.wscale ? a.wscale[n] : 1.f;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm * (BM / WM) + 16 * i + 4 * g + v;
        if (m >= M) continue;
        const size_t off = (size_t)m * a.cout + n;
        float o = acc[i][j][v] * scl + bias;
        if (a.res) o += a.res[off];
        a.out[off] = o;
      }
  }
}

template <bool W8, int BN, int WM, int WN>
void launch_lp_cfg(hipStream_t st, const ConvLpArgs& a, bool fast) {
  const int M = a.nb << (a.lh + a.lw);
  const int mt = (M + 127) / 128, nt = a.cout / BN;
  if (a.taps == 9 && fast)
    hipLaunchKernelGGL((conv_bf16_kernel<9, true, W8, BN, WM, WN>), dim3(mt * nt), dim3(256), 0, st, a, nt);
  else if (a.taps == 9)
    hipLaunchKernelGGL((conv_bf16_kernel<9, false, W8, BN, WM, WN>), dim3(mt * nt), dim3(256), 0, st, a, nt);
  else if (fast)
    hipLaunchKernelGGL((conv_bf16_kernel<1, true, W8, BN, WM, WN>), dim3(mt * nt), dim3(256), 0, st, a, nt);
  else
    hipLaunchKernelGGL((conv_bf16_kernel<1, false, W8, BN, WM, WN>), dim3(mt * nt), dim3(256), 0, st, a, nt);
  TD_LAUNCHED();
}

template <int BN, int WM, int WN>
void launch_lp_w(hipStream_t st, const ConvLpArgs& a, bool fast) {
  if (a.w8) launch_lp_cfg<true, BN, WM, WN>(st, a, fast);
  else launch_lp_cfg<false, BN, WM, WN>(st, a, fast);
}

}  // namespace

void launch_conv_lp(hipStream_t st, const ConvLpArgs& a) {
  TD_CHECK(a.cin % 8 == 0 && a.cout % 16 == 0 && a.cout > 0, -5,
           "bf16 conv: needs C_in % 8 == 0 and C_out % 16 == 0");
  TD_CHECK(a.taps == 9 || a.taps == 1, -5, "bf16 conv: taps must be 9 or 1");
  if (!a.nb) return;
  const bool fast = a.cin % 32 == 0;
  const int BK = 32;
  TD_CHECK(a.kp % BK == 0 && a.kp >= a.taps * a.cin, -5, "bf16 conv: bad padded K");
  const double Md = (double)(a.nb << (a.lh + a.lw));
  prof_begin(st);
  TD_CHECK(!a.w8 || a.wscale, -5, "fp8 weights need per-channel scales");
  if (a.cout % 128 == 0) launch_lp_w<128, 2, 2>(st, a, fast);
  else if (a.cout % 64 == 0) launch_lp_w<64, 2, 2>(st, a, fast);
  else if (a.cout % 32 == 0) launch_lp_w<32, 4, 1>(st, a, fast);
  else launch_lp_w<16, 4, 1>(st, a, fast);
  prof_end(st, a.taps == 9 ? K_CONV3_LP : K_CONV1_LP, 2.0 * Md * a.cout * a.taps * a.cin,
           2.0 * Md * a.cin + 2.0 * a.kp * a.cout + 4.0 * Md * a.cout * (a.res ? 2 : 1));
}

}  // namespace td
