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
//
// 3x3 convolutions with FAST shapes and BF16 weights use a second kernel
// that copies the segments straight from global memory into a three-stage
// LDS ring (global_load_lds_dwordx4), two stages ahead of the MFMAs; see
// conv_bf16_dl_kernel.
#include <type_traits>
#include <utility>

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
  bool pok[AL];            // the loaded segment is inside the image (FAST)
  bool lok[AL];            // the same for the general path
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
      // out-of-image segments load a valid pixel and are zeroed when
      // stored to LDS, after the MFMAs, so no wait for the load sits here
      if (FAST) {
        ra[j] = *reinterpret_cast<const u4v*>(pix[j] + ci0);
      } else {
        const int k = k0 + 8 * sg;
        const int t = k / cin, ci = k - t * cin;
        int dy = 0, dx = 0;
        if (TAPS == 9) { dy = t / 3 - 1; dx = t % 3 - 1; }
        const int yy = ((mpix[j] >> lw) & (H - 1)) + dy, xx = (mpix[j] & (W - 1)) + dx;
        const bool ok = mval[j] && k < K && yy >= 0 && yy < H && xx >= 0 && xx < W;
        const int p = ok ? mpix[j] + dy * W + dx : 0;
        lok[j] = ok;
        ra[j] = *reinterpret_cast<const u4v*>(act + ((size_t)p * cin + (ok ? ci : 0)));
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
      As[buf][row * SEGS + swz(row, sg)] = (FAST ? pok[j] : lok[j]) ? ra[j] : zero;
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
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      const int seg = 4 * kk + g;
      bf8v bv[TN];
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int col = wn * (BN / WN) + 16 * j + r16;
        bv[j] = __builtin_bit_cast(bf8v, Bs[buf][col * SEGS + swz(col, seg)]);
      }
      // A tile i + 1 is read while the MFMAs of tile i run
      auto a_tile = [&](int i) {
        const int row = wm * (BM / WM) + 16 * i + r16;
        return __builtin_bit_cast(bf8v, As[buf][row * SEGS + swz(row, seg)]);
      };
      bf8v ac = a_tile(0);
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        bf8v an = ac;
        if (i + 1 < TM) an = a_tile(i + 1);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ac, bv[j], acc[i][j], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
        ac = an;
      }
    }
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

// 16 zero bytes: the source of the direct loads of out-of-image segments.
__device__ __attribute__((aligned(16))) u4v g_zero16[1];

// Wait until at most N vector-memory operations of this wave are
// outstanding, then barrier; the clobber keeps the compiler from moving LDS
// accesses across it.
template <int N>
__device__ __forceinline__ void wait_vm_barrier() {
  asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" ::"n"(N) : "memory");
}

// The value, held in scalar registers from here on (not re-derived from
// memory inside a loop whose asm statements clobber memory).
__device__ __forceinline__ const u4v* in_sgprs(const u4v* p) {
  asm volatile("" : "+s"(p));
  return p;
}

// 16 bytes per lane from global memory straight into LDS: lane L writes
// bytes [16 L, 16 L + 16) after the wave-uniform LDS address dst.
__device__ __forceinline__ void copy16_to_lds(const void* src, void* dst) {
  __builtin_amdgcn_global_load_lds(src, dst, 16, 0, 0);
}

// LDS byte address of a __shared__ object.
__device__ __forceinline__ uint32_t lds_addr(const void* p) {
  return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) char*)p;
}

// The operand reads of the direct-load kernel are issued as plain
// ds_read_b128 so that the compiler does not guard them with a wait for
// every outstanding direct load (which would serialise the ring); their
// completion is awaited explicitly with lgkm_wait, whose register operands
// make each MFMA depend on the wait that covers its inputs.
__device__ __forceinline__ u4v ds_read16(uint32_t addr) {
  u4v v;
  asm volatile("ds_read_b128 %0, %1" : "=v"(v) : "v"(addr));
  return v;
}
template <int N>
__device__ __forceinline__ void lgkm_wait(u4v& a, u4v& b0, u4v& b1, u4v& b2, u4v& b3) {
  asm volatile("s_waitcnt lgkmcnt(%5)" : "+v"(a), "+v"(b0), "+v"(b1), "+v"(b2), "+v"(b3) : "n"(N));
}

// Direct-to-LDS variant (C_in a multiple of BK, BF16 weights, BN >= 64):
// every 16-byte segment goes from global memory straight into LDS
// (global_load_lds_dwordx4; no staging registers), through a ring of NS
// stages with loads issued NS - 1 stages ahead.  A wave's load instruction
// fills 1 KB of LDS contiguously (lane L at byte 16 L), so the XOR swizzle
// is applied on the global side: lane L copies the segment that the reader
// expects at LDS slot L.  Out-of-image pixels copy 16 zero bytes.  The
// MFMA sequence per accumulator is that of conv_bf16_kernel.
template <int TAPS, int BM, int BN, int WM, int WN, int MINB>
__global__ __launch_bounds__(256, MINB) void conv_bf16_dl_kernel(ConvLpArgs a, int n_tiles_n) {
  constexpr int BK = 32, SEGS = BK / 8, NS = 3;
  constexpr int AL = BM * SEGS / 256;      // A segment loads per thread per stage
  constexpr int BL = BN * SEGS / 256;      // B segment loads per thread per stage
  static_assert(BN * SEGS % 256 == 0, "every wave loads the same number of B segments");
  static_assert(BN / WN / 16 <= 4, "at most four B tiles per wave");
  constexpr int TM = BM / WM / 16, TN = BN / WN / 16;
  __shared__ __attribute__((aligned(16))) u4v As[NS][BM * SEGS];
  __shared__ __attribute__((aligned(16))) u4v Bs[NS][BN * SEGS];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int bid = blockIdx.x, nblk = gridDim.x;
  const int tile = ((nblk & 7) == 0) ? (bid & 7) * (nblk >> 3) + (bid >> 3) : bid;
  const int tn = tile % n_tiles_n, tm = tile / n_tiles_n;
  const int m0 = tm * BM, n0 = tn * BN;
  const int lw = a.lw, lh = a.lh, W = 1 << lw, H = 1 << lh, lhw = lw + lh;
  const int M = a.nb << lhw;
  const int cin = a.cin, Kp = a.kp;
  const __bf16* act = reinterpret_cast<const __bf16*>(a.act);
  const __bf16* wts = reinterpret_cast<const __bf16*>(a.wt);

  // Lane L of wave w fills LDS slot L of 1 KB chunk (w + 4 j): row
  // r0 + 64 j, position sg; it copies global segment seg of that row.
  const int sg = tid % SEGS, r0 = tid / SEGS;
  const int seg = swz(r0, sg);             // (row >> 1) & 3 is the same for every j
  int mpix[AL];
  bool mval[AL];
#pragma unroll
  for (int j = 0; j < AL; ++j) {
    const int m = m0 + r0 + 64 * j;
    mval[j] = m < M;
    mpix[j] = mval[j] ? m : 0;
  }
  const __bf16* pix[AL];
  bool pok[AL];
  auto set_tap = [&](int tap) {
    int dy = 0, dx = 0;
    if (TAPS == 9) { dy = tap / 3 - 1; dx = tap % 3 - 1; }
#pragma unroll
    for (int j = 0; j < AL; ++j) {
      const int yy = ((mpix[j] >> lw) & (H - 1)) + dy, xx = (mpix[j] & (W - 1)) + dx;
      pok[j] = mval[j] && yy >= 0 && yy < H && xx >= 0 && xx < W;
      const int p = pok[j] ? mpix[j] + dy * W + dx : 0;
      pix[j] = act + ((size_t)p * cin + 8 * seg);
    }
  };
  const __bf16* wrow[BL];
#pragma unroll
  for (int j = 0; j < BL; ++j) wrow[j] = wts + ((size_t)(n0 + r0 + 64 * j) * Kp + 8 * seg);
  const u4v* zero = in_sgprs(g_zero16);
  auto issue = [&](int slot, int k0, int ci0) {
#pragma unroll
    for (int j = 0; j < AL; ++j) {
      const void* src = pok[j] ? (const void*)(pix[j] + ci0) : (const void*)zero;
      copy16_to_lds(src, &As[slot][(16 * wave + 64 * j) * SEGS]);
    }
#pragma unroll
    for (int j = 0; j < BL; ++j)
      copy16_to_lds(wrow[j] + k0, &Bs[slot][(16 * wave + 64 * j) * SEGS]);
  };

  f4v acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = (f4v){0.f, 0.f, 0.f, 0.f};

  const int nst = Kp / BK;
  // (tap, ci) of the next stage to issue
  int tap = 0, ci = 0;
  auto advance = [&]() {
    ci += BK;
    if (ci == cin) {
      ci = 0;
      ++tap;
      if (tap < TAPS) set_tap(tap);
    }
  };
  set_tap(0);
#pragma unroll
  for (int s = 0; s < NS - 1; ++s)
    if (s < nst) {
      issue(s, s * BK, ci);
      advance();
    }

  const int g = lane >> 4, r16 = lane & 15;
  const uint32_t a_base = lds_addr(&As[0][0]), b_base = lds_addr(&Bs[0][0]);
  uint32_t a_off[TM], b_off[4];
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    const int row = wm * (BM / WM) + 16 * i + r16;
    a_off[i] = (row * SEGS + swz(row, g)) * 16;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int col = wn * (BN / WN) + 16 * (j < TN ? j : 0) + r16;
    b_off[j] = (col * SEGS + swz(col, g)) * 16;
  }
  for (int st = 0; st < nst; ++st) {
    // stage st has landed once only the loads of the NS - 2 later stages
    // may still be outstanding; the barrier also ends every wave's reads of
    // the slot the next issue overwrites
    if (st + NS - 2 < nst) wait_vm_barrier<(NS - 2) * (AL + BL)>();
    else wait_vm_barrier<0>();
    if (st + NS - 1 < nst) {
      issue((st + NS - 1) % NS, (st + NS - 1) * BK, ci);
      advance();
    }
    const int buf = st % NS;
    const uint32_t ab = a_base + buf * (BM * SEGS * 16), bb = b_base + buf * (BN * SEGS * 16);
    u4v bv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) bv[j] = (j < TN) ? ds_read16(bb + b_off[j]) : (u4v){0u, 0u, 0u, 0u};
    u4v ac = ds_read16(ab + a_off[0]);
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      u4v an = ac;
      if (i + 1 < TM) {
        an = ds_read16(ab + a_off[i + 1]);
        lgkm_wait<1>(ac, bv[0], bv[1], bv[2], bv[3]);
      } else {
        lgkm_wait<0>(ac, bv[0], bv[1], bv[2], bv[3]);
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int j = 0; j < TN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8v, ac),
                                                            __builtin_bit_cast(bf8v, bv[j]), acc[i][j], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
      ac = an;
    }
  }

#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int n = n0 + wn * (BN / WN) + 16 * j + r16;
    const float bias = a.bias ? a.bias[n] : 0.f;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm * (BM / WM) + 16 * i + 4 * g + v;
        if (m >= M) continue;
        const size_t off = (size_t)m * a.cout + n;
        float o = acc[i][j][v] + bias;
        if (a.res) o += a.res[off];
        a.out[off] = o;
      }
  }
}


template <int N>
__device__ __forceinline__ void lgkm_wait4(u4v& a0, u4v& a1, u4v& a2, u4v& a3) {
  asm volatile("s_waitcnt lgkmcnt(%4)" : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3) : "n"(N));
}

typedef float f16v __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------------------
// Halo-staged 3x3 convolution (square images of side 8..64, C_in % 32 == 0,
// C_out % 128 == 0, BF16 weights) on v_mfma_f32_32x32x16_bf16; the same
// kernel with TAPS = 1 and no halo border runs the 1x1 convolutions.
//
// A workgroup computes 256 output pixels (whole rows of one image, or
// whole 8x8 images) x 128 output channels.  For each 32-channel input chunk
// stages the tile's halo -- its rows plus one above and below, its columns
// plus the zero columns on either side -- into LDS once (loaded into
// registers at the start of the previous chunk, written at its end), and
// the nine taps read their A operands from that patch at shifted pixel
// positions: each input element is staged once per chunk instead of once
// per tap.
//
// The B operands (weights) do not go through LDS: they are stored at load
// time in MFMA fragment order (conv_lp_frag_index) and loaded straight into
// registers P K-steps ahead of their use.
//
// Four waves (2 x 2), each 128 pixels x 64 channels: 4 x 2 tiles of 32 x 32,
// 8 MFMAs per 16-value K step against 4 LDS operand reads.  K runs chunk by
// chunk, tap by tap within a chunk, in a fixed order: results do not depend
// on the batch.
//
// LDS patch layout: halo pixel q holds its 32 chunk channels in 64 bytes at
// byte 80 q (16 bytes of padding per pixel).  Eight consecutive pixels --
// the lanes one LDS cycle serves -- then start at distinct 16-byte positions
// of the 128-byte bank line, so operand reads are conflict free, and a tap
// moves every lane's address by the same constant (an instruction offset).
template <int L, int TAPS>
struct HaloGeom {
  static constexpr int W = 1 << L;
  static constexpr int HW = W * W;
  static constexpr int NI = HW >= 256 ? 1 : 256 / HW;        // images per tile
  static constexpr int ROWS = HW >= 256 ? 256 / W : W;        // output rows per image
  static constexpr int BORDER = TAPS == 9 ? 1 : 0;            // halo pixels on each side
  static constexpr int QW = W + 2 * BORDER, RH = ROWS + 2 * BORDER;   // halo width and rows
  static constexpr int NQ = NI * RH * QW;                     // halo pixels
  static constexpr int NINS = (5 * NQ + 63) / 64;             // 1 KB copies per chunk
  static constexpr int NPL = (NINS + 3) / 4;                  // copies per wave
};

// 16 bytes of LDS read at a register address plus a constant offset (see
// ds_read16 for why this is asm).
template <int OFF>
__device__ __forceinline__ u4v ds_read16_off(uint32_t addr) {
  u4v v;
  asm volatile("ds_read_b128 %0, %1 offset:%2" : "=v"(v) : "v"(addr), "n"(OFF));
  return v;
}

// LDS writes done and every wave arrived, without waiting for outstanding
// global loads (the weight prefetches).
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// f(std::integral_constant<int, r>) for r = 0 .. N-1, in order.
template <class F, int... R>
__device__ __forceinline__ void unroll_seq(F& f, std::integer_sequence<int, R...>) {
  (f(std::integral_constant<int, R>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void unroll(F& f) {
  unroll_seq(f, std::make_integer_sequence<int, N>{});
}

// SKIP (TAPS = 9): after the 3x3 chunks over act, 1x1 chunks over act2
// (cin2 channels) run on the centre tap of the same patch layout; their
// weights follow the 3x3 ones in K.
// ACT (TAPS = 9, one source, one window per tile): the input is staged as
// SiLU(x * scale + shift) with the window's per-channel GroupNorm affine.
// Measured against a separate apply pass plus the plain kernel (outputs
// bit-identical): faster for windows of side 32 and 64 (-8%, -11%), slower
// at 16 (+13%); with SKIP the kernel spills registers (3x slower), so the
// launcher takes it for sides 32 and 64 without SKIP only.
template <int L, int P, int TAPS, bool SKIP, bool ACT>
__global__ __launch_bounds__(256, 2) void conv_bf16_halo_kernel(ConvLpArgs a, int n_tiles_n) {
  using G = HaloGeom<L, TAPS>;
  constexpr int STEPS = 2 * TAPS;                  // 16-value K steps per 32-channel chunk
  constexpr int W = G::W, QW = G::QW, RH = G::RH;
  constexpr int TM = 4, TN = 2;                    // 32 x 32 tiles per wave
  constexpr int SLOTS = G::NPL * 256;              // 16-byte slots per patch buffer
  static_assert(STEPS % P == 0, "the B ring must divide the K steps of a chunk");
  // two patch buffers; after the main loop the same LDS holds the BF16
  // output tile (256 rows of TROW bytes) and the GroupNorm exchange
  constexpr int TROW = 272;                        // 256 bytes + 16: rows 4 apart fall on other banks
  constexpr int TILE_BYTES = 256 * TROW, RED_BYTES = 2 * 2 * 32 * 2 * 8;
  constexpr int LDS_SLOTS = (2 * SLOTS > (TILE_BYTES + RED_BYTES) / 16) ? 2 * SLOTS : (TILE_BYTES + RED_BYTES) / 16;
  __shared__ __attribute__((aligned(16))) u4v lds[LDS_SLOTS];
  static_assert(!ACT || (TAPS == 9 && !SKIP && (1 << (2 * L)) >= 256),
                "the staged activation: 3x3, one source, one window per tile");
  __shared__ __attribute__((aligned(16))) float2 actss[ACT ? kActMaxCin : 1];   // (scale, shift) per channel

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int bid = blockIdx.x, nblk = gridDim.x;
  const int tile = ((nblk & 7) == 0) ? (bid & 7) * (nblk >> 3) + (bid >> 3) : bid;
  const int tn = tile % n_tiles_n, tm = tile / n_tiles_n;
  const int m0 = tm * 256, n0 = tn * 128;
  const int M = a.nb << (2 * L);
  const int cin = a.cin;
  const int cin2 = SKIP ? a.cin2 : 0;
  const int KB = (TAPS * cin + cin2) / 16;         // 16-value K blocks
  const u4v* act = reinterpret_cast<const u4v*>(a.act);
  const u4v* wf = reinterpret_cast<const u4v*>(a.wfrag);

  // ---- halo slots owned by this thread: slot 64 (wave + 4 j) + lane, which
  // is segment slot % 5 of halo pixel slot / 5 (segment 4 is padding; slots
  // past the halo are loaded and stored too, as zeros, so that every wave
  // issues the same loads with no branches around them).
  // hpack: 8 x its pixel index + its segment, or ~0 for zeros.
  const int b0 = m0 >> (2 * L);                    // first image of the tile
  const int row0 = (G::NI == 1) ? ((m0 >> L) & (W - 1)) : 0;
  uint32_t hpack[G::NPL];
#pragma unroll
  for (int j = 0; j < G::NPL; ++j) {
    const int ins = wave + 4 * j;
    const int slot = 64 * ins + lane;
    const int q = slot / 5, seg = slot - 5 * q;
    const int img = q / (RH * QW), rem = q - img * (RH * QW);
    const int hy = rem / QW, hx = rem - hy * QW;
    const int y = row0 + hy - G::BORDER, x = hx - G::BORDER, b = b0 + img;
    const bool ok = ins < G::NINS && seg < 4 && q < G::NQ && b < a.nb && y >= 0 && y < W && x >= 0 && x < W;
    hpack[j] = ok ? (uint32_t)((((b * W + y) * W + x) << 3) + seg) : ~0u;
  }
  u4v hreg[G::NPL];
  typedef const __attribute__((address_space(1))) u4v gu4v;
  gu4v* gzero = (gu4v*)in_sgprs(g_zero16);
  const int nch_a = cin / 32, nch = nch_a + cin2 / 32;   // 3x3 (or 1x1) chunks, all chunks
  // the patch of chunk g (past the last: the last again, unused, so that no
  // branch surrounds the loads)
  auto load_halo = [&](int g) {
    g = g < nch ? g : nch - 1;
    const bool second = SKIP && g >= nch_a;
    gu4v* src = (gu4v*)(second ? reinterpret_cast<const u4v*>(a.act2) : act);
    const int q8 = second ? cin2 / 8 : cin / 8;
    const int c8 = 4 * (second ? g - nch_a : g);
#pragma unroll
    for (int j = 0; j < G::NPL; ++j)
      hreg[j] = *(hpack[j] != ~0u ? src + ((size_t)(hpack[j] >> 3) * q8 + (hpack[j] & 7) + c8) : gzero);
  };
  // the patch of chunk g into buffer buf (with ACT, first-source chunks are
  // activated: in-image values only, the zero slots stay zero)
  auto store_halo = [&](int buf, int g) {
#pragma unroll
    for (int j = 0; j < G::NPL; ++j) {
      if constexpr (ACT) {
        if (g < nch_a && hpack[j] != ~0u) {
          const float4* ss = reinterpret_cast<const float4*>(&actss[32 * g + 8 * (hpack[j] & 7)]);
          const uint32_t w[4] = {hreg[j][0], hreg[j][1], hreg[j][2], hreg[j][3]};
          uint32_t o[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const float4 p = ss[k];                      // (scale, shift) of channels 2k, 2k + 1
            float v0 = __uint_as_float(w[k] << 16), v1 = __uint_as_float(w[k] & 0xffff0000u);
            v0 = v0 * p.x + p.y;
            v1 = v1 * p.z + p.w;
            v0 = v0 * __builtin_amdgcn_rcpf(1.0f + __expf(-v0));
            v1 = v1 * __builtin_amdgcn_rcpf(1.0f + __expf(-v1));
            typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
            const bf2 pk = {(__bf16)v0, (__bf16)v1};
            o[k] = __builtin_bit_cast(uint32_t, pk);
          }
          hreg[j] = u4v{o[0], o[1], o[2], o[3]};
        }
      }
      lds[buf * SLOTS + 64 * (wave + 4 * j) + lane] = hreg[j];
    }
  };

  // ---- A operands: tile i of this wave, lane pixel (lane & 31); the base
  // is the up-left neighbour's byte address plus the lane's K group
  uint32_t abase[TM];
  const uint32_t pbase = lds_addr(&lds[0]);
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    const int pl = wm * 128 + 32 * i + (lane & 31);
    const int img = pl >> (2 * L), y = (pl >> L) & (W - 1), x = pl & (W - 1);
    abase[i] = pbase + 80 * ((img * RH + y) * QW + x) + 16 * (lane >> 5);
  }

  // ---- B fragments: block n32 = n0 / 32 + 2 wn + j, K block kb
  const u4v* wrow[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) wrow[j] = wf + ((size_t)((n0 >> 5) + 2 * wn + j) * KB) * 64 + lane;
  const int NA = nch_a * STEPS;                    // K steps of the first source
  const int NS = NA + 2 * (nch - nch_a);
  u4v bq[P][TN];
  auto issue_b = [&](int slot, int step) {
    // steps past the last one load block 0, unused
    int kb = 0;
    if (step < NA) {
      const int ch = step / STEPS, r = step - STEPS * ch;
      kb = ((r >> 1) * cin + 32 * ch) / 16 + (r & 1);
    } else if (step < NS) {
      kb = (TAPS * cin) / 16 + (step - NA);
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) bq[slot][j] = wrow[j][(size_t)kb * 64];
  };

  f16v acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

  load_halo(0);
  if constexpr (ACT) {
    for (int c = tid; c < cin; c += 256)
      actss[c] = make_float2(a.act_scale[(size_t)b0 * cin + c], a.act_shift[(size_t)b0 * cin + c]);
    __syncthreads();
  }
  store_halo(0, 0);
#pragma unroll
  for (int s = 0; s < P; ++s) issue_b(s, s);
  __syncthreads();

  // one chunk: NSTEP K steps over patch buffer g & 1, the first at global
  // step step0; CENTER: the 1x1 chunks of the second source (centre tap)
  auto chunk = [&](auto nstep_c, auto center_c, int g, int step0) {
    constexpr int NSTEP = decltype(nstep_c)::value;
    constexpr bool CENTER = decltype(center_c)::value;
    const int buf = g & 1;
    load_halo(g + 1);
    const uint32_t boff = buf * (SLOTS * 16);
    uint32_t ab[TM];
#pragma unroll
    for (int i = 0; i < TM; ++i) ab[i] = abase[i] + boff;
    // the A operands of step r + 1 are read while the MFMAs of step r run
    auto read_a = [&](auto rc, u4v* av) {
      constexpr int r = decltype(rc)::value;
      constexpr int tap = CENTER ? 4 : r >> 1, half = r & 1;
      constexpr int OFF = 80 * ((tap / 3) * QW + tap % 3) + 32 * half;
#pragma unroll
      for (int i = 0; i < TM; ++i) av[i] = ds_read16_off<OFF>(ab[i]);
    };
    u4v acur[TM], anext[TM];
    read_a(std::integral_constant<int, 0>{}, acur);
    auto step = [&](auto rc) {
      constexpr int r = decltype(rc)::value;
      if constexpr (r + 1 < NSTEP) read_a(std::integral_constant<int, r + 1>{}, anext);
      u4v bv[TN];
#pragma unroll
      for (int j = 0; j < TN; ++j) bv[j] = bq[r % P][j];
      issue_b(r % P, step0 + r + P);
      // LDS reads complete in order: at most the next step's TM are pending
      if constexpr (r + 1 < NSTEP) lgkm_wait4<TM>(acur[0], acur[1], acur[2], acur[3]);
      else lgkm_wait4<0>(acur[0], acur[1], acur[2], acur[3]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8v, acur[i]),
                                                              __builtin_bit_cast(bf8v, bv[j]), acc[i][j], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int i = 0; i < TM; ++i) acur[i] = anext[i];
    };
    unroll<NSTEP>(step);
    // the next chunk's patch goes to the other buffer, which every wave
    // finished reading before the previous barrier
    store_halo(buf ^ 1, g + 1);
    lds_barrier();
  };
  for (int g = 0; g < nch_a; ++g)
    chunk(std::integral_constant<int, STEPS>{}, std::false_type{}, g, STEPS * g);
  if constexpr (SKIP)
    for (int g = nch_a; g < nch; ++g)
      chunk(std::integral_constant<int, 2>{}, std::true_type{}, g, NA + 2 * (g - nch_a));
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // the unused last prefetches

  // ---- epilogue: tile (i, j) register e holds row 8 (e / 4) + 4 (lane / 32)
  // + e % 4, column lane % 32.  The output is stored as FP32 (plus the
  // residual), or as BF16 through an LDS transpose so that each lane writes
  // 16 contiguous bytes.  With a.stats, the GroupNorm sums of the output's
  // FP32 values per (window, tile of the window, group) are formed in a
  // fixed order: over the lane's rows (FP32), then in FP64 with the lane
  // holding the other rows of its column, over the group's columns, and over
  // the tile's two row halves (one window per tile when a window spans whole
  // tiles).
  const int kg = lane >> 5;
  const bool want_stats = a.stats != nullptr;
  char* const otile = reinterpret_cast<char*>(lds);
  float f1[TN][2] = {}, f2[TN][2] = {};
  float biasv[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) biasv[j] = a.bias ? a.bias[n0 + 64 * wn + 32 * j + (lane & 31)] : 0.f;
  if (a.out16) {
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int nl = 64 * wn + 32 * j + (lane & 31);
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int pr = 128 * wm + 32 * i + 8 * (e >> 2) + 4 * kg + (e & 3);
          const float o = acc[i][j][e] + biasv[j];
          *reinterpret_cast<uint16_t*>(otile + pr * TROW + 2 * nl) = __builtin_bit_cast(uint16_t, (__bf16)o);
          const int part = G::NI == 1 ? 0 : (i >> 1);   // 8x8 windows: rows of two windows
          if (m0 + pr < M) {
            f1[j][part] += o;
            f2[j][part] += o * o;
          }
        }
    }
    __syncthreads();
    const int c16 = tid & 15;
#pragma unroll 4
    for (int k = 0; k < 16; ++k) {
      const int pr = (tid >> 4) + 16 * k, m = m0 + pr;
      if (m < M)
        *reinterpret_cast<u4v*>(a.out16 + (size_t)m * a.cout + n0 + 8 * c16) =
            *reinterpret_cast<const u4v*>(otile + pr * TROW + 16 * c16);
    }
  } else {
    // FP32 output, 32 x 32 tile t = (j, i) at a time: one base address per
    // tile, row offsets that are the same for every lane, and a bounds test
    // per tile that is the same for every lane (M is a multiple of 64 and a
    // tile's 32 rows start at a multiple of 32, so they are all below M or
    // all past it).  The residuals of tile t + 1 are loaded before the
    // outputs of tile t are stored: loads and stores retire in order, so a
    // load issued behind stores waits for them, and a per-element load /
    // store sequence pays a memory round trip per element.
    float rb[2][16];
    auto rows_ok = [&](int i) { return __builtin_amdgcn_readfirstlane(m0 + 128 * wm + 32 * i) < M; };
    auto row_ptr = [&](auto* base, int i, int j) {
      return base + (size_t)(m0 + 128 * wm + 32 * i + 4 * kg) * a.cout + n0 + 64 * wn + 32 * j + (lane & 31);
    };
    auto load_res = [&](auto tc) {
      constexpr int t = decltype(tc)::value, j = t / TM, i = t % TM;
      if (a.res && rows_ok(i)) {
        const float* rp = row_ptr(a.res, i, j);
#pragma unroll
        for (int e = 0; e < 16; ++e) rb[t & 1][e] = rp[(8 * (e >> 2) + (e & 3)) * a.cout];
      } else {
#pragma unroll
        for (int e = 0; e < 16; ++e) rb[t & 1][e] = 0.f;
      }
    };
    auto store_tile = [&](auto tc) {
      constexpr int t = decltype(tc)::value, j = t / TM, i = t % TM;
      constexpr int part = G::NI == 1 ? 0 : (i >> 1);
      if (rows_ok(i)) {
        float* op = row_ptr(a.out, i, j);
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const float o = (acc[i][j][e] + biasv[j]) + rb[t & 1][e];
          op[(8 * (e >> 2) + (e & 3)) * a.cout] = o;
          f1[j][part] += o;
          f2[j][part] += o * o;
        }
      }
    };
    load_res(std::integral_constant<int, 0>{});
    auto stage = [&](auto tc) {
      constexpr int t = decltype(tc)::value;
      if constexpr (t + 1 < TM * TN) load_res(std::integral_constant<int, t + 1>{});
      __builtin_amdgcn_sched_barrier(0);
      store_tile(tc);
      __builtin_amdgcn_sched_barrier(0);
    };
    unroll<TM * TN>(stage);
  }
  double s1[TN][2], s2[TN][2];
#pragma unroll
  for (int j = 0; j < TN; ++j)
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      s1[j][p] = f1[j][p];
      s2[j][p] = f2[j][p];
    }
  if (a.chstats) {
    // per-channel sums: lanes l and l ^ 32 hold the two row halves of
    // column l % 32; with whole-row tiles wave wm = 1 hands its sums to wm = 0
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        s1[j][p] += __shfl_xor(s1[j][p], 32);
        s2[j][p] += __shfl_xor(s2[j][p], 32);
      }
    if (G::NI == 1) {
      double* red = reinterpret_cast<double*>(otile + TILE_BYTES);
      if (wm == 1 && lane < 32)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          red[((wn * TN + j) * 32 + lane) * 2] = s1[j][0];
          red[((wn * TN + j) * 32 + lane) * 2 + 1] = s2[j][0];
        }
      __syncthreads();
      if (wm == 0 && lane < 32) {
        const int slots = conv_lp_stat_slots(2 * L), slot = (m0 >> 8) & (slots - 1);
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int n = n0 + 64 * wn + 32 * j + lane;
          double* d = a.chstats + (((size_t)b0 * slots + slot) * a.cout + n) * 2;
          d[0] = s1[j][0] + red[((wn * TN + j) * 32 + lane) * 2];
          d[1] = s2[j][0] + red[((wn * TN + j) * 32 + lane) * 2 + 1];
        }
      }
    } else if (lane < 32) {
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          const int b = b0 + 2 * wm + p;
          if (b >= a.nb) continue;
          double* d = a.chstats + ((size_t)b * a.cout + n0 + 64 * wn + 32 * j + lane) * 2;
          d[0] = s1[j][p];
          d[1] = s2[j][p];
        }
    }
  }
  if (want_stats) {
    const int gs = a.cout / a.groups;                // channels per group: 1..32, a power of two
    const int slots = conv_lp_stat_slots(2 * L);
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        s1[j][p] += __shfl_xor(s1[j][p], 32);
        s2[j][p] += __shfl_xor(s2[j][p], 32);
        for (int off = 1; off < gs; off <<= 1) {
          s1[j][p] += __shfl_xor(s1[j][p], off);
          s2[j][p] += __shfl_xor(s2[j][p], off);
        }
      }
    const bool writer = lane < 32 && (lane & (gs - 1)) == 0;
    if (G::NI == 1) {
      // the two row halves of the tile: wave wm = 1 hands its sums to wm = 0
      double* red = reinterpret_cast<double*>(otile + TILE_BYTES);   // past the output tile
      if (wm == 1 && writer)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          red[((wn * TN + j) * 32 + lane) * 2] = s1[j][0];
          red[((wn * TN + j) * 32 + lane) * 2 + 1] = s2[j][0];
        }
      __syncthreads();
      if (wm == 0 && writer) {
        const int slot = (m0 >> 8) & (slots - 1);
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int g = (n0 + 64 * wn + 32 * j + lane) / gs;
          double* d = a.stats + (((size_t)b0 * slots + slot) * a.groups + g) * 2;
          d[0] = s1[j][0] + red[((wn * TN + j) * 32 + lane) * 2];
          d[1] = s2[j][0] + red[((wn * TN + j) * 32 + lane) * 2 + 1];
        }
      }
    } else if (writer) {
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          const int b = b0 + 2 * wm + p;
          if (b >= a.nb) continue;
          const int g = (n0 + 64 * wn + 32 * j + lane) / gs;
          double* d = a.stats + ((size_t)b * a.groups + g) * 2;
          d[0] = s1[j][p];
          d[1] = s2[j][p];
        }
    }
  }
}

template <int BM, int BN, int WM, int WN, int MINB>
void launch_dl(hipStream_t st, const ConvLpArgs& a) {
  const int M = a.nb << (a.lh + a.lw);
  const int mt = (M + BM - 1) / BM, nt = a.cout / BN;
  if (a.taps == 9)
    hipLaunchKernelGGL((conv_bf16_dl_kernel<9, BM, BN, WM, WN, MINB>), dim3(mt * nt), dim3(256), 0, st, a, nt);
  else
    hipLaunchKernelGGL((conv_bf16_dl_kernel<1, BM, BN, WM, WN, MINB>), dim3(mt * nt), dim3(256), 0, st, a, nt);
  TD_LAUNCHED();
}

template <int L>
void launch_halo(hipStream_t st, const ConvLpArgs& a) {
  const int M = a.nb << (2 * L);
  const int mt = (M + 255) / 256, nt = a.cout / 128;
  const dim3 grid(mt * nt);
  if constexpr (L >= 5) {
    if (a.act_scale) {
      hipLaunchKernelGGL((conv_bf16_halo_kernel<L, 2, 9, false, true>), grid, dim3(256), 0, st, a, nt);
      TD_LAUNCHED();
      return;
    }
  }
  if (a.taps == 9 && a.act2)
    hipLaunchKernelGGL((conv_bf16_halo_kernel<L, 2, 9, true, false>), grid, dim3(256), 0, st, a, nt);
  else if (a.taps == 9)
    hipLaunchKernelGGL((conv_bf16_halo_kernel<L, 2, 9, false, false>), grid, dim3(256), 0, st, a, nt);
  else
    hipLaunchKernelGGL((conv_bf16_halo_kernel<L, 2, 1, false, false>), grid, dim3(256), 0, st, a, nt);
  TD_LAUNCHED();
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

namespace {
// the halo-staged kernel's shapes: square images of side 8..64, C_in % 32 ==
// 0, C_out % 128 == 0, fragment-ordered BF16 weights, fewer than 2^28 pixels
bool halo_shape(const ConvLpArgs& a) {
  return a.wfrag && !a.w8 && a.lh == a.lw && a.lw >= 3 && a.lw <= 6 && a.cin % 32 == 0 && a.cout % 128 == 0 &&
         ((int64_t)a.nb << (a.lh + a.lw)) < ((int64_t)1 << 28);
}
}  // namespace

bool conv_lp_fused_ok(const ConvLpArgs& a) {
  const bool halo = halo_shape(a);
  if (!halo || (a.out16 && a.res)) return false;
  if (a.act2 && (a.taps != 9 || a.cin2 < 32 || a.cin2 % 32 != 0)) return false;
  if (a.act_scale && (!a.act_shift || a.taps != 9 || a.lw < 5 || a.cin > kActMaxCin || a.out16 || a.act2))
    return false;
  if (a.chstats && (a.out16 || a.stats)) return false;
  if (!a.stats) return true;
  const int gs = a.groups > 0 && a.cout % a.groups == 0 ? a.cout / a.groups : 0;
  return gs >= 1 && gs <= 32 && (gs & (gs - 1)) == 0;
}

void launch_conv_lp(hipStream_t st, const ConvLpArgs& a) {
  TD_CHECK(a.cin % 8 == 0 && a.cout % 16 == 0 && a.cout > 0, -5,
           "bf16 conv: needs C_in % 8 == 0 and C_out % 16 == 0");
  TD_CHECK(a.taps == 9 || a.taps == 1, -5, "bf16 conv: taps must be 9 or 1");
  TD_CHECK(a.lh + a.lw <= 20, -5, "bf16 conv: image too large");
  check_conv_rows(a.nb, a.lh + a.lw);
  if (!a.nb) return;
  const bool fast = a.cin % 32 == 0;
  const int BK = 32;
  TD_CHECK(a.kp % BK == 0 && a.kp >= a.taps * a.cin, -5, "bf16 conv: bad padded K");
  const double Md = (double)((int64_t)a.nb << (a.lh + a.lw));
  prof_begin(st);
  TD_CHECK(!a.w8 || a.wscale, -5, "fp8 weights need per-channel scales");
  // square images of side 8..64 with C_in % 32 == 0, C_out % 128 == 0 and
  // fragment-ordered BF16 weights: the halo-staged kernel (3x3 and 1x1).
  // Other 3x3 shapes with C_in % 32 == 0: the direct-to-LDS ring; the rest
  // (and FP8 weights): the register-staged kernel.
  const bool halo = halo_shape(a);
  TD_CHECK(!(a.out16 || a.stats || a.chstats || a.act2 || a.act_scale) || conv_lp_fused_ok(a), -5,
           "bf16 conv: a BF16 output, GroupNorm sums, a fused 1x1 or a staged activation need the halo-staged kernel");
  if (halo && a.lw == 6) launch_halo<6>(st, a);
  else if (halo && a.lw == 5) launch_halo<5>(st, a);
  else if (halo && a.lw == 4) launch_halo<4>(st, a);
  else if (halo) launch_halo<3>(st, a);
  else if (fast && !a.w8 && a.taps == 9 && a.cout % 128 == 0) launch_dl<128, 128, 2, 2, 3>(st, a);
  else if (fast && !a.w8 && a.taps == 9 && a.cout % 64 == 0) launch_dl<128, 64, 2, 2, 3>(st, a);
  else if (a.cout % 128 == 0) launch_lp_w<128, 2, 2>(st, a, fast);
  else if (a.cout % 64 == 0) launch_lp_w<64, 2, 2>(st, a, fast);
  else if (a.cout % 32 == 0) launch_lp_w<32, 4, 1>(st, a, fast);
  else launch_lp_w<16, 4, 1>(st, a, fast);
  const double cin2 = a.act2 ? a.cin2 : 0.0;
  prof_end(st, a.taps == 9 ? K_CONV3_LP : K_CONV1_LP, 2.0 * Md * a.cout * (a.taps * a.cin + cin2),
           2.0 * Md * (a.cin + cin2) + 2.0 * (a.kp + cin2) * a.cout + (a.out16 ? 2.0 : 4.0) * Md * a.cout +
               (a.res ? 4.0 * Md * a.cout : 0.0));
}

}  // namespace td
