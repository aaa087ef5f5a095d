// Implicit-GEMM convolution on CDNA4 matrix cores in FP32
// (v_mfma_f32_16x16x4_f32, FP32 accumulation), batched over windows.
//
// GEMM view (activations NHWC, one image per window):
//   M = windows * h * w output pixels, N = C_out, K = taps * C_in,
//   out[m][n] = bias[n] + res[m][n] + sum_k act(A[m][k]) * Wt[k][n]
// where A is the shifted input (3x3 with zero padding, or 1x1), read
// through a virtual channel concat of two tensors (decoder skip
// connections), with optional nearest 2x upsampling of the first
// (decoder resolution change) and an optional GroupNorm affine + SiLU
// prologue applied while staging into LDS (padding stays exactly zero).
//
// Tiling: 128 (M) x BN (N) per 256-thread workgroup, 4 waves of 64 lanes in
// a WM x WN grid; K advances 16 input channels of one tap per stage, double
// buffered in LDS.  Each lane of an MFMA reads its TM (resp. TN) operands
// for all of its wave's tiles with one vector LDS read: tile r of a wave
// owns rows {TM*i + r}, so the rows a lane needs are contiguous.  The
// K-loop order is fixed (tap-major, then channel chunks), so every output
// element is reduced in the same order whatever the batch composition:
// results are batch-invariant, which the bit-exact seed consistency of the
// sampler relies on.
//
// Convolutions whose input is already activated and dense (one source, no
// upsampling) take a specialisation with fewer live registers that reads
// the LDS operands of k-step kk + 1 while the MFMAs of kk run; the MFMA
// sequence per accumulator is unchanged, so results are identical.
//
// Workgroups are remapped so that each XCD (blockIdx % 8) walks a
// contiguous range of tiles: neighbouring N tiles of one M tile share the
// activation rows in that XCD's L2.
#include "td_internal.h"

namespace td {
namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float silu_f(float v) {
  return v * __builtin_amdgcn_rcpf(1.0f + __expf(-v));
}

// GroupNorm sums of a conv output tile (128 pixels x BN channels), from each
// lane's FP64 sums over its 16 rows for its TN consecutive channels
// (columns n_wave + TN * (lane % 16) + j): over the four lanes holding the
// other rows of those columns, over the group's channels, then over the
// tile's two row halves when both belong to one window (a window of at
// least 128 pixels); in that fixed order.  Written per (window, tile of the
// window, group) to a.stats.  lds: at least 2 KB of LDS free for the
// exchange (the operand buffers after the K loop).
template <int TN, int WM>
__device__ void conv_stats_epilogue(const ConvArgs& a, double* s1, double* s2, int m0, int n_wave, int lane, int wm,
                                    int wn, int M, int lhw, float* lds) {
  static_assert(WM == 2, "two row halves per tile");
#pragma unroll
  for (int j = 0; j < TN; ++j)
    for (int off = 16; off < 64; off <<= 1) {
      s1[j] += __shfl_xor(s1[j], off);
      s2[j] += __shfl_xor(s2[j], off);
    }
  const int gs = a.cout / a.groups;
  // per group: within the lane (gs <= TN) or over gs / TN neighbouring lanes
  double g1[TN], g2[TN];
  int ng = 0;
  if (gs <= TN) {
    for (int j0 = 0; j0 < TN; j0 += gs) {
      double t1 = 0, t2 = 0;
      for (int j = j0; j < j0 + gs; ++j) {
        t1 += s1[j];
        t2 += s2[j];
      }
      g1[ng] = t1;
      g2[ng] = t2;
      ++ng;
    }
  } else {
    double t1 = 0, t2 = 0;
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      t1 += s1[j];
      t2 += s2[j];
    }
    for (int off = 1; off < gs / TN; off <<= 1) {
      t1 += __shfl_xor(t1, off);
      t2 += __shfl_xor(t2, off);
    }
    g1[0] = t1;
    g2[0] = t2;
    ng = 1;
  }
  const int l16 = lane & 15;
  const bool writer = lane < 16 && (gs <= TN || (l16 & (gs / TN - 1)) == 0);
  const int gbase = (n_wave + TN * l16) / gs;   // first group of this lane's columns
  const int hw = 1 << lhw;
  double* red = reinterpret_cast<double*>(lds);
  if (hw >= 128) {
    // both row halves are one window: wave wm = 1 hands its sums to wm = 0
    __syncthreads();
    if (wm == 1 && writer)
      for (int q = 0; q < ng; ++q) {
        red[((wn * 16 + l16) * TN + q) * 2] = g1[q];
        red[((wn * 16 + l16) * TN + q) * 2 + 1] = g2[q];
      }
    __syncthreads();
    if (wm == 0 && writer && m0 < M) {
      const int slots = conv_stat_slots(lhw);
      const int b = m0 >> lhw, slot = (m0 >> 7) & (slots - 1);
      for (int q = 0; q < ng; ++q) {
        double* d = a.stats + (((size_t)b * slots + slot) * a.groups + gbase + q) * 2;
        d[0] = g1[q] + red[((wn * 16 + l16) * TN + q) * 2];
        d[1] = g2[q] + red[((wn * 16 + l16) * TN + q) * 2 + 1];
      }
    }
  } else if (writer) {
    // 64-pixel windows: each row half is a window of its own
    const int m = m0 + 64 * wm;
    if (m < M)
      for (int q = 0; q < ng; ++q) {
        double* d = a.stats + ((size_t)(m >> lhw) * a.groups + gbase + q) * 2;
        d[0] = g1[q];
        d[1] = g2[q];
      }
  }
}

// DENSE: one source, no upsampling, no activation (the input is already
// activated); fewer live registers, which leaves room to double-buffer the
// LDS operand reads of consecutive k-steps.
// Zeros that the dense path's out-of-image taps read instead of the image
// (C_in <= kConvDenseMaxCin), so that no select follows their loads.
__device__ __attribute__((aligned(16))) float g_conv_zero[kConvDenseMaxCin + 16];

template <int TAPS, int BN, int WM, int WN, bool DENSE>
__global__ __launch_bounds__(256, 4) void conv_kernel(ConvArgs a, int n_tiles_n) {
  constexpr int BM = 128, BK = 16, KS = BK / 4;
  constexpr int TM = BM / WM / 16, TN = BN / WN / 16;
  constexpr int AS = BM + 4, BS = BN + 4;
  constexpr int NBL = (BK * BN / 4 + 255) / 256;  // float4 B loads per thread
  __shared__ __attribute__((aligned(16))) float As[2][BK * AS];
  __shared__ __attribute__((aligned(16))) float Bs[2][BK * BS];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;

  const int bid = blockIdx.x;
  const int nblk = gridDim.x;
  const int tile = ((nblk & 7) == 0) ? (bid & 7) * (nblk >> 3) + (bid >> 3) : bid;
  const int tn = tile % n_tiles_n, tm = tile / n_tiles_n;
  const int m0 = tm * BM, n0 = tn * BN;

  const int lw = a.lw, lh = a.lh;
  const int W = 1 << lw, H = 1 << lh, lhw = lw + lh;
  const int M = a.nb << lhw;
  const int c0 = a.c0, c1 = DENSE ? 0 : a.c1, cin = c0 + c1;

  // Per-thread A staging slots: 2 float4 (pixel aml, channel quad akq).
  int ab[2], ay[2], ax[2], akq[2], aml[2];
  bool aval[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int e = tid + 256 * i;
    aml[i] = e % BM;
    akq[i] = e / BM;
    const int m = m0 + aml[i];
    aval[i] = m < M;
    const int mm = aval[i] ? m : 0;
    ab[i] = mm >> lhw;
    const int r = mm & ((1 << lhw) - 1);
    ay[i] = r >> lw;
    ax[i] = r & (W - 1);
  }

  // Tap state of the chunk being loaded: per-slot base pointers of the
  // shifted pixel in both sources.  Out-of-image pixels point at the zero
  // array (dense path), or at a valid pixel and are zeroed after the load
  // (branch-free, always in bounds).
  const float* p0[2];
  const float* p1[2];
  bool pok[2];
  auto set_tap = [&](int tap) {
    int dy = 0, dx = 0;
    if (TAPS == 9) { dy = tap / 3 - 1; dx = tap % 3 - 1; }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int yy = ay[i] + dy, xx = ax[i] + dx;
      const bool ok = aval[i] && yy >= 0 && yy < H && xx >= 0 && xx < W;
      const int yc = ok ? yy : 0, xc = ok ? xx : 0;
      pok[i] = ok;
      if (!DENSE && a.up0)
        p0[i] = a.src0 + ((((size_t)ab[i] << (lhw - 2)) + ((size_t)(yc >> 1) << (lw - 1)) + (xc >> 1)) * c0 + 4 * akq[i]);
      else if (DENSE && !ok)
        p0[i] = g_conv_zero + 4 * akq[i];
      else
        p0[i] = a.src0 + ((((size_t)ab[i] << lhw) + ((size_t)yc << lw) + xc) * c0 + 4 * akq[i]);
      p1[i] = (!DENSE && c1) ? a.src1 + ((((size_t)ab[i] << lhw) + ((size_t)yc << lw) + xc) * c1 + 4 * akq[i]) : a.src0;
    }
  };

  f4v ra[2], rb[NBL];
  auto load_chunk = [&](int tap, int ci0) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const float* p = (DENSE || ci0 < c0) ? p0[i] + ci0 : p1[i] + (ci0 - c0);
      ra[i] = *reinterpret_cast<const f4v*>(p);

    }
#pragma unroll
    for (int i = 0; i < NBL; ++i) {
      const int e = tid + 256 * i;
      if (e < BK * BN / 4) {
        const int row = e / (BN / 4), c4 = e % (BN / 4);
        rb[i] = *reinterpret_cast<const f4v*>(a.wt + ((size_t)(tap * cin + ci0 + row) * a.cout + n0 + 4 * c4));
      }
    }
  };

  auto store_chunk = [&](int buf, int ci0) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      f4v v = ra[i];
      if (!DENSE && a.act) {
        const size_t so = (size_t)ab[i] * cin + ci0 + 4 * akq[i];
        v = v * *reinterpret_cast<const f4v*>(a.gn_scale + so) + *reinterpret_cast<const f4v*>(a.gn_shift + so);
        if (a.act == 2) {
          v.x = silu_f(v.x); v.y = silu_f(v.y); v.z = silu_f(v.z); v.w = silu_f(v.w);
        }
      }
      if (!DENSE && !pok[i]) v = (f4v){0.f, 0.f, 0.f, 0.f};
      float* dst = &As[buf][(4 * akq[i]) * AS + aml[i]];
      dst[0] = v.x;
      dst[AS] = v.y;
      dst[2 * AS] = v.z;
      dst[3 * AS] = v.w;
    }
#pragma unroll
    for (int i = 0; i < NBL; ++i) {
      const int e = tid + 256 * i;
      if (e < BK * BN / 4) {
        const int row = e / (BN / 4), c4 = e % (BN / 4);
        *reinterpret_cast<f4v*>(&Bs[buf][row * BS + 4 * c4]) = rb[i];
      }
    }
  };

  f4v acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = (f4v){0.f, 0.f, 0.f, 0.f};

  const int nchunks = TAPS * (cin / BK);
  int tap_n = 0, ci_n = 0;
  set_tap(0);
  load_chunk(0, 0);
  store_chunk(0, 0);
  __syncthreads();

  const int arow = wm * (BM / WM) + TM * (lane & 15);
  const int brow = wn * (BN / WN) + TN * (lane & 15);
  const int kl = lane >> 4;

  for (int c = 0; c < nchunks; ++c) {
    const int buf = c & 1;
    const bool more = c + 1 < nchunks;
    if (more) {
      ci_n += BK;
      if (ci_n == cin) {
        ci_n = 0;
        ++tap_n;
        set_tap(tap_n);
      }
      load_chunk(tap_n, ci_n);
    }
    const float* Ab = As[buf];
    const float* Bb = Bs[buf];
    if constexpr (DENSE && TM == 4 && TN == 4) {
      // operands of k-step kk + 1 are read while the MFMAs of kk run
      f4v ac = *reinterpret_cast<const f4v*>(&Ab[kl * AS + arow]);
      f4v bc = *reinterpret_cast<const f4v*>(&Bb[kl * BS + brow]);
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) {
        f4v an = ac, bn = bc;
        if (kk + 1 < KS) {
          an = *reinterpret_cast<const f4v*>(&Ab[((kk + 1) * 4 + kl) * AS + arow]);
          bn = *reinterpret_cast<const f4v*>(&Bb[((kk + 1) * 4 + kl) * BS + brow]);
        }
        __builtin_amdgcn_sched_barrier(0);   // keep those reads ahead of this k-step's MFMAs
        const float av4[4] = {ac.x, ac.y, ac.z, ac.w}, bv4[4] = {bc.x, bc.y, bc.z, bc.w};
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av4[i], bv4[j], acc[i][j], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
        ac = an;
        bc = bn;
      }
    } else {
      // All LDS operand reads of the stage first, then the MFMA chain.
      float av[KS][TM], bv[KS][TN];
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) {
        const int krow = kk * 4 + kl;
        if constexpr (TM == 4) {
          f4v t = *reinterpret_cast<const f4v*>(&Ab[krow * AS + arow]);
          av[kk][0] = t.x; av[kk][1] = t.y; av[kk][2] = t.z; av[kk][3] = t.w;
        } else {
#pragma unroll
          for (int r = 0; r < TM; ++r) av[kk][r] = Ab[krow * AS + arow + r];
        }
        if constexpr (TN == 4) {
          f4v t = *reinterpret_cast<const f4v*>(&Bb[krow * BS + brow]);
          bv[kk][0] = t.x; bv[kk][1] = t.y; bv[kk][2] = t.z; bv[kk][3] = t.w;
        } else {
#pragma unroll
          for (int r = 0; r < TN; ++r) bv[kk][r] = Bb[krow * BS + brow + r];
        }
      }
#pragma unroll
      for (int kk = 0; kk < KS; ++kk)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[kk][i], bv[kk][j], acc[i][j], 0, 0, 0);
    }
    if (more) store_chunk(buf ^ 1, ci_n);
    __syncthreads();
  }

  // Epilogue: lane holds D[4*(lane/16)+v][lane%16] of every tile.
  const int nb0 = n0 + brow;
  double st1[TN], st2[TN];   // GroupNorm sums of this lane's columns (a.stats)
#pragma unroll
  for (int j = 0; j < TN; ++j) st1[j] = st2[j] = 0.0;
  float bias_v[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) bias_v[j] = a.bias ? a.bias[nb0 + j] : 0.f;
#pragma unroll
  for (int i = 0; i < TM; ++i) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int m = m0 + wm * (BM / WM) + TM * (4 * kl + v) + i;
      if (m >= M) continue;
      float o[TN];
#pragma unroll
      for (int j = 0; j < TN; ++j) o[j] = acc[i][j][v] + bias_v[j];
      const size_t off = (size_t)m * a.cout + nb0;
      if (a.res) {
        if constexpr (TN == 4) {
          f4v r = *reinterpret_cast<const f4v*>(a.res + off);
          o[0] += r.x; o[1] += r.y; o[2] += r.z; o[3] += r.w;
        } else {
#pragma unroll
          for (int j = 0; j < TN; ++j) o[j] += a.res[off + j];
        }
      }
      if constexpr (TN == 4) {
        *reinterpret_cast<f4v*>(a.out + off) = (f4v){o[0], o[1], o[2], o[3]};
      } else {
#pragma unroll
        for (int j = 0; j < TN; ++j) a.out[off + j] = o[j];
      }
      if (a.stats)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          st1[j] += (double)o[j];
          st2[j] += (double)o[j] * o[j];
        }
    }
  }
  if constexpr (WM == 2 && TAPS == 9 && DENSE)   // the launcher allows sums for dense C_out % 128 == 0 (2 x 2 waves) only
    if (a.stats) conv_stats_epilogue<TN, WM>(a, st1, st2, m0, n0 + wn * (BN / WN), lane, wm, wn, M, lhw, &As[0][0]);
}

template <int BN, int WM, int WN>
void launch_cfg(hipStream_t st, const ConvArgs& a) {
  int M = a.nb << (a.lh + a.lw);
  int mt = (M + 127) / 128;
  int nt = a.cout / BN;
  // the dense path's out-of-image taps read g_conv_zero, which covers kConvDenseMaxCin channels
  const bool dense = !a.src1 && !a.c1 && !a.up0 && !a.act && a.c0 <= kConvDenseMaxCin;
  if (a.taps == 9 && dense)
    hipLaunchKernelGGL((conv_kernel<9, BN, WM, WN, true>), dim3(mt * nt), dim3(256), 0, st, a, nt);
  else if (a.taps == 9)
    hipLaunchKernelGGL((conv_kernel<9, BN, WM, WN, false>), dim3(mt * nt), dim3(256), 0, st, a, nt);
  else if (dense)
    hipLaunchKernelGGL((conv_kernel<1, BN, WM, WN, true>), dim3(mt * nt), dim3(256), 0, st, a, nt);
  else
    hipLaunchKernelGGL((conv_kernel<1, BN, WM, WN, false>), dim3(mt * nt), dim3(256), 0, st, a, nt);
  TD_LAUNCHED();
}

}  // namespace

void launch_conv(hipStream_t st, const ConvArgs& a) {
  int cin = a.c0 + a.c1;
  TD_CHECK(cin % 16 == 0 && (a.c1 == 0 || a.c0 % 16 == 0), -5, "conv: input channels must be multiples of 16");
  TD_CHECK(a.taps == 9 || a.taps == 1, -5, "conv: taps must be 9 or 1");
  TD_CHECK(!a.up0 || (a.lh >= 1 && a.lw >= 1), -5, "conv: upsampled source needs h, w >= 2");
  TD_CHECK(a.lh + a.lw <= 20, -5, "conv: image too large");
  check_conv_rows(a.nb, a.lh + a.lw);
  if (a.nb == 0) return;
  TD_CHECK(a.cout % 16 == 0 && a.cout > 0, -5, "conv: output channels must be a multiple of 16");
  if (a.stats) {
    const int gs = a.groups > 0 && a.cout % a.groups == 0 ? a.cout / a.groups : 0;
    TD_CHECK(a.taps == 9 && !a.src1 && !a.c1 && !a.up0 && !a.act && a.c0 <= kConvDenseMaxCin && a.cout % 128 == 0 &&
                 gs >= 1 && gs <= 64 &&
                 (gs & (gs - 1)) == 0 && a.lh + a.lw >= 6 && conv_stat_slots(a.lh + a.lw) <= 32,
             -5, "conv: GroupNorm sums need a dense 3x3 conv with C_out % 128 == 0 and windows of at least 64 px");
  }
  const double M = (double)a.nb * (1 << (a.lh + a.lw));
  const double in_bytes = 4.0 * (a.up0 ? M / 4 * a.c0 + M * a.c1 : M * cin);
  const double bytes = in_bytes + 4.0 * a.taps * cin * a.cout + 4.0 * M * a.cout * (a.res ? 2 : 1);
  prof_begin(st);
  if (a.cout % 128 == 0) launch_cfg<128, 2, 2>(st, a);
  else if (a.cout % 64 == 0) launch_cfg<64, 2, 2>(st, a);
  else if (a.cout % 32 == 0) launch_cfg<32, 4, 1>(st, a);
  else launch_cfg<16, 4, 1>(st, a);
  prof_end(st, a.taps == 9 ? K_CONV3 : K_CONV1, 2.0 * M * a.cout * a.taps * cin, bytes);
}

}  // namespace td
