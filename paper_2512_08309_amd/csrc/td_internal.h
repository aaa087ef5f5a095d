// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "td_error.h"

namespace td {

// ---------------------------------------------------------------- errors --

#define TD_HIP(expr)                                                          \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess) {                                                   \
      throw ::td::Error{e_ == hipErrorOutOfMemory ? -2 : -3,                  \
                        std::string(#expr) + ": " + hipGetErrorString(e_)};   \
    }                                                                         \
  } while (0)

// Row count of a batched convolution, windows x pixels: the kernels index
// rows and tiles in 32-bit ints, so it must stay below 2^31 with a tile of
// slack.  The automatic batch keeps it far below; an explicit batch option
// can ask for more, which is refused here before any launch.
inline void check_conv_rows(int nb, int lhw) {
  TD_CHECK(nb >= 0 && lhw >= 0 && lhw <= 20 && ((int64_t)nb << lhw) <= (int64_t)0x7fffffff - 4096, -1,
           "conv: windows x pixels per launch must stay below 2^31");
}

// Launch check: catches bad launch configurations immediately.
#define TD_LAUNCHED() TD_HIP(hipGetLastError())

// ------------------------------------------------------------- profiling --
// Opt-in per-launch event timing (kernel class, algorithmic FLOPs and HBM
// bytes of the launch).  When no profiler is installed the hooks are no-ops.
enum KClass {
  K_CONV3 = 0, K_CONV1, K_GN, K_CONV_IN, K_CONV_OUT, K_ATTN, K_POOL, K_NOISE, K_BLEND, K_DECODE, K_LG, K_EMB,
  K_CONV3_LP, K_CONV1_LP, K_APPLY, K_GATHER, K_WGRAD, K_APPLY32, K_ENCODE, K_NCLASS
};
const char* kclass_name(int k);
struct Profiler;
extern thread_local Profiler* g_prof;
void prof_begin(hipStream_t st);
void prof_end(hipStream_t st, int cls, double flops, double bytes);

// ---------------------------------------------------------------- kernels --

// Geometry of one level's window set relative to a dense canvas.
struct WinGeom {
  int size;       // window side H
  int stride;     // s
  int channels;   // C
};

// Counter-hash Gaussian noise scaled by `scale` on a region.  layout 0:
// [h][w][C] with row pitch w*C; layout 1: planar [C][h][w].  accumulate:
// out += scale * G instead of out = scale * G.
void launch_noise(hipStream_t st, uint64_t seed, int64_t x0, int64_t y0,
                  int w, int h, int C, uint32_t step, float scale, int layout,
                  float* out, int accumulate = 0);

// Blend of cached window contributions:
//   out(p) = sum_i V_i(p - o_i) / sum_i W(p - o_i)   (0 where no window covers p)
// Pixel p = (bx + rx, by + ry) for rx in [0,w), ry in [0,h); (bx, by) is the
// origin of window (ix0, iy0).  ptrs[(iy-iy0)*nx + (ix-ix0)] -> [H][H][C].
void launch_blend(hipStream_t st, const WinGeom& g, int rx0, int ry0, int w,
                  int h, int nx, int ny, const float* const* ptrs,
                  const float* w1d, int layout, float* out);

void launch_fill(hipStream_t st, float* p, size_t n, float v);

// Window gather (Alg. 1's J_{t+1}[R_i]) from per-window canvases into a
// dense batch [nb][H][H][C]; src[b] points at the window's first pixel,
// pitch[b] is its canvas row length in pixels.
void launch_gather(hipStream_t st, const float* const* src, const int* pitch, int nb, int H, int C, float* out);

// Conditioning windows of a child model (hierarchy): window b reads a
// parent-resolution canvas base ([rows][pitch][cc]) nearest-upsampled by
// `factor`; its pixel (u, v) takes parent pixel ((offx + u) / factor,
// (offy + v) / factor) with offx, offy >= 0 the window origin relative to
// factor * (canvas origin).  out: [nb][H][H][cc].
struct CondSrc {
  const float* base;
  int pitch;
  int offx, offy;
  int pad;
};
void launch_cond_gather(hipStream_t st, const CondSrc* src, int nb, int H, int cc, int factor, float* out);

// Analytic linear-Gaussian denoiser + Euler step + weighting (see kernels).
// cond (nullable): [nwin][H][H][cc] conditioning added to the prior mean.
// direct: Phi = D (consistency sampling) instead of the Euler step.
void launch_lg_step(hipStream_t st, const WinGeom& g, const float* canvas,
                    int canvas_w, const int* origins, const int* widx,
                    const float* cond, int cc,
                    int nwin, double prior_std, double sigma, float c_euler,
                    int direct, const float* w1d, float* const* slots, int mode,
                    float* dout);

// Teacher judge of consistency sampling: per window b, r = RMS over the
// window of (ds - dt) ([nwin][H][H][C] each); flags[b] = (r > thr);
// counter (device, nullable) counts the flagged windows.
void launch_judge(hipStream_t st, const float* ds, const float* dt, int nwin, int H, int C, float thr, int* flags,
                  unsigned long long* counter);
// slots[b] = W (x) (pos[b] < 0 ? ds[b] : fb[pos[b]]) for b < nwin.
void launch_select(hipStream_t st, const float* ds, const float* fb, const int* pos, int nwin, int H, int C,
                   const float* w1d, float* const* slots);

struct ConvArgs {
  const float* src0;
  const float* src1;
  int c0, c1;            // channels of src0 / src1 (input = concat)
  int up0;               // src0 stored at half resolution (nearest 2x)
  const float* gn_scale; // [nb][cin] (act != 0)
  const float* gn_shift;
  int act;               // 0 none, 1 affine, 2 affine + SiLU
  int nb, lh, lw;        // batch, log2(height), log2(width)
  int cout;
  int taps;              // 9 (3x3, zero pad 1) or 1
  const float* wt;       // [taps][cin][cout]
  const float* bias;     // [cout]
  const float* res;      // [nb][h][w][cout] or null
  float* out;            // [nb][h][w][cout]
  // set: the output's GroupNorm sums (sum, sum of squares, FP64) per
  // (window, 128-pixel tile of the window, group of C_out / groups
  // channels), in the layout of the GroupNorm partials with
  // conv_stat_slots(lh + lw) tiles per window (3x3, dense input only)
  double* stats;
  int groups;
};
void launch_conv(hipStream_t st, const ConvArgs& a);
__host__ __device__ inline int conv_stat_slots(int lhw) { return lhw > 7 ? 1 << (lhw - 7) : 1; }
// Input channels of the dense (single-source, pre-activated) specialisation,
// which GroupNorm sums require.
constexpr int kConvDenseMaxCin = 8192;

// Reduced-precision conv: BF16 operands, FP32 accumulation and output.
struct ConvLpArgs {
  const uint16_t* act;   // [nb][h][w][cin] BF16, activation already applied
  int cin;
  int nb, lh, lw;
  int cout;
  int taps;              // 9 (3x3, zero pad 1) or 1
  int kp;                // padded K = round_up(taps * cin, 64 or 32)
  const void* wt;        // [cout][kp] BF16 (w8 = 0) or FP8 e4m3 (w8 = 1), K = tap * cin + c_in
  int w8;
  const float* wscale;   // per-output-channel weight scale (required for FP8) or null
  const float* bias;     // [cout]
  const float* res;      // [nb][h][w][cout] FP32 or null
  float* out;            // [nb][h][w][cout] FP32
  // BF16 weights in MFMA fragment order (conv_lp_frag_index), or null; used
  // for square images of side 8..64 with C_in % 32 == 0 and C_out % 128 == 0
  const void* wfrag;
  // Fused epilogue of that kernel only (conv_lp_fused_ok): out16 set stores
  // the output as BF16 instead of out (no residual); stats set writes the
  // output's GroupNorm sums (sum, sum of squares, FP64) per (window, tile of
  // the window, group of C_out / groups channels) in the layout of the
  // GroupNorm partials, with conv_lp_stat_slots(lh + lw) tiles per window.
  uint16_t* out16;
  double* stats;
  int groups;
  // set (FP32 output, with or without the residual): the output's per-
  // channel sums (sum, sum of squares, FP64) per (window, tile of the
  // window): [nb][conv_lp_stat_slots(lh + lw)][cout][2].  They let the
  // next GroupNorm over this tensor, alone or concatenated, skip its
  // statistics pass (launch_gn_finalize_ch).
  double* chstats;
  // set (3x3, halo-staged kernel only): a 1x1 convolution of act2 ([nb][h][w]
  // [cin2] BF16, cin2 % 32 == 0) is added in the same accumulators, its
  // weights following the 3x3 ones in K (fragment order over K = 9 cin +
  // cin2): a residual block's conv2 plus its skip projection in one pass.
  const uint16_t* act2;
  int cin2;
  // set (3x3 without act2, halo-staged kernel, square windows of side 32 or
  // 64, C_in <= kActMaxCin): act holds the raw tensor and the kernel stages SiLU(x *
  // act_scale + act_shift) of it (per-window GroupNorm affine [nb][cin]),
  // bit for bit as launch_apply_bf16 would have written it; out-of-image
  // taps stay zero.
  const float* act_scale;
  const float* act_shift;
};
constexpr int kActMaxCin = 512;
void launch_conv_lp(hipStream_t st, const ConvLpArgs& a);
bool conv_lp_fused_ok(const ConvLpArgs& a);
__host__ __device__ inline int conv_lp_stat_slots(int lhw) { return lhw > 8 ? 1 << (lhw - 8) : 1; }
// Element index, in the fragment-ordered weights of a convolution with K =
// taps * cin, of output channel o and K index k = tap * cin + c_in: for
// output block o / 32 and K block k / 16, the 64 lanes' 8-value B operands
// of v_mfma_f32_32x32x16_bf16 back to back (lane L: column L % 32, K values
// 8 (L / 32) .. + 7 of the block).
inline size_t conv_lp_frag_index(int o, int k, int K) {
  const int kb = k / 16, r = k % 16, lane = (o % 32) + 32 * (r / 8);
  return (((size_t)(o / 32) * (K / 16) + kb) * 64 + lane) * 8 + r % 8;
}
// K padding a weight matrix for launch_conv_lp needs.
inline int conv_lp_kp(int taps, int cin) { return (taps * cin + 31) / 32 * 32; }

// GroupNorm apply (+ SiLU) of the virtual conv input, written NHWC as BF16
// (out) or FP32 (out32, when set): act 0 = copy / convert only, 1 = affine,
// 2 = affine + SiLU.
struct ApplyArgs {
  const float* src0;
  const float* src1;
  int c0, c1, up0;
  const float* scale;
  const float* shift;
  int act;
  int nb, lh, lw;
  uint16_t* out;         // [nb][h][w][c0 + c1] BF16
  float* out32;          // [nb][h][w][c0 + c1] FP32 (instead of out)
  uint16_t* raw;         // with out: the input itself as BF16 too (no affine), or null
};
void launch_apply(hipStream_t st, const ApplyArgs& a);
// act(x * scale + shift) of a BF16 tensor [nb][h][w][C] into BF16 (the
// GroupNorm apply of a conv output stored as BF16).
void launch_apply_bf16(hipStream_t st, const uint16_t* src, int C, const float* scale, const float* shift, int act,
                       int nb, int lh, int lw, uint16_t* out);

struct GnArgs {
  const float* src0;
  const float* src1;
  int c0, c1, up0;
  int nb, lh, lw;
  int groups;
  float eps;
  const float* gamma;
  const float* beta;
  double* partial;       // workspace [nb][nchunk][groups][2]
  float* scale;          // [nb][cin]
  float* shift;
  float* mean = nullptr; // optional [nb][groups] statistics (training)
  float* rstd = nullptr;
};
size_t gn_partial_doubles(int nb, int lh, int lw, int cin, int groups);
void launch_gn(hipStream_t st, const GnArgs& a);
// scale/shift (and mean/rstd when set) from partials already in a.partial
// ([nb][nchunk][groups][2] sums and sums of squares), e.g. written by a
// convolution's epilogue.
void launch_gn_finalize(hipStream_t st, const GnArgs& a, int nchunk);
// scale/shift (and mean/rstd) of a GroupNorm over concat(src0, src1) (src0
// nearest-upsampled when a.up0) from the per-channel sums the producers of
// the two tensors wrote ([nb][slots][C][2], ConvLpArgs::chstats); a.src0 and
// a.src1 are not read.
void launch_gn_finalize_ch(hipStream_t st, const GnArgs& a, const double* ch0, int slots0, const double* ch1,
                           int slots1);
// GroupNorm statistics and apply (+ SiLU for act 2; act 1 affine only) of
// whole small windows in one pass, written as BF16 (out) or FP32 (out32);
// the partial/scale/shift fields of g are not used.  Fits when the window's
// virtual input is at most 32K elements (see gn_apply_window_fits).
bool gn_apply_window_fits(int lh, int lw, int c0, int c1, int up0, int groups);
void launch_gn_apply_window(hipStream_t st, const GnArgs& g, int act, uint16_t* out, float* out32);

void launch_avgpool(hipStream_t st, const float* in, float* out, int nb, int h,
                    int w, int C);

// conv_in: gathers each window from the canvas, scales by c_in, appends the
// window's conditioning channels (cond [nwin][H][H][ccond], unscaled; none
// when ccond = 0) and applies the 3x3 input conv (weights [9][cimg +
// ccond][c0]).  origins: [nwin][2] canvas-relative (x, y).
void launch_conv_in(hipStream_t st, const float* canvas, int canvas_w,
                    const int* origins, int nwin, int H, int cimg,
                    const float* cond, int ccond, int c0,
                    float c_in, const float* wt, const float* bias,
                    float* out);

// Output conv (GN + SiLU + 3x3 to cimg channels) fused with EDM
// preconditioning, the Euler step and the window weighting.  mode 0 writes
// V = W (x) Phi into slots[b]; mode 1 writes D to dout [nwin][H][H][cimg];
// mode 2 writes the Euler-stepped window (unweighted) to dout.
struct OutArgs {
  const float* h;        // [nb][H][H][c0]
  const float* gn_scale;
  const float* gn_shift;
  int nb, H, c0, cimg;
  const float* wt;       // [9][c0][cimg]
  const float* bias;     // [cimg]
  const float* canvas;   // window inputs x (un-preconditioned)
  int canvas_w;
  const int* origins;
  float c_skip, c_out, c_euler;
  int direct;            // 1: Phi = D (consistency sampling)
  const float* w1d;
  float* const* slots;
  int mode;
  float* dout;
};
void launch_conv_out(hipStream_t st, const OutArgs& a);

void launch_attention(hipStream_t st, const float* qkv, float* out, int nb,
                      int T, int C, int heads);

// out[k][o] = act(sum_i W[o][i] in[k][i] + b[o] + add[o]) for k < nk.
void launch_gemv(hipStream_t st, const float* W, const float* b,
                 const float* add, const float* in, float* out, int nk,
                 int nin, int nout, int act_silu);
void launch_pos_emb(hipStream_t st, const float* c_noise, int nk, int dim,
                    float max_period, float* out);

// Laplacian decode (see kernels file for the exact definition).
struct DecodeArgs {
  const float* latent;   // [lh][lw][C]
  int64_t lx0, ly0;
  int lw, lh, C;
  int64_t X0, Y0;
  int W, H;
  float* out;            // [H][W]
  float sigma_low, sigma_res;
  const float* taps;     // 2R+1 Gaussian taps
  int radius;
  const float* atoms;    // [3][8][8] atoms, then their 3 block means
  float* work0;          // latent-resolution scratch
  float* work1;
};
size_t decode_work_floats(const DecodeArgs& a);
// The fixed decode scratch of a device (16 MiB): init_decode_scratch looks
// up its address once per device (call with that device current);
// decode_scratch returns it (null before).
constexpr size_t kDecodeScratchFloats = (size_t)1 << 22;
constexpr int kMaxDevices = 64;
void init_decode_scratch(int device);
float* decode_scratch(int device);
void launch_decode(hipStream_t st, const DecodeArgs& a);

// Laplacian encode of elevation on an 8-aligned region [H][W] into the latent
// of blocks (R + 1 .. W/8 - R - 2) x (R + 1 .. H/8 - R - 2), [oh][ow][C].
struct EncodeArgs {
  const float* height;   // [H][W]
  int W, H, C;
  float sigma_low, sigma_res;
  const float* taps;     // 2R+1 Gaussian taps
  int radius;
  const float* atoms;    // [3][8][8]
  float* work0;          // (W/8) x (H/8) floats each
  float* work1;
  float* latent;         // [oh][ow][C]
};
void launch_encode(hipStream_t st, const EncodeArgs& a);

}  // namespace td
