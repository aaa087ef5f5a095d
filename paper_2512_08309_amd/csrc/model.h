// Loaded model: header constants, device weights in kernel layouts, the
// window-denoiser executor and its workspace.
#pragma once

#include <map>
#include <string>
#include <vector>

#include "header.h"
#include "td_internal.h"

namespace td {

struct ResBlockW {
  int cin = 0, cout = 0;
  bool has_skip = false;
  const float *gn1_g = nullptr, *gn1_b = nullptr, *w1 = nullptr, *gn2_g = nullptr, *gn2_b = nullptr;
  const float *w2 = nullptr, *b2 = nullptr, *wskip = nullptr, *bskip = nullptr;
  size_t bias_off = 0;     // offset of this block's [K + extra][cout] table in bias_eff
  const float *emb_w = nullptr, *emb_b = nullptr, *b1 = nullptr;   // Lin_emb and conv1 bias
  // reduced precision: [cout][kp] BF16 weights (K = tap * cin + c_in)
  const uint16_t *w1_lp = nullptr, *w2_lp = nullptr, *wskip_lp = nullptr;
  int kp1 = 0, kp2 = 0, kps = 0;
  // the weights again in MFMA fragment order (null where the halo-staged
  // kernel does not apply)
  const uint16_t *w1_fr = nullptr, *w2_fr = nullptr, *wskip_fr = nullptr;
  // conv2 and the skip projection as one convolution (K = 9 cout + cin,
  // fragment order) with bias b2 + bskip; null where the halo-staged
  // kernel does not apply
  const uint16_t* w2s_fr = nullptr;
  const float* b2s = nullptr;
  // FP8 e4m3 weights, same layout, with per-output-channel scales
  const uint8_t *w1_8 = nullptr, *w2_8 = nullptr, *wskip_8 = nullptr;
  const float *s1_8 = nullptr, *s2_8 = nullptr, *sskip_8 = nullptr;
};

struct AttnW {
  int C = 0;
  const float *gn_g = nullptr, *gn_b = nullptr, *wqkv = nullptr, *bqkv = nullptr, *wproj = nullptr,
              *bproj = nullptr;
  const uint16_t *wqkv_lp = nullptr, *wproj_lp = nullptr;
  int kpq = 0, kpp = 0;
  const uint16_t *wqkv_fr = nullptr, *wproj_fr = nullptr;   // MFMA fragment order
  const uint8_t *wqkv_8 = nullptr, *wproj_8 = nullptr;
  const float *sqkv_8 = nullptr, *sproj_8 = nullptr;
};

// Batch of windows for one denoiser round: inputs are read from a dense
// canvas ([rows][canvas_w][C]) at per-window origins.
struct WindowBatch {
  const float* canvas = nullptr;
  int canvas_w = 0;
  const int* d_origins = nullptr;   // [n][2] device
  const int* d_widx = nullptr;      // [n][2] device (window indices, analytic kind)
  float* const* d_slots = nullptr;  // [n] device pointers, mode 0
  float* dout = nullptr;            // mode 1: [n][H][H][C]
  const float* cond = nullptr;      // [n][H][H][Cc] conditioning windows (Cc > 0)
  int n = 0;
  int mode = 0;                     // 0: contributions W (x) Phi, 1: raw D, 2: Phi to dout
  // host copies for a judged consistency model (mode 0): window indices
  // [n][2], and the query seed (one for the batch, or per window)
  const int* h_widx = nullptr;
  uint64_t seed = 0;
  const uint64_t* h_seeds = nullptr;
};

// A judged window that falls back: its query seed and window index.
struct FallbackReq {
  uint64_t seed;
  int64_t ix, iy;
};
// Writes the judge's plain sample J_0 on the region of window req[j] to
// out[j] ([H][H][C]) for j < n; enqueued after everything on `st`, which
// waits for it.
using FallbackFn = void (*)(void* user, const FallbackReq* req, int n, float* out, hipStream_t st);

class Model {
 public:
  ModelDesc d;
  ~Model();
  void load(const std::string& path, hipStream_t st);
  // One denoiser round of a batch (n <= max_batch) at schedule index k
  // (sigma = sched[k]), Euler target sched[k+1]; k >= K selects a noise
  // level added by sigma_slot (raw estimates, mode 1, only).
  void run_batch(hipStream_t st, const WindowBatch& b, int k);
  // Index of noise level sigma: its schedule index, or a row of embedding
  // biases computed on first use (at most kExtraSigmas such levels).
  int sigma_slot(hipStream_t st, double sigma);
  double sigma_of(int k) const;
  // Consistency sampling with a teacher judge: a window whose estimate
  // differs from the teacher's one-step estimate by more than `threshold`
  // RMS takes the teacher's plain sample J_0 on its region, supplied by
  // `fallback`; `counter` (device) counts such windows.  teacher null: off.
  void set_judge(Model* teacher, float threshold, unsigned long long* counter, FallbackFn fallback = nullptr,
                 void* user = nullptr);
  // Phi of blend level t: the Euler steps points[T-t-1] .. points[T-t]-1 on
  // every window of the batch, the last one writing b.mode's output.
  void run_level(hipStream_t st, const WindowBatch& b, int t);
  int level_steps(int t) const { return d.points[d.T - t] - d.points[d.T - t - 1]; }
  size_t workspace_bytes_per_window() const;
  void ensure_workspace(int max_batch);
  int max_batch() const { return ws_batch_; }
  // [max_batch][H][H][Cc] conditioning windows of one batch (Cc > 0)
  float* cond_buffer() const { return cond_; }
  const float* w1d() const { return w1d_; }
  const float* decode_taps() const { return taps_; }
  const float* decode_atoms() const { return atoms_; }
  // 0: FP32 (FP32 MFMA); 1: BF16 operands, FP32 accumulation; 2: BF16
  // activations with FP8 e4m3 per-output-channel-scaled weights.
  void set_precision(int p);
  int precision() const { return prec_; }

 private:
  int prec_ = 0;
  std::vector<void*> allocs_;
  std::map<std::string, const float*> t_;
  float* w1d_ = nullptr;
  float* taps_ = nullptr;
  float* atoms_ = nullptr;
  // unet
  const float *conv_in_w_ = nullptr, *conv_in_b_ = nullptr, *out_gn_g_ = nullptr, *out_gn_b_ = nullptr;
  const float *out_w_ = nullptr, *out_b_ = nullptr;
  std::map<std::string, ResBlockW> rb_;
  std::map<std::string, AttnW> at_;
  float* bias_eff_ = nullptr;
  // workspace
  int ws_batch_ = 0;
  void* ws_ = nullptr;
  struct LevelBufs {
    float *T, *R, *X, *Y, *P, *Q, *O;
    std::vector<float*> S;
    uint16_t *A, *A0;      // BF16 operand buffers (reduced precision)
    float* F;              // activated FP32 input of a 3x3 conv (FP32)
  };
  std::vector<LevelBufs> lb_;
  float *gn_scale_ = nullptr, *gn_shift_ = nullptr;
  double* gn_part_ = nullptr;
  // Per-channel GroupNorm sums of the level buffers X, Y and S[j] (reduced
  // precision): written by the convolution that produced the buffer's
  // current contents (valid), [nb][slots][C][2].
  struct ChStats {
    double* buf = nullptr;
    int slots = 0, C = 0;
    bool valid = false;
  };
  std::map<const float*, ChStats> chs_;
  ChStats* chstats_of(const float* t);
  float* cond_ = nullptr;         // conditioning windows of a batch
  static constexpr int kExtraSigmas = 8;
  std::vector<double> extra_sigma_;
  const float *emb_l1w_ = nullptr, *emb_l1b_ = nullptr, *emb_l2w_ = nullptr, *emb_l2b_ = nullptr;
  float* emb_scratch_ = nullptr;
  Model* judge_ = nullptr;
  float judge_thr_ = 0.f;
  unsigned long long* judge_count_ = nullptr;
  FallbackFn fallback_ = nullptr;
  void* fallback_user_ = nullptr;
  float *judge_s_ = nullptr, *judge_t_ = nullptr;   // student / teacher estimates of a batch
  int *judge_flags_ = nullptr, *judge_pos_ = nullptr;
  // sigma_next_override >= 0: the Euler step goes to that level (mode 2)
  void run_net(hipStream_t st, const WindowBatch& b, int k, double sigma_next_override = -1.0);
  float* state_ = nullptr;        // window states between the steps of one Phi
  int* state_origins_ = nullptr;  // (0, b*H) for b < ws_batch_

  float* dalloc(size_t n);
  const float* upload(const std::vector<float>& v);
  const uint16_t* upload_lp(const std::vector<float>& w, int co, int ci, int k, int* kp);
  const uint16_t* upload_frag(const std::vector<float>& w, int co, int ci, int k);
  // [co][9 co] 3x3 weights followed in K by [co][ci] 1x1 weights, fragment order
  const uint16_t* upload_frag_cat(const std::vector<float>& w3, const std::vector<float>& w1, int co, int ci);
  const uint8_t* upload_fp8(const std::vector<float>& w, int co, int ci, int k, const float** scale);
  int cin_max(int lvl) const;
  // With track set, the output's per-channel sums are written where the
  // halo-staged kernel runs, and out's ChStats (if any) records whether they
  // were.
  void conv_lp(hipStream_t st, const uint16_t* act, int cin, int nb, int lr, int cout, int taps,
               const uint16_t* wt, const uint8_t* w8, const float* w8s, int kp, const float* bias,
               const float* res, float* out, const uint16_t* wfrag = nullptr, bool track = false,
               const float* act_scale = nullptr, const float* act_shift = nullptr);
  // conv1 of a BF16 residual block through the fused epilogue: BF16 output
  // into out16 and the GroupNorm sums of gn2 into gn_part_; false (nothing
  // launched) where the halo-staged kernel does not apply.
  bool conv1_fused(hipStream_t st, const ResBlockW& w, const uint16_t* act, int nb, int lr, const float* bias,
                   uint16_t* out16);
  // conv2 of a BF16 residual block with a 1x1 skip: one halo-staged launch
  // over (act, conv2 taps) then (act2, skip weights) into out, with its
  // per-channel sums; false (nothing launched) where that kernel does not apply
  bool conv2_skip_fused(hipStream_t st, const ResBlockW& w, const uint16_t* act, const uint16_t* act2, int nb, int lr,
                        float* out);
  // conv2 of a BF16 residual block with an identity skip can stage GroupNorm 2
  // + SiLU of conv1's raw BF16 output itself (gn_scale_ / gn_shift_)
  bool conv2_act_ok(const ResBlockW& w, int nb, int lr) const;
  void apply(hipStream_t st, const float* s0, int c0, int up0, const float* s1, int c1, int act, int nb,
             int lr, uint16_t* out, float* out32 = nullptr, uint16_t* raw = nullptr);
  void gn_apply(hipStream_t st, const float* s0, int c0, int up0, const float* s1, int c1, int nb, int lr,
                const float* g, const float* b, int act, uint16_t* out, float* out32);
  void conv3_f32(hipStream_t st, const float* in, int cin, int nb, int lr, int cout, const float* wt,
                 const float* bias, const float* res, float* out, double* stats = nullptr);
  void build_unet(const std::map<std::string, std::vector<float>>& host,
                  const std::map<std::string, std::vector<int>>& shapes, hipStream_t st);
  void gn(hipStream_t st, const float* s0, int c0, int up0, const float* s1, int c1, int nb, int lh, int lw,
          const float* g, const float* b);
  // gn's affine, from the producers' per-channel sums when both sources
  // carry valid ones, else through the statistics pass
  void gn_stats(hipStream_t st, const float* s0, int c0, int up0, const float* s1, int c1, int nb, int lh, int lw,
                const float* g, const float* b);
  void resblock(hipStream_t st, const ResBlockW& w, int k, const float* s0, int c0, int up0, const float* s1,
                int c1, int nb, int lvl, float* out);
  void attention(hipStream_t st, const AttnW& w, const float* in, int nb, int lvl, float* out);
};

}  // namespace td
