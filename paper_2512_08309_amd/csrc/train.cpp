// Student training: forward of the window UNet that keeps what its backward
// needs, the hand-written backward, the distillation loss and AdamW.
//
// Parameters live in one flat FP32 buffer laid out as the .tdw data section
// (every tensor at its file offset, file layout [co][ci][kh][kw] for convs),
// so the caller can load, update and save them as they are.  Gradients use
// the same layout.  A forward records a tape (one entry per layer) of the
// activations it saved; the next backward walks it in reverse.
//
// Layer math is the sampler's network (EDM-preconditioned UNet, GroupNorm +
// SiLU ResBlocks, 2x2 average pooling, nearest 2x upsampling with skip
// concatenation, window attention, positional noise embedding).  Forward
// kernels are the sampler's FP32 MFMA kernels; data gradients of convs run
// the same kernel on flipped, transposed weights; weight gradients,
// GroupNorm and attention backward are in k_train.hip.
#include <cmath>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/td.h"
#include "json.h"
#include "td_internal.h"

namespace td {

void tr_relayout(hipStream_t st, const float* w, int co, int ci, int kk, int co_pad, float* fwd, float* flip);
void tr_dense_in(hipStream_t st, const float* s0, int c0, int up0, const float* s1, int c1, int nb, int lh, int lw,
                 float* out);
void tr_act(hipStream_t st, const float* x, const float* scale, const float* shift, int nb, int hw, int C, int act,
            float* out);
void tr_gn_bwd(hipStream_t st, const float* x, const float* mean, const float* rstd, const float* gamma,
               const float* beta, const float* dA, int nb, int hw, int C, int groups, int act, int accumulate,
               float* dx, float* dgam_part, float* dbet_part);
void tr_sum_rows(hipStream_t st, const float* in, int rows, int C, int accumulate, float* out);
void tr_colsum(hipStream_t st, const float* in, size_t M, int C, float* part, int nchunk, int accumulate,
               float* out);
void tr_wgrad(hipStream_t st, const float* A, const float* dY, int nb, int lh, int lw, int ci, int co, int taps,
              float* part, int nsplit, float* grad);
void tr_attention_bwd(hipStream_t st, const float* qkv, const float* dO, int nb, int T, int C, int heads,
                      float* dqkv);
void tr_emb_bwd(hipStream_t st, float c_noise, int c0, int emb, float max_period, const float* W1, const float* b1,
                const float* W2, const float* b2, const float* de2, float* dW1, float* db1, float* dW2, float* db2);
void tr_emb_bias_bwd(hipStream_t st, const float* db, const float* e2, const float* Wemb, int cout, int emb,
                     float* dWemb, float* dbemb, float* dcb, float* de2);
void tr_mse(hipStream_t st, const float* D, const float* y, size_t n, float gscale, float* d, float* part);
void tr_pad_scale(hipStream_t st, const float* in, size_t npix, int C, int cpad, float s, float* out);
void tr_add(hipStream_t st, float* a, const float* b, size_t n);
void tr_pool_bwd(hipStream_t st, const float* dy, int nb, int lh, int lw, int C, int accumulate, float* dx);
void tr_split_bwd(hipStream_t st, const float* dd, int c0, int up0, int c1, int nb, int lh, int lw, int acc0,
                  float* ds0, float* ds1);
void tr_adamw(hipStream_t st, float* w, const float* g, float* m, float* v, size_t n, float lr, float b1, float b2,
              float eps, float wd, int step);
void tr_lp_weights(hipStream_t st, const float* w, int co, int ci, int kk, int kp, int flip, uint16_t* out);

namespace {

int ilog2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// Device memory in chunks that are never moved: pointers stay valid until reset.
class ChunkArena {
 public:
  ~ChunkArena() {
    for (auto& c : chunks_) (void)hipFree(c.p);
  }
  void reset() {
    cur_ = 0;
    for (auto& c : chunks_) c.used = 0;
  }
  float* take(size_t nfloat) {
    const size_t bytes = (nfloat * sizeof(float) + 255) / 256 * 256;
    while (cur_ < chunks_.size()) {
      Chunk& c = chunks_[cur_];
      if (c.used + bytes <= c.cap) {
        float* r = (float*)((char*)c.p + c.used);
        c.used += bytes;
        return r;
      }
      ++cur_;
    }
    Chunk c;
    c.cap = std::max<size_t>(bytes, (size_t)256 << 20);
    TD_HIP(hipMalloc(&c.p, c.cap));
    c.used = bytes;
    chunks_.push_back(c);
    cur_ = chunks_.size() - 1;
    return (float*)c.p;
  }

 private:
  struct Chunk {
    void* p = nullptr;
    size_t cap = 0, used = 0;
  };
  std::vector<Chunk> chunks_;
  size_t cur_ = 0;
};

struct TRef {
  size_t off = 0;   // floats into the flat parameter buffer
  std::vector<int> shape;
};

}  // namespace

class Trainer {
 public:
  ~Trainer() {
    if (origins_) (void)hipFree(origins_);
  }
  void load(const std::string& path);
  size_t param_floats() const { return nparam_; }
  // 0: FP32 convolutions; 1: BF16 operands of the forward and data-gradient
  // convolutions (FP32 accumulation, FP32 master weights and weight gradients)
  void set_precision(int p) {
    TD_CHECK(p == 0 || p == 1, -1, "training precision must be 0 or 1");
    prec_ = p;
  }
  void forward(hipStream_t st, const float* P, const float* x, int nb, double sigma, float* D);
  void backward(hipStream_t st, const float* P, const float* dD, float* G);

  // architecture
  int C = 0, H = 0, nres = 0, heads = 1, groups = 1, emb = 0;
  std::vector<int> ch;
  std::vector<int> attn_levels;
  bool mid_attn = false;
  float gn_eps = 1e-5f;
  double pe_max_period = 10000, sigma_data = 0.5;

 private:
  enum Kind { CONV_IN, RES, ATTN, POOL, OUT };
  struct Node {
    Kind kind;
    std::string p;         // parameter prefix
    int lvl = 0, lh = 0, cin = 0, cout = 0;
    // inputs
    const float* s0 = nullptr;
    const float* s1 = nullptr;
    int c0 = 0, c1 = 0, up0 = 0;
    const float* in = nullptr;   // dense input (== s0 when no concat/upsample)
    bool dense = false;
    // saved
    float *m1 = nullptr, *r1 = nullptr, *A1 = nullptr, *h1 = nullptr, *m2 = nullptr, *r2 = nullptr,
          *A2 = nullptr, *qkv = nullptr, *O = nullptr, *bias = nullptr;
    const float* out = nullptr;
  };

  std::map<std::string, TRef> t_;
  size_t nparam_ = 0;
  ChunkArena fa_, ba_;          // forward (saved) and backward (temporaries)
  std::vector<Node> tape_;
  int nb_ = 0;
  double sigma_ = 0;
  const float* x_ = nullptr;
  float* e2_ = nullptr;         // noise embedding of the tape's sigma
  float* Ain_ = nullptr;        // c_in x
  int* origins_ = nullptr;
  int origins_cap_ = 0;
  std::unordered_map<const float*, float*> grad_;
  // per-forward weight layouts: forward [tap][ci][co] and flipped [tap][co_pad][ci]
  std::map<std::string, std::pair<float*, float*>> wl_;
  // BF16 copies (precision 1): forward [co][kp] and data-gradient [ci][kp']
  struct LpW {
    uint16_t *fwd = nullptr, *flip = nullptr;
    int kp = 0, kpf = 0;
  };
  std::map<const float*, LpW> lp_;   // keyed by the forward layout's pointer
  int prec_ = 0;
  float* gn_scale_ = nullptr;
  float* gn_shift_ = nullptr;
  double* gn_part_ = nullptr;
  size_t gn_cap_ = 0;

  const float* P_ = nullptr;
  const float* prm(const std::string& n) const {
    auto it = t_.find(n);
    TD_CHECK(it != t_.end(), -5, "training: missing tensor " + n);
    return P_ + it->second.off;
  }
  float* grd(float* G, const std::string& n) const { return G + t_.at(n).off; }
  bool has(const std::string& n) const { return t_.count(n) > 0; }
  bool attn_at(int l) const {
    for (int a : attn_levels)
      if (a == l) return true;
    return false;
  }

  void layouts(hipStream_t st, const std::string& name, int co, int ci, int kk, int co_pad) {
    auto& e = wl_[name];
    if (!e.first) {
      e.first = fa_.take((size_t)co * ci * kk);
      e.second = fa_.take((size_t)co_pad * ci * kk);
    }
    tr_relayout(st, prm(name), co, ci, kk, co_pad, e.first, e.second);
    if (!prec_) return;
    // the BF16 kernel takes inputs in multiples of 8 channels and outputs in
    // multiples of 16; other shapes (the 4-channel input and output convs) stay FP32
    LpW l;
    if (co % 16 == 0 && ci % 8 == 0) {
      l.kp = conv_lp_kp(kk, ci);
      l.fwd = (uint16_t*)fa_.take(((size_t)co * l.kp + 1) / 2);
      tr_lp_weights(st, prm(name), co, ci, kk, l.kp, 0, l.fwd);
    }
    if (ci % 16 == 0 && co % 8 == 0) {
      l.kpf = conv_lp_kp(kk, co);
      l.flip = (uint16_t*)fa_.take(((size_t)ci * l.kpf + 1) / 2);
      tr_lp_weights(st, prm(name), co, ci, kk, l.kpf, 1, l.flip);
    }
    lp_[e.first] = l;
    lp_[e.second] = l;
  }
  // BF16 copy of a dense FP32 activation (precision 1)
  const uint16_t* to_bf16(ChunkArena& ar, const float* x, int C_, int lh) {
    uint16_t* o = (uint16_t*)ar.take((((size_t)nb_ << (2 * lh)) * C_ + 1) / 2);
    ApplyArgs a{};
    a.src0 = x;
    a.c0 = C_;
    a.act = 0;
    a.nb = nb_;
    a.lh = lh;
    a.lw = lh;
    a.out = o;
    launch_apply(st_, a);
    return o;
  }
  hipStream_t st_ = nullptr;
  // GroupNorm statistics of the virtual input concat(up0 ? up(s0) : s0, s1)
  void gn_stats(hipStream_t st, const float* s0, int c0, int up0, const float* s1, int c1, int lh, float* mean,
                float* rstd, const std::string& pre);
  void gn_stats(hipStream_t st, const float* x, int C_, int lh, float* mean, float* rstd, const std::string& pre) {
    gn_stats(st, x, C_, 0, nullptr, 0, lh, mean, rstd, pre);
  }
  float* conv(hipStream_t st, const float* A, int cin, int lh, int cout, int taps, const float* wfwd,
              const float* bias, const float* res);
  float* dgrad(hipStream_t st, const float* dY, int co, int lh, int ci, int taps, const float* flip);
  float* gradbuf(const float* act, size_t n, hipStream_t st);
  void bias_grad(hipStream_t st, const float* dY, size_t M, int C_, float* out);
  void gn_param_grads(hipStream_t st, const float* dgp, const float* dbp, int C_, float* G, const std::string& pre);
  const float* res_fwd(hipStream_t st, Node& n);
  void res_bwd(hipStream_t st, Node& n, float* G, float* de2);
  const float* attn_fwd(hipStream_t st, Node& n);
  void attn_bwd(hipStream_t st, Node& n, float* G);
};

void Trainer::load(const std::string& path) {
  std::ifstream f(path, std::ios::binary);
  TD_CHECK(f.good(), -4, "cannot open " + path);
  char head[8];
  f.read(head, 8);
  TD_CHECK(f.good() && std::memcmp(head, "TDW1", 4) == 0, -5, "not a TDW1 weight file");
  uint32_t n = 0;
  std::memcpy(&n, head + 4, 4);
  std::string htxt(n, '\0');
  f.read(&htxt[0], n);
  TD_CHECK(f.good(), -5, "truncated header");
  Json h = JsonParser(htxt).parse();
  const Json& dn = h.at("denoiser");
  TD_CHECK(dn.at("kind").str() == "unet", -5, "training needs a UNet denoiser");
  TD_CHECK(!h.has("cond"), -5, "training of conditioned models is not supported");
  C = (int)dn.at("in_channels").integer();
  ch.clear();
  for (const Json& v : dn.at("channels").arr()) ch.push_back((int)v.integer());
  nres = (int)dn.at("num_res_blocks").integer();
  attn_levels.clear();
  for (const Json& v : dn.at("attn_levels").arr()) attn_levels.push_back((int)v.integer());
  mid_attn = dn.at("mid_attn").boolean();
  heads = (int)dn.at("num_heads").integer();
  groups = (int)dn.at("gn_groups").integer();
  gn_eps = (float)dn.at("gn_eps").num();
  emb = (int)dn.at("emb_mult").integer() * ch[0];
  pe_max_period = dn.at("pe_max_period").num();
  sigma_data = h.at("sampler").at("sigma_data").num();
  H = (int)h.at("window").at("size").integer();
  TD_CHECK(H >= 16 && (H & (H - 1)) == 0 && (H >> (ch.size() - 1)) >= 2, -5, "training: window must be a power of 2");
  nparam_ = 0;
  t_.clear();
  for (const Json& e : h.at("tensors").arr()) {
    TRef r;
    r.off = (size_t)e.at("offset").integer() / 4;
    size_t cnt = 1;
    for (const Json& d : e.at("shape").arr()) {
      r.shape.push_back((int)d.integer());
      cnt *= (size_t)d.integer();
    }
    nparam_ = std::max(nparam_, r.off + cnt);
    t_[e.at("name").str()] = r;
  }
}

void Trainer::gn_stats(hipStream_t st, const float* s0, int c0, int up0, const float* s1, int c1, int lh,
                       float* mean, float* rstd, const std::string& pre) {
  const size_t need = (size_t)nb_ * (c0 + c1);
  if (need > gn_cap_) {
    gn_cap_ = std::max(need, (size_t)nb_ * 1024);
    gn_scale_ = fa_.take(gn_cap_);
    gn_shift_ = fa_.take(gn_cap_);
    gn_part_ = (double*)fa_.take(gn_partial_doubles(nb_, 8, 8, 1024, groups) * 2 + (size_t)nb_ * 16 * groups * 4);
  }
  GnArgs a;
  a.src0 = s0;
  a.src1 = s1;
  a.c0 = c0;
  a.c1 = c1;
  a.up0 = up0;
  a.nb = nb_;
  a.lh = lh;
  a.lw = lh;
  a.groups = groups;
  a.eps = gn_eps;
  a.gamma = prm(pre + ".weight");
  a.beta = prm(pre + ".bias");
  a.partial = gn_part_;
  a.scale = gn_scale_;
  a.shift = gn_shift_;
  a.mean = mean;
  a.rstd = rstd;
  launch_gn(st, a);
}

float* Trainer::conv(hipStream_t st, const float* A, int cin, int lh, int cout, int taps, const float* wfwd,
                     const float* bias, const float* res) {
  float* out = fa_.take(((size_t)nb_ << (2 * lh)) * cout);
  auto lp = lp_.find(wfwd);
  if (prec_ && lp != lp_.end() && lp->second.fwd) {
    st_ = st;
    ConvLpArgs c{};
    c.act = to_bf16(ba_, A, cin, lh);
    c.cin = cin;
    c.nb = nb_;
    c.lh = lh;
    c.lw = lh;
    c.cout = cout;
    c.taps = taps;
    c.kp = lp->second.kp;
    c.wt = lp->second.fwd;
    c.bias = bias;
    c.res = res;
    c.out = out;
    launch_conv_lp(st, c);
    return out;
  }
  ConvArgs c{};
  c.src0 = A;
  c.c0 = cin;
  c.nb = nb_;
  c.lh = lh;
  c.lw = lh;
  c.cout = cout;
  c.taps = taps;
  c.wt = wfwd;
  c.bias = bias;
  c.res = res;
  c.out = out;
  launch_conv(st, c);
  return out;
}

float* Trainer::dgrad(hipStream_t st, const float* dY, int co, int lh, int ci, int taps, const float* flip) {
  float* out = ba_.take(((size_t)nb_ << (2 * lh)) * ci);
  auto lp = lp_.find(flip);
  if (prec_ && lp != lp_.end() && lp->second.flip) {
    st_ = st;
    ConvLpArgs c{};
    c.act = to_bf16(ba_, dY, co, lh);
    c.cin = co;
    c.nb = nb_;
    c.lh = lh;
    c.lw = lh;
    c.cout = ci;
    c.taps = taps;
    c.kp = lp->second.kpf;
    c.wt = lp->second.flip;
    c.out = out;
    launch_conv_lp(st, c);
    return out;
  }
  ConvArgs c{};
  c.src0 = dY;
  c.c0 = co;
  c.nb = nb_;
  c.lh = lh;
  c.lw = lh;
  c.cout = ci;
  c.taps = taps;
  c.wt = flip;
  c.out = out;
  launch_conv(st, c);
  return out;
}

float* Trainer::gradbuf(const float* act, size_t n, hipStream_t st) {
  auto it = grad_.find(act);
  if (it != grad_.end()) return it->second;
  float* g = ba_.take(n);
  launch_fill(st, g, n, 0.f);
  grad_[act] = g;
  return g;
}

void Trainer::bias_grad(hipStream_t st, const float* dY, size_t M, int C_, float* out) {
  const int nchunk = (int)std::min<size_t>(1024, (M + 255) / 256);
  float* part = ba_.take((size_t)nchunk * C_);
  tr_colsum(st, dY, M, C_, part, nchunk, 1, out);
}

void Trainer::gn_param_grads(hipStream_t st, const float* dgp, const float* dbp, int C_, float* G,
                             const std::string& pre) {
  tr_sum_rows(st, dgp, nb_, C_, 1, grd(G, pre + ".weight"));
  tr_sum_rows(st, dbp, nb_, C_, 1, grd(G, pre + ".bias"));
}

const float* Trainer::res_fwd(hipStream_t st, Node& n) {
  const int lh = n.lh, hw = 1 << (2 * lh);
  const size_t px = (size_t)nb_ * hw;
  n.cin = n.c0 + n.c1;
  n.dense = n.c1 > 0 || n.up0;
  if (n.dense) {
    float* d = fa_.take(px * n.cin);
    tr_dense_in(st, n.s0, n.c0, n.up0, n.s1, n.c1, nb_, lh, lh, d);
    n.in = d;
  } else {
    n.in = n.s0;
  }
  const std::string& p = n.p;
  // noise-level bias of conv1: conv1.bias + Lin_emb(e2)
  n.bias = fa_.take(n.cout);
  launch_gemv(st, prm(p + "emb.weight"), prm(p + "emb.bias"), prm(p + "conv1.bias"), e2_, n.bias, 1, emb, n.cout, 0);
  n.m1 = fa_.take((size_t)nb_ * groups);
  n.r1 = fa_.take((size_t)nb_ * groups);
  gn_stats(st, n.s0, n.c0, n.up0, n.s1, n.c1, lh, n.m1, n.r1, p + "gn1");
  n.A1 = fa_.take(px * n.cin);
  tr_act(st, n.in, gn_scale_, gn_shift_, nb_, hw, n.cin, 2, n.A1);
  layouts(st, p + "conv1.weight", n.cout, n.cin, 9, n.cout);
  n.h1 = conv(st, n.A1, n.cin, lh, n.cout, 9, wl_[p + "conv1.weight"].first, n.bias, nullptr);
  n.m2 = fa_.take((size_t)nb_ * groups);
  n.r2 = fa_.take((size_t)nb_ * groups);
  gn_stats(st, n.h1, n.cout, lh, n.m2, n.r2, p + "gn2");
  n.A2 = fa_.take(px * n.cout);
  tr_act(st, n.h1, gn_scale_, gn_shift_, nb_, hw, n.cout, 2, n.A2);
  const float* skip = n.in;
  if (has(p + "skip.weight")) {
    layouts(st, p + "skip.weight", n.cout, n.cin, 1, n.cout);
    skip = conv(st, n.in, n.cin, lh, n.cout, 1, wl_[p + "skip.weight"].first, prm(p + "skip.bias"), nullptr);
  } else {
    TD_CHECK(n.cin == n.cout && !n.dense, -5, "training: identity skip needs equal channels");
  }
  layouts(st, p + "conv2.weight", n.cout, n.cout, 9, n.cout);
  n.out = conv(st, n.A2, n.cout, lh, n.cout, 9, wl_[p + "conv2.weight"].first, prm(p + "conv2.bias"), skip);
  return n.out;
}

void Trainer::res_bwd(hipStream_t st, Node& n, float* G, float* de2) {
  const int lh = n.lh, hw = 1 << (2 * lh);
  const size_t px = (size_t)nb_ * hw;
  const std::string& p = n.p;
  const float* dY = gradbuf(n.out, px * n.cout, st);
  const int nsplit = (int)std::max<size_t>(1, std::min<size_t>(64, px / 1024));
  float* part = ba_.take((size_t)nsplit * 9 * std::max(n.cin, n.cout) * n.cout);
  // gradient of the (dense) block input
  float* din = ba_.take(px * n.cin);
  if (has(p + "skip.weight")) {
    tr_wgrad(st, n.in, dY, nb_, lh, lh, n.cin, n.cout, 1, part, nsplit, grd(G, p + "skip.weight"));
    bias_grad(st, dY, px, n.cout, grd(G, p + "skip.bias"));
    float* d = dgrad(st, dY, n.cout, lh, n.cin, 1, wl_[p + "skip.weight"].second);
    TD_HIP(hipMemcpyAsync(din, d, px * n.cin * sizeof(float), hipMemcpyDeviceToDevice, st));
  } else {
    TD_HIP(hipMemcpyAsync(din, dY, px * n.cin * sizeof(float), hipMemcpyDeviceToDevice, st));
  }
  // conv2 and GN2 + SiLU
  bias_grad(st, dY, px, n.cout, grd(G, p + "conv2.bias"));
  tr_wgrad(st, n.A2, dY, nb_, lh, lh, n.cout, n.cout, 9, part, nsplit, grd(G, p + "conv2.weight"));
  float* dA2 = dgrad(st, dY, n.cout, lh, n.cout, 9, wl_[p + "conv2.weight"].second);
  float* dh1 = ba_.take(px * n.cout);
  float* dgp = ba_.take((size_t)nb_ * std::max(n.cin, n.cout));
  float* dbp = ba_.take((size_t)nb_ * std::max(n.cin, n.cout));
  tr_gn_bwd(st, n.h1, n.m2, n.r2, prm(p + "gn2.weight"), prm(p + "gn2.bias"), dA2, nb_, hw, n.cout, groups, 2, 0,
            dh1, dgp, dbp);
  gn_param_grads(st, dgp, dbp, n.cout, G, p + "gn2");
  // noise-level bias (conv1.bias + Lin_emb(e2))
  float* db = ba_.take(n.cout);
  const int nchunk = (int)std::min<size_t>(1024, (px + 255) / 256);
  float* cp = ba_.take((size_t)nchunk * n.cout);
  tr_colsum(st, dh1, px, n.cout, cp, nchunk, 0, db);
  tr_emb_bias_bwd(st, db, e2_, prm(p + "emb.weight"), n.cout, emb, grd(G, p + "emb.weight"), grd(G, p + "emb.bias"),
                  grd(G, p + "conv1.bias"), de2);
  // conv1 and GN1 + SiLU
  tr_wgrad(st, n.A1, dh1, nb_, lh, lh, n.cin, n.cout, 9, part, nsplit, grd(G, p + "conv1.weight"));
  float* dA1 = dgrad(st, dh1, n.cout, lh, n.cin, 9, wl_[p + "conv1.weight"].second);
  tr_gn_bwd(st, n.in, n.m1, n.r1, prm(p + "gn1.weight"), prm(p + "gn1.bias"), dA1, nb_, hw, n.cin, groups, 2, 1, din,
            dgp, dbp);
  gn_param_grads(st, dgp, dbp, n.cin, G, p + "gn1");
  // onto the sources
  if (!n.dense) {
    tr_add(st, gradbuf(n.s0, px * n.c0, st), din, px * n.cin);
  } else {
    const size_t n0 = (size_t)nb_ * (hw >> (n.up0 ? 2 : 0)) * n.c0;
    float* g0 = gradbuf(n.s0, n0, st);
    float* g1 = n.c1 ? gradbuf(n.s1, px * n.c1, st) : nullptr;
    tr_split_bwd(st, din, n.c0, n.up0, n.c1, nb_, lh, lh, 1, g0, g1);
  }
}

const float* Trainer::attn_fwd(hipStream_t st, Node& n) {
  const int lh = n.lh, hw = 1 << (2 * lh), c = n.cin;
  const size_t px = (size_t)nb_ * hw;
  const std::string& p = n.p;
  n.m1 = fa_.take((size_t)nb_ * groups);
  n.r1 = fa_.take((size_t)nb_ * groups);
  gn_stats(st, n.in, c, lh, n.m1, n.r1, p + "gn");
  n.A1 = fa_.take(px * c);
  tr_act(st, n.in, gn_scale_, gn_shift_, nb_, hw, c, 1, n.A1);
  layouts(st, p + "qkv.weight", 3 * c, c, 1, 3 * c);
  n.qkv = conv(st, n.A1, c, lh, 3 * c, 1, wl_[p + "qkv.weight"].first, prm(p + "qkv.bias"), nullptr);
  n.O = fa_.take(px * c);
  launch_attention(st, n.qkv, n.O, nb_, hw, c, heads);
  layouts(st, p + "proj.weight", c, c, 1, c);
  n.out = conv(st, n.O, c, lh, c, 1, wl_[p + "proj.weight"].first, prm(p + "proj.bias"), n.in);
  return n.out;
}

void Trainer::attn_bwd(hipStream_t st, Node& n, float* G) {
  const int lh = n.lh, hw = 1 << (2 * lh), c = n.cin;
  const size_t px = (size_t)nb_ * hw;
  const std::string& p = n.p;
  const float* dY = gradbuf(n.out, px * c, st);
  float* dx = gradbuf(n.in, px * c, st);
  tr_add(st, dx, dY, px * c);   // residual
  const int nsplit = (int)std::max<size_t>(1, std::min<size_t>(64, px / 1024));
  float* part = ba_.take((size_t)nsplit * c * 3 * c);
  tr_wgrad(st, n.O, dY, nb_, lh, lh, c, c, 1, part, nsplit, grd(G, p + "proj.weight"));
  bias_grad(st, dY, px, c, grd(G, p + "proj.bias"));
  float* dO = dgrad(st, dY, c, lh, c, 1, wl_[p + "proj.weight"].second);
  float* dqkv = ba_.take(px * 3 * c);
  tr_attention_bwd(st, n.qkv, dO, nb_, hw, c, heads, dqkv);
  tr_wgrad(st, n.A1, dqkv, nb_, lh, lh, c, 3 * c, 1, part, nsplit, grd(G, p + "qkv.weight"));
  bias_grad(st, dqkv, px, 3 * c, grd(G, p + "qkv.bias"));
  float* dA = dgrad(st, dqkv, 3 * c, lh, c, 1, wl_[p + "qkv.weight"].second);
  float* dgp = ba_.take((size_t)nb_ * c);
  float* dbp = ba_.take((size_t)nb_ * c);
  tr_gn_bwd(st, n.in, n.m1, n.r1, prm(p + "gn.weight"), prm(p + "gn.bias"), dA, nb_, hw, c, groups, 1, 1, dx, dgp,
            dbp);
  gn_param_grads(st, dgp, dbp, c, G, p + "gn");
}

void Trainer::forward(hipStream_t st, const float* P, const float* x, int nb, double sigma, float* D) {
  TD_CHECK(nb >= 1, -1, "training: empty batch");
  P_ = P;
  nb_ = nb;
  sigma_ = sigma;
  x_ = x;
  fa_.reset();
  ba_.reset();
  wl_.clear();
  lp_.clear();
  gn_cap_ = 0;
  tape_.clear();
  const int nl = (int)ch.size(), c0 = ch[0], lH = ilog2i(H);
  const double sd = sigma_data, s2 = sigma * sigma + sd * sd;
  const float c_in = (float)(1.0 / std::sqrt(s2));
  // noise embedding e2 for this sigma
  float* cn = fa_.take(1);
  launch_fill(st, cn, 1, (float)(0.25 * std::log(sigma)));
  float* pe = fa_.take(c0);
  float* e1 = fa_.take(emb);
  e2_ = fa_.take(emb);
  launch_pos_emb(st, cn, 1, c0, (float)pe_max_period, pe);
  launch_gemv(st, prm("emb.lin1.weight"), prm("emb.lin1.bias"), nullptr, pe, e1, 1, c0, emb, 1);
  launch_gemv(st, prm("emb.lin2.weight"), prm("emb.lin2.bias"), nullptr, e1, e2_, 1, emb, emb, 1);
  // input conv on c_in x
  if (origins_cap_ < nb) {
    std::vector<int> o(2 * (size_t)nb);
    for (int b = 0; b < nb; ++b) {
      o[2 * b] = 0;
      o[2 * b + 1] = b * H;
    }
    if (origins_) TD_HIP(hipFree(origins_));
    TD_HIP(hipMalloc(&origins_, o.size() * sizeof(int)));
    TD_HIP(hipMemcpy(origins_, o.data(), o.size() * sizeof(int), hipMemcpyHostToDevice));
    origins_cap_ = nb;
  }
  const size_t px0 = (size_t)nb << (2 * lH);
  Ain_ = fa_.take(px0 * C);
  tr_pad_scale(st, x, px0, C, C, c_in, Ain_);
  layouts(st, "conv_in.weight", c0, C, 9, c0);
  float* h0 = fa_.take(px0 * c0);
  launch_conv_in(st, x, H, origins_, nb, H, C, nullptr, 0, c0, c_in, wl_["conv_in.weight"].first, prm("conv_in.bias"),
                 h0);
  Node ni;
  ni.kind = CONV_IN;
  ni.out = h0;
  tape_.push_back(ni);
  const float* h = h0;
  int hc = c0, hl = 0;
  std::vector<std::pair<const float*, int>> skips;
  for (int l = 0; l < nl; ++l) {
    if (l > 0) {
      Node np;
      np.kind = POOL;
      np.lh = lH - l;
      np.cin = hc;
      np.in = h;
      float* o = fa_.take(((size_t)nb << (2 * np.lh)) * hc);
      launch_avgpool(st, h, o, nb, 1 << (np.lh + 1), 1 << (np.lh + 1), hc);
      np.out = o;
      tape_.push_back(np);
      h = o;
    }
    for (int j = 0; j < nres; ++j) {
      Node n;
      n.kind = RES;
      n.p = "enc." + std::to_string(l) + "." + std::to_string(j) + ".";
      n.lvl = l;
      n.lh = lH - l;
      n.s0 = h;
      n.c0 = hc;
      n.cout = ch[l];
      h = res_fwd(st, n);
      tape_.push_back(n);
      hc = ch[l];
      if (attn_at(l)) {
        Node a;
        a.kind = ATTN;
        a.p = n.p + "attn.";
        a.lh = lH - l;
        a.cin = hc;
        a.in = h;
        h = attn_fwd(st, a);
        tape_.push_back(a);
      }
      skips.push_back({h, hc});
    }
  }
  hl = nl - 1;
  {
    Node n;
    n.kind = RES;
    n.p = "mid.0.";
    n.lh = lH - hl;
    n.s0 = h;
    n.c0 = hc;
    n.cout = hc;
    h = res_fwd(st, n);
    tape_.push_back(n);
    if (mid_attn) {
      Node a;
      a.kind = ATTN;
      a.p = "mid.attn.";
      a.lh = lH - hl;
      a.cin = hc;
      a.in = h;
      h = attn_fwd(st, a);
      tape_.push_back(a);
    }
    Node m;
    m.kind = RES;
    m.p = "mid.1.";
    m.lh = lH - hl;
    m.s0 = h;
    m.c0 = hc;
    m.cout = hc;
    h = res_fwd(st, m);
    tape_.push_back(m);
  }
  for (int l = nl - 1; l >= 0; --l) {
    for (int j = 0; j < nres; ++j) {
      Node n;
      n.kind = RES;
      n.p = "dec." + std::to_string(l) + "." + std::to_string(j) + ".";
      n.lvl = l;
      n.lh = lH - l;
      n.s0 = h;
      n.c0 = hc;
      n.up0 = hl != l ? 1 : 0;
      n.s1 = skips.back().first;
      n.c1 = skips.back().second;
      skips.pop_back();
      n.cout = ch[l];
      h = res_fwd(st, n);
      tape_.push_back(n);
      hc = ch[l];
      hl = l;
      if (attn_at(l)) {
        Node a;
        a.kind = ATTN;
        a.p = n.p + "attn.";
        a.lh = lH - l;
        a.cin = hc;
        a.in = h;
        h = attn_fwd(st, a);
        tape_.push_back(a);
      }
    }
  }
  // output: GN + SiLU + 3x3 conv to C channels + EDM preconditioning
  Node no;
  no.kind = OUT;
  no.lh = lH;
  no.cin = hc;
  no.in = h;
  no.m1 = fa_.take((size_t)nb * groups);
  no.r1 = fa_.take((size_t)nb * groups);
  gn_stats(st, h, hc, lH, no.m1, no.r1, "out.gn");
  no.A1 = fa_.take(px0 * hc);
  tr_act(st, h, gn_scale_, gn_shift_, nb, 1 << (2 * lH), hc, 2, no.A1);
  layouts(st, "out.conv.weight", C, hc, 9, 16);
  OutArgs oa{};
  oa.h = h;
  oa.gn_scale = gn_scale_;
  oa.gn_shift = gn_shift_;
  oa.nb = nb;
  oa.H = H;
  oa.c0 = hc;
  oa.cimg = C;
  oa.wt = wl_["out.conv.weight"].first;
  oa.bias = prm("out.conv.bias");
  oa.canvas = x;
  oa.canvas_w = H;
  oa.origins = origins_;
  oa.c_skip = (float)(sd * sd / s2);
  oa.c_out = (float)(sigma * sd / std::sqrt(s2));
  oa.c_euler = 0.f;
  oa.mode = 1;
  oa.dout = D;
  launch_conv_out(st, oa);
  tape_.push_back(no);
}

void Trainer::backward(hipStream_t st, const float* P, const float* dD, float* G) {
  TD_CHECK(!tape_.empty() && P == P_, -6, "training: backward needs the forward of the same parameters");
  ba_.reset();
  grad_.clear();
  const int c0 = ch[0], lH = ilog2i(H);
  const size_t px0 = (size_t)nb_ << (2 * lH);
  const double sd = sigma_data, s2 = sigma_ * sigma_ + sd * sd;
  const float c_out = (float)(sigma_ * sd / std::sqrt(s2));
  float* de2 = ba_.take(emb);
  launch_fill(st, de2, emb, 0.f);
  const int nsplit0 = (int)std::max<size_t>(1, std::min<size_t>(64, px0 / 1024));
  for (int i = (int)tape_.size() - 1; i >= 0; --i) {
    Node& n = tape_[i];
    switch (n.kind) {
      case OUT: {
        // D = c_skip x + c_out (conv(A) + b): dF = c_out dD
        float* dF = ba_.take(px0 * C);
        tr_pad_scale(st, dD, px0, C, C, c_out, dF);
        float* dF16 = ba_.take(px0 * 16);
        tr_pad_scale(st, dD, px0, C, 16, c_out, dF16);
        float* part = ba_.take((size_t)nsplit0 * 9 * n.cin * C);
        tr_wgrad(st, n.A1, dF, nb_, lH, lH, n.cin, C, 9, part, nsplit0, grd(G, "out.conv.weight"));
        bias_grad(st, dF, px0, C, grd(G, "out.conv.bias"));
        float* dA = dgrad(st, dF16, 16, lH, n.cin, 9, wl_["out.conv.weight"].second);
        float* dh = gradbuf(n.in, px0 * n.cin, st);
        float* dgp = ba_.take((size_t)nb_ * n.cin);
        float* dbp = ba_.take((size_t)nb_ * n.cin);
        tr_gn_bwd(st, n.in, n.m1, n.r1, prm("out.gn.weight"), prm("out.gn.bias"), dA, nb_, 1 << (2 * lH), n.cin,
                  groups, 2, 1, dh, dgp, dbp);
        gn_param_grads(st, dgp, dbp, n.cin, G, "out.gn");
        break;
      }
      case ATTN:
        attn_bwd(st, n, G);
        break;
      case RES:
        res_bwd(st, n, G, de2);
        break;
      case POOL: {
        const float* dy = gradbuf(n.out, ((size_t)nb_ << (2 * n.lh)) * n.cin, st);
        float* dx = gradbuf(n.in, ((size_t)nb_ << (2 * (n.lh + 1))) * n.cin, st);
        tr_pool_bwd(st, dy, nb_, n.lh + 1, n.lh + 1, n.cin, 1, dx);
        break;
      }
      case CONV_IN: {
        const float* dh0 = gradbuf(n.out, px0 * c0, st);
        float* part = ba_.take((size_t)nsplit0 * 9 * C * c0);
        tr_wgrad(st, Ain_, dh0, nb_, lH, lH, C, c0, 9, part, nsplit0, grd(G, "conv_in.weight"));
        bias_grad(st, dh0, px0, c0, grd(G, "conv_in.bias"));
        break;
      }
    }
  }
  tr_emb_bwd(st, (float)(0.25 * std::log(sigma_)), c0, emb, (float)pe_max_period, prm("emb.lin1.weight"),
             prm("emb.lin1.bias"), prm("emb.lin2.weight"), prm("emb.lin2.bias"), de2, grd(G, "emb.lin1.weight"),
             grd(G, "emb.lin1.bias"), grd(G, "emb.lin2.weight"), grd(G, "emb.lin2.bias"));
}

}  // namespace td

struct td_trainer {
  int device = 0;
  td::Trainer tr;
  float* part = nullptr;
  size_t part_cap = 0;
  std::string err;
};

namespace {

template <class F>
td_status tguard(td_trainer* t, F&& f) {
  try {
    if (t) t->err.clear();
    f();
    return TD_OK;
  } catch (const td::Error& e) {
    if (t) t->err = e.msg;
    if (e.status == TD_E_NOMEM || e.status == TD_E_DEVICE) (void)hipGetLastError();   // reported once
    return (td_status)e.status;
  } catch (const std::exception& e) {
    if (t) t->err = e.what();
    return TD_E_DEVICE;
  }
}

// NULL is the device's default stream, as in HIP (so that callers whose work
// is on the default stream, torch's included, are ordered with ours).
hipStream_t tstream(td_trainer*, void* s) { return s == TD_STREAM_DEFAULT ? nullptr : (hipStream_t)s; }

}  // namespace

extern "C" {

td_status td_train_create(int hip_device, const char* path, td_trainer** out) {
  if (!out || !path) return TD_E_INVAL;
  *out = nullptr;
  td_trainer* t = new (std::nothrow) td_trainer();
  if (!t) return TD_E_NOMEM;
  td_status s = tguard(t, [&] {
    int n = 0;
    TD_HIP(hipGetDeviceCount(&n));
    TD_CHECK(hip_device >= 0 && hip_device < n, TD_E_INVAL, "no such HIP device");
    t->device = hip_device;
    TD_HIP(hipSetDevice(hip_device));
    t->tr.load(path);
  });
  if (s != TD_OK) {
    td_train_destroy(t);
    return s;
  }
  *out = t;
  return TD_OK;
}

void td_train_destroy(td_trainer* t) {
  if (!t) return;
  (void)hipSetDevice(t->device);
  (void)hipDeviceSynchronize();
  if (t->part) (void)hipFree(t->part);
  delete t;
}

const char* td_train_last_error(const td_trainer* t) { return t ? t->err.c_str() : ""; }

td_status td_train_set_precision(td_trainer* t, int32_t precision) {
  if (!t) return TD_E_INVAL;
  return tguard(t, [&] { t->tr.set_precision(precision); });
}

td_status td_train_param_count(td_trainer* t, size_t* n) {
  if (!t || !n) return TD_E_INVAL;
  *n = t->tr.param_floats();
  return TD_OK;
}

td_status td_train_forward(td_trainer* t, const float* params, const float* x, int32_t n, double sigma, float* D,
                           void* stream) {
  if (!t) return TD_E_INVAL;
  return tguard(t, [&] {
    TD_CHECK(params && x && D && n >= 1 && sigma > 0, TD_E_INVAL, "bad arguments");
    TD_HIP(hipSetDevice(t->device));
    t->tr.forward(tstream(t, stream), params, x, n, sigma, D);
  });
}

td_status td_train_backward(td_trainer* t, const float* params, const float* dD, float* grads, void* stream) {
  if (!t) return TD_E_INVAL;
  return tguard(t, [&] {
    TD_CHECK(params && dD && grads, TD_E_INVAL, "bad arguments");
    TD_HIP(hipSetDevice(t->device));
    t->tr.backward(tstream(t, stream), params, dD, grads);
  });
}

td_status td_train_mse(td_trainer* t, const float* D, const float* y, size_t n, float weight, float* dD,
                       double* loss, void* stream) {
  if (!t) return TD_E_INVAL;
  return tguard(t, [&] {
    TD_CHECK(D && y && dD && n > 0, TD_E_INVAL, "bad arguments");
    TD_HIP(hipSetDevice(t->device));
    hipStream_t st = tstream(t, stream);
    const size_t nblk = (n + 255) / 256;
    if (nblk > t->part_cap) {
      TD_HIP(hipStreamSynchronize(st));
      if (t->part) TD_HIP(hipFree(t->part));
      TD_HIP(hipMalloc(&t->part, nblk * sizeof(float)));
      t->part_cap = nblk;
    }
    td::tr_mse(st, D, y, n, (float)(2.0 * weight / (double)n), dD, t->part);
    if (loss) {
      std::vector<float> h(nblk);
      TD_HIP(hipMemcpyAsync(h.data(), t->part, nblk * sizeof(float), hipMemcpyDeviceToHost, st));
      TD_HIP(hipStreamSynchronize(st));
      double s = 0;
      for (float v : h) s += v;
      *loss = weight * s / (double)n;
    }
  });
}

td_status td_train_adamw(td_trainer* t, float* params, const float* grads, float* m, float* v, size_t n, float lr,
                         float beta1, float beta2, float eps, float weight_decay, int32_t step, void* stream) {
  if (!t) return TD_E_INVAL;
  return tguard(t, [&] {
    TD_CHECK(params && grads && m && v && step >= 1, TD_E_INVAL, "bad arguments");
    TD_HIP(hipSetDevice(t->device));
    td::tr_adamw(tstream(t, stream), params, grads, m, v, n, lr, beta1, beta2, eps, weight_decay, step);
  });
}

}  // extern "C"
