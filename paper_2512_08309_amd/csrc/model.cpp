// Weight-file parsing, device weight layouts and the batched window
// denoiser D(x; sigma) = c_skip x + c_out F(c_in x; c_noise) (EDM
// preconditioning) with F a GroupNorm/SiLU UNet.  One call runs one
// batched round of Phi evaluations for a level (Parallelization theorem of
// the appendix: all windows of a level are independent).
#include "model.h"

#include <cmath>
#include <cstring>
#include <fstream>
#include <sstream>

#include "json.h"

namespace td {


Model::~Model() {
  for (void* p : allocs_) (void)hipFree(p);
  if (ws_) (void)hipFree(ws_);
}

float* Model::dalloc(size_t n) {
  void* p = nullptr;
  TD_HIP(hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(float)));
  allocs_.push_back(p);
  return (float*)p;
}

const float* Model::upload(const std::vector<float>& v) {
  float* p = dalloc(v.size());
  TD_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(float), hipMemcpyHostToDevice));
  return p;
}

namespace {
// float -> bfloat16, round to nearest even (NaN kept quiet).
uint16_t to_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
}  // namespace

// File layout [co][ci][k][k] -> [co][kp] BF16 with K = tap * ci + c, zero padded.
const uint16_t* Model::upload_lp(const std::vector<float>& w, int co, int ci, int k, int* kp) {
  const int taps = k * k;
  *kp = conv_lp_kp(taps, ci);
  std::vector<uint16_t> r((size_t)co * *kp, 0);
  for (int o = 0; o < co; ++o)
    for (int i = 0; i < ci; ++i)
      for (int t = 0; t < taps; ++t) r[(size_t)o * *kp + t * ci + i] = to_bf16(w[((size_t)o * ci + i) * taps + t]);
  void* p = nullptr;
  TD_HIP(hipMalloc(&p, std::max<size_t>(r.size(), 1) * sizeof(uint16_t)));
  allocs_.push_back(p);
  TD_HIP(hipMemcpy(p, r.data(), r.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
  return (const uint16_t*)p;
}

// File layout [co][ci][k][k] -> fragment order of the halo-staged kernel
// (conv_lp_frag_index, K = k * k * ci), BF16.
const uint16_t* Model::upload_frag(const std::vector<float>& w, int co, int ci, int k) {
  TD_CHECK(ci % 16 == 0 && co % 32 == 0, -5, "fragment-ordered weights need C_in % 16 == 0 and C_out % 32 == 0");
  const int taps = k * k;
  std::vector<uint16_t> r((size_t)co * taps * ci);
  for (int o = 0; o < co; ++o)
    for (int i = 0; i < ci; ++i)
      for (int t = 0; t < taps; ++t)
        r[conv_lp_frag_index(o, t * ci + i, taps * ci)] = to_bf16(w[((size_t)o * ci + i) * taps + t]);
  void* p = nullptr;
  TD_HIP(hipMalloc(&p, r.size() * sizeof(uint16_t)));
  allocs_.push_back(p);
  TD_HIP(hipMemcpy(p, r.data(), r.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
  return (const uint16_t*)p;
}

const uint16_t* Model::upload_frag_cat(const std::vector<float>& w3, const std::vector<float>& w1, int co, int ci) {
  TD_CHECK(ci % 16 == 0 && co % 32 == 0, -5, "fragment-ordered weights need C_in % 16 == 0 and C_out % 32 == 0");
  const int K = 9 * co + ci;
  std::vector<uint16_t> r((size_t)co * K);
  for (int o = 0; o < co; ++o) {
    for (int i = 0; i < co; ++i)
      for (int t = 0; t < 9; ++t) r[conv_lp_frag_index(o, t * co + i, K)] = to_bf16(w3[((size_t)o * co + i) * 9 + t]);
    for (int i = 0; i < ci; ++i) r[conv_lp_frag_index(o, 9 * co + i, K)] = to_bf16(w1[(size_t)o * ci + i]);
  }
  void* p = nullptr;
  TD_HIP(hipMalloc(&p, r.size() * sizeof(uint16_t)));
  allocs_.push_back(p);
  TD_HIP(hipMemcpy(p, r.data(), r.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
  return (const uint16_t*)p;
}

namespace {
// Nearest OCP FP8 e4m3 code (round half to even) of x, |x| <= 448 expected
// (saturates).  Normal: (1 + m/8) 2^(e-7), e = 1..15 (e = 15, m = 7 is NaN);
// subnormal: m 2^-9.
uint8_t to_e4m3(double x) {
  uint8_t sgn = x < 0 ? 0x80 : 0;
  double a = std::fabs(x);
  if (!(a == a)) return 0x7f;
  if (a >= 448.0) return sgn | 0x7e;
  if (a < std::ldexp(1.0, -6)) {                       // subnormal range
    int m = (int)std::nearbyint(a / std::ldexp(1.0, -9));
    return sgn | (uint8_t)(m == 8 ? 0x08 : m);         // m == 8 rounds up to 2^-6
  }
  int e = std::ilogb(a);
  double m = a / std::ldexp(1.0, e) - 1.0;
  int mq = (int)std::nearbyint(m * 8.0);
  if (mq == 8) {
    mq = 0;
    ++e;
  }
  if (e > 8 || (e == 8 && mq > 6)) return sgn | 0x7e;
  return sgn | (uint8_t)(((e + 7) << 3) | mq);
}
}  // namespace

// [co][ci][k][k] -> [co][kp] FP8 e4m3 with scale[o] = max|w[o]| / 448.
const uint8_t* Model::upload_fp8(const std::vector<float>& w, int co, int ci, int k, const float** scale) {
  const int taps = k * k;
  const int kp = conv_lp_kp(taps, ci);
  std::vector<uint8_t> r((size_t)co * kp, 0);
  std::vector<float> sc(co);
  for (int o = 0; o < co; ++o) {
    double mx = 0;
    for (size_t e = 0; e < (size_t)ci * taps; ++e) mx = std::max(mx, (double)std::fabs(w[(size_t)o * ci * taps + e]));
    const double s = mx > 0 ? mx / 448.0 : 1.0;
    sc[o] = (float)s;
    for (int i = 0; i < ci; ++i)
      for (int t = 0; t < taps; ++t) r[(size_t)o * kp + t * ci + i] = to_e4m3(w[((size_t)o * ci + i) * taps + t] / (double)sc[o]);
  }
  void* p = nullptr;
  TD_HIP(hipMalloc(&p, std::max<size_t>(r.size(), 1)));
  allocs_.push_back(p);
  TD_HIP(hipMemcpy(p, r.data(), r.size(), hipMemcpyHostToDevice));
  *scale = upload(sc);
  return (const uint8_t*)p;
}

int Model::cin_max(int l) const {
  const int nl = (int)d.ch.size();
  int c = d.ch[l];
  if (l > 0) c = std::max(c, d.ch[l - 1]);
  int up = l < nl - 1 ? d.ch[l + 1] : d.ch[l];
  c = std::max(c, up + d.ch[l]);
  return c;
}

void Model::set_precision(int p) {
  TD_CHECK(p >= 0 && p <= 2, -1, "precision must be 0 (fp32), 1 (bf16) or 2 (bf16 + fp8 weights)");
  if (p != 0) TD_CHECK(d.kind == "unet", -1, "reduced precision applies to the network denoiser only");
  if ((p != 0) != (prec_ != 0) && ws_) {
    TD_HIP(hipDeviceSynchronize());
    TD_HIP(hipFree(ws_));
    ws_ = nullptr;
    ws_batch_ = 0;
  }
  prec_ = p;
}

void Model::load(const std::string& path, hipStream_t st) {
  std::ifstream f(path, std::ios::binary);
  TD_CHECK(f.good(), -4, "cannot open weight file: " + path);
  std::stringstream ss;
  ss << f.rdbuf();
  WeightFile wf;
  parse_weight_file(ss.str(), path, &wf);
  d = wf.d;

  // window weights w(u) = eps + (1-eps)(1 - |2u-(H-1)|/(H-1))  (Sec. 6 setup)
  std::vector<float> w1(d.H);
  for (int u = 0; u < d.H; ++u) {
    double v = d.H == 1 ? 1.0 : d.win_eps + (1.0 - d.win_eps) * (1.0 - std::fabs(2.0 * u - (d.H - 1)) / (d.H - 1));
    w1[u] = (float)v;
  }
  w1d_ = (float*)upload(w1);
  // decode tables: Gaussian taps and DCT atoms
  {
    int R = d.blur_radius;
    std::vector<double> g(2 * R + 1);
    double s = 0;
    for (int j = -R; j <= R; ++j) s += (g[j + R] = std::exp(-0.5 * (j / d.blur_sigma) * (j / d.blur_sigma)));
    std::vector<float> gf(2 * R + 1);
    for (int j = 0; j <= 2 * R; ++j) gf[j] = (float)(g[j] / s);
    taps_ = (float*)upload(gf);
    const double PI = 3.14159265358979323846;
    double b0 = 1.0 / std::sqrt(8.0);
    std::vector<float> at(3 * 64 + 3);
    for (int y = 0; y < 8; ++y)
      for (int x = 0; x < 8; ++x) {
        double bx = 0.5 * std::cos(PI * (2 * x + 1) / 16.0), by = 0.5 * std::cos(PI * (2 * y + 1) / 16.0);
        at[0 * 64 + y * 8 + x] = (float)(bx * b0);   // atom (1,0): varies along x
        at[1 * 64 + y * 8 + x] = (float)(b0 * by);   // atom (0,1): varies along y
        at[2 * 64 + y * 8 + x] = (float)(bx * by);   // atom (1,1)
      }
    for (int k = 0; k < 3; ++k) {   // block means of the stored (rounded) atoms
      double m = 0;
      for (int e = 0; e < 64; ++e) m += at[k * 64 + e];
      at[3 * 64 + k] = (float)(m / 64.0);
    }
    atoms_ = (float*)upload(at);
  }

  if (d.kind == "unet") build_unet(wf.host, wf.shapes, st);
  TD_HIP(hipStreamSynchronize(st));
}

void Model::build_unet(const std::map<std::string, std::vector<float>>& host,
                       const std::map<std::string, std::vector<int>>& shapes, hipStream_t st) {
  auto get = [&](const std::string& name, std::vector<int> shape) -> const std::vector<float>& {
    auto it = host.find(name);
    TD_CHECK(it != host.end(), -5, "weight file lacks tensor " + name);
    TD_CHECK(shapes.at(name) == shape, -5, "tensor " + name + " has an unexpected shape");
    return it->second;
  };
  // [co][ci][k][k] -> [tap][ci][co]
  auto conv_layout = [&](const std::string& name, int co, int ci, int k) {
    const std::vector<float>& w = get(name, {co, ci, k, k});
    std::vector<float> r((size_t)k * k * ci * co);
    for (int o = 0; o < co; ++o)
      for (int i = 0; i < ci; ++i)
        for (int t = 0; t < k * k; ++t) r[((size_t)t * ci + i) * co + o] = w[((size_t)o * ci + i) * k * k + t];
    return upload(r);
  };
  auto vec = [&](const std::string& name, int n) { return upload(get(name, {n})); };
  auto lp = [&](const std::string& name, int co, int ci, int k, int* kp) {
    return upload_lp(get(name, {co, ci, k, k}), co, ci, k, kp);
  };
  auto f8 = [&](const std::string& name, int co, int ci, int k, const float** sc) {
    return upload_fp8(get(name, {co, ci, k, k}), co, ci, k, sc);
  };

  const int nl = (int)d.ch.size();
  const int c0 = d.ch[0];
  const int emb = d.emb_mult * c0;
  conv_in_w_ = conv_layout("conv_in.weight", c0, d.C + d.Cc, 3);
  conv_in_b_ = vec("conv_in.bias", c0);

  // per-level embedding: pe -> lin1 -> SiLU -> lin2 -> SiLU, for every sigma_k
  std::vector<float> cn(d.K);
  for (int k = 0; k < d.K; ++k) cn[k] = (float)(0.25 * std::log(d.sched[k]));
  const float* d_cn = upload(cn);
  float* pe = dalloc((size_t)d.K * c0);
  float* e1 = dalloc((size_t)d.K * emb);
  float* e2 = dalloc((size_t)d.K * emb);
  launch_pos_emb(st, d_cn, d.K, c0, (float)d.pe_max_period, pe);
  const float* l1w = upload(get("emb.lin1.weight", {emb, c0}));
  const float* l1b = vec("emb.lin1.bias", emb);
  const float* l2w = upload(get("emb.lin2.weight", {emb, emb}));
  const float* l2b = vec("emb.lin2.bias", emb);
  emb_l1w_ = l1w;
  emb_l1b_ = l1b;
  emb_l2w_ = l2w;
  emb_l2b_ = l2b;
  launch_gemv(st, l1w, l1b, nullptr, pe, e1, d.K, c0, emb, 1);
  launch_gemv(st, l2w, l2b, nullptr, e1, e2, d.K, emb, emb, 1);

  std::vector<std::pair<std::string, int>> order;  // (prefix, cout) for bias table
  auto make_rb = [&](const std::string& p, int cin, int cout) {
    ResBlockW w;
    w.cin = cin;
    w.cout = cout;
    w.gn1_g = vec(p + "gn1.weight", cin);
    w.gn1_b = vec(p + "gn1.bias", cin);
    w.w1 = conv_layout(p + "conv1.weight", cout, cin, 3);
    w.gn2_g = vec(p + "gn2.weight", cout);
    w.gn2_b = vec(p + "gn2.bias", cout);
    w.w2 = conv_layout(p + "conv2.weight", cout, cout, 3);
    w.b2 = vec(p + "conv2.bias", cout);
    w.w1_lp = lp(p + "conv1.weight", cout, cin, 3, &w.kp1);
    w.w2_lp = lp(p + "conv2.weight", cout, cout, 3, &w.kp2);
    if (cout % 128 == 0) {
      if (cin % 32 == 0) w.w1_fr = upload_frag(get(p + "conv1.weight", {cout, cin, 3, 3}), cout, cin, 3);
      if (cout % 32 == 0) w.w2_fr = upload_frag(get(p + "conv2.weight", {cout, cout, 3, 3}), cout, cout, 3);
    }
    w.w1_8 = f8(p + "conv1.weight", cout, cin, 3, &w.s1_8);
    w.w2_8 = f8(p + "conv2.weight", cout, cout, 3, &w.s2_8);
    w.has_skip = cin != cout;
    if (w.has_skip) {
      w.wskip = conv_layout(p + "skip.weight", cout, cin, 1);
      w.bskip = vec(p + "skip.bias", cout);
      w.wskip_lp = lp(p + "skip.weight", cout, cin, 1, &w.kps);
      if (cout % 128 == 0 && cin % 32 == 0) {
        w.wskip_fr = upload_frag(get(p + "skip.weight", {cout, cin, 1, 1}), cout, cin, 1);
        w.w2s_fr = upload_frag_cat(get(p + "conv2.weight", {cout, cout, 3, 3}),
                                   get(p + "skip.weight", {cout, cin, 1, 1}), cout, cin);
        std::vector<float> b2 = get(p + "conv2.bias", {cout}), bs = get(p + "skip.bias", {cout});
        for (int o = 0; o < cout; ++o) b2[o] += bs[o];
        w.b2s = upload(b2);
      }
      w.wskip_8 = f8(p + "skip.weight", cout, cin, 1, &w.sskip_8);
    }
    TD_CHECK(cin % d.groups == 0 && cout % d.groups == 0, -5, "GroupNorm groups must divide channels");
    rb_[p] = w;
    order.push_back({p, cout});
  };
  auto make_at = [&](const std::string& p, int C) {
    AttnW w;
    w.C = C;
    w.gn_g = vec(p + "gn.weight", C);
    w.gn_b = vec(p + "gn.bias", C);
    w.wqkv = conv_layout(p + "qkv.weight", 3 * C, C, 1);
    w.bqkv = vec(p + "qkv.bias", 3 * C);
    w.wproj = conv_layout(p + "proj.weight", C, C, 1);
    w.bproj = vec(p + "proj.bias", C);
    w.wqkv_lp = lp(p + "qkv.weight", 3 * C, C, 1, &w.kpq);
    w.wproj_lp = lp(p + "proj.weight", C, C, 1, &w.kpp);
    if (C % 128 == 0) {
      w.wqkv_fr = upload_frag(get(p + "qkv.weight", {3 * C, C, 1, 1}), 3 * C, C, 1);
      w.wproj_fr = upload_frag(get(p + "proj.weight", {C, C, 1, 1}), C, C, 1);
    }
    w.wqkv_8 = f8(p + "qkv.weight", 3 * C, C, 1, &w.sqkv_8);
    w.wproj_8 = f8(p + "proj.weight", C, C, 1, &w.sproj_8);
    at_[p] = w;
  };
  std::vector<int> skipc;
  int c = c0;
  for (int l = 0; l < nl; ++l)
    for (int j = 0; j < d.nres; ++j) {
      std::string p = "enc." + std::to_string(l) + "." + std::to_string(j) + ".";
      make_rb(p, c, d.ch[l]);
      c = d.ch[l];
      if (d.attn_at(l)) make_at(p + "attn.", c);
      skipc.push_back(c);
    }
  make_rb("mid.0.", c, c);
  if (d.mid_attn) make_at("mid.attn.", c);
  make_rb("mid.1.", c, c);
  for (int l = nl - 1; l >= 0; --l)
    for (int j = 0; j < d.nres; ++j) {
      std::string p = "dec." + std::to_string(l) + "." + std::to_string(j) + ".";
      int cs = skipc.back();
      skipc.pop_back();
      make_rb(p, c + cs, d.ch[l]);
      c = d.ch[l];
      if (d.attn_at(l)) make_at(p + "attn.", c);
    }
  out_gn_g_ = vec("out.gn.weight", c);
  out_gn_b_ = vec("out.gn.bias", c);
  out_w_ = conv_layout("out.conv.weight", d.C, c, 3);
  out_b_ = vec("out.conv.bias", d.C);

  // bias_eff[block][k][cout] = conv1.bias + Lin_emb(emb_k), with kExtraSigmas
  // more rows per block for noise levels off the schedule (sigma_slot)
  size_t total = 0;
  for (auto& o : order) total += (size_t)(d.K + kExtraSigmas) * o.second;
  bias_eff_ = dalloc(total);
  size_t off = 0;
  for (auto& o : order) {
    ResBlockW& w = rb_[o.first];
    w.bias_off = off;
    w.emb_w = upload(get(o.first + "emb.weight", {o.second, emb}));
    w.emb_b = vec(o.first + "emb.bias", o.second);
    w.b1 = vec(o.first + "conv1.bias", o.second);
    launch_gemv(st, w.emb_w, w.emb_b, w.b1, e2, bias_eff_ + off, d.K, emb, o.second, 0);
    off += (size_t)(d.K + kExtraSigmas) * o.second;
  }
  emb_scratch_ = dalloc((size_t)c0 + 2 * emb + 1);
}

int Model::sigma_slot(hipStream_t st, double sigma) {
  for (int k = 0; k < d.K; ++k)
    if (d.sched[k] == sigma) return k;
  for (size_t j = 0; j < extra_sigma_.size(); ++j)
    if (extra_sigma_[j] == sigma) return d.K + (int)j;
  TD_CHECK(sigma > 0, -1, "noise level must be positive");
  TD_CHECK(extra_sigma_.size() < (size_t)kExtraSigmas, -1, "too many noise levels off the schedule");
  const int k = d.K + (int)extra_sigma_.size();
  if (d.kind == "unet") {
    const int c0 = d.ch[0], emb = d.emb_mult * c0;
    float* pe = emb_scratch_;
    float* e1 = pe + c0;
    float* e2 = e1 + emb;
    float* cn = e2 + emb;
    const float h = (float)(0.25 * std::log(sigma));
    TD_HIP(hipMemcpyAsync(cn, &h, sizeof(float), hipMemcpyHostToDevice, st));
    launch_pos_emb(st, cn, 1, c0, (float)d.pe_max_period, pe);
    launch_gemv(st, emb_l1w_, emb_l1b_, nullptr, pe, e1, 1, c0, emb, 1);
    launch_gemv(st, emb_l2w_, emb_l2b_, nullptr, e1, e2, 1, emb, emb, 1);
    for (auto& kv : rb_) {
      const ResBlockW& w = kv.second;
      launch_gemv(st, w.emb_w, w.emb_b, w.b1, e2, bias_eff_ + w.bias_off + (size_t)k * w.cout, 1, emb, w.cout, 0);
    }
    TD_HIP(hipStreamSynchronize(st));   // the host value above must stay alive until copied
  }
  extra_sigma_.push_back(sigma);
  return k;
}

double Model::sigma_of(int k) const { return k < d.K ? d.sched[k] : extra_sigma_.at(k - d.K); }

void Model::set_judge(Model* teacher, float threshold, unsigned long long* counter, FallbackFn fallback,
                      void* user) {
  judge_ = teacher;
  judge_thr_ = threshold;
  judge_count_ = counter;
  fallback_ = fallback;
  fallback_user_ = user;
}

size_t Model::workspace_bytes_per_window() const {
  const size_t state = (d.T < d.K ? (size_t)d.H * d.H * d.C * sizeof(float) + 2 * sizeof(int) : 0) +
                       (size_t)d.H * d.H * d.Cc * sizeof(float) +
                       (d.consistency ? 2 * (size_t)d.H * d.H * d.C * sizeof(float) + 7 * sizeof(int) + 5 * 256 : 0);
  if (d.kind != "unet") return state;
  size_t f = 0;
  const int nl = (int)d.ch.size();
  for (int l = 0; l < nl; ++l) {
    size_t r2 = (size_t)(d.H >> l) * (d.H >> l);
    size_t c = d.ch[l];
    f += r2 * c * (4 + d.nres);                   // T R X Y + skips
    if (l > 0) f += r2 * d.ch[l - 1];             // pooled input
    if (d.attn_at(l) || (l == nl - 1 && d.mid_attn)) f += r2 * c * 4;  // qkv + attn out
  }
  f += 2 * 1024;                                  // GN scale/shift
  size_t lp = 0;
  if (prec_)
    for (int l = 0; l < nl; ++l) {
      lp += 2 * (size_t)(d.H >> l) * (d.H >> l) * cin_max(l);   // A, A0 (BF16)
      // per-channel sums of X, Y and the skips: 2 doubles per (slot, channel)
      f += (size_t)(2 + d.nres) * conv_lp_stat_slots(2 * ilog2(d.H >> l)) * d.ch[l] * 4 + 64 * (2 + d.nres);
    }
  else
    for (int l = 0; l < nl; ++l) f += (size_t)(d.H >> l) * (d.H >> l) * cin_max(l);       // F (FP32)
  return state + f * sizeof(float) + lp * sizeof(uint16_t) + (size_t)16 * d.groups * 2 * sizeof(double) + 64 * 256;
}

void Model::ensure_workspace(int max_batch) {
  if (max_batch <= ws_batch_) return;
  if (ws_) {
    TD_HIP(hipDeviceSynchronize());
    TD_HIP(hipFree(ws_));
    ws_ = nullptr;
    ws_batch_ = 0;
  }
  size_t bytes = workspace_bytes_per_window() * (size_t)max_batch + 4096 * 64;
  TD_HIP(hipMalloc(&ws_, bytes));
  char* p = (char*)ws_;
  auto take = [&](size_t nfloat) {
    float* r = (float*)p;
    p += (nfloat * sizeof(float) + 255) / 256 * 256;
    return r;
  };
  state_ = nullptr;
  state_origins_ = nullptr;
  cond_ = d.Cc ? take((size_t)max_batch * d.H * d.H * d.Cc) : nullptr;
  judge_s_ = judge_t_ = nullptr;
  judge_flags_ = judge_pos_ = nullptr;
  if (d.consistency) {
    judge_s_ = take((size_t)max_batch * d.H * d.H * d.C);
    judge_t_ = take((size_t)max_batch * d.H * d.H * d.C);
    judge_flags_ = (int*)take((size_t)max_batch);
    judge_pos_ = (int*)take((size_t)max_batch);
  }
  if (d.T < d.K) {
    state_ = take((size_t)max_batch * d.H * d.H * d.C);
    state_origins_ = (int*)take((size_t)max_batch * 2);
    std::vector<int> o(2 * (size_t)max_batch);
    for (int b = 0; b < max_batch; ++b) {
      o[2 * b] = 0;
      o[2 * b + 1] = b * d.H;
    }
    TD_HIP(hipMemcpy(state_origins_, o.data(), o.size() * sizeof(int), hipMemcpyHostToDevice));
  }
  const int nl = d.kind == "unet" ? (int)d.ch.size() : 0;
  lb_.assign(nl, LevelBufs{});
  chs_.clear();
  for (int l = 0; l < nl; ++l) {
    size_t r2 = (size_t)(d.H >> l) * (d.H >> l) * max_batch;
    size_t c = d.ch[l];
    LevelBufs& b = lb_[l];
    b.T = take(r2 * c);
    b.R = take(r2 * c);
    b.X = take(r2 * c);
    b.Y = take(r2 * c);
    b.S.clear();
    for (int j = 0; j < d.nres; ++j) b.S.push_back(take(r2 * c));
    b.P = l > 0 ? take(r2 * d.ch[l - 1]) : nullptr;
    if (d.attn_at(l) || (l == nl - 1 && d.mid_attn)) {
      b.Q = take(r2 * 3 * c);
      b.O = take(r2 * c);
    } else {
      b.Q = b.O = nullptr;
    }
    b.A = b.A0 = nullptr;
    b.F = nullptr;
    if (prec_) {
      b.A = (uint16_t*)take((r2 * cin_max(l) + 1) / 2);
      b.A0 = (uint16_t*)take((r2 * cin_max(l) + 1) / 2);
      const int slots = conv_lp_stat_slots(2 * ilog2(d.H >> l));
      std::vector<const float*> tracked = {b.X, b.Y};
      for (float* sk : b.S) tracked.push_back(sk);
      for (const float* t : tracked) {
        ChStats cs;
        cs.buf = (double*)take((size_t)max_batch * slots * c * 4);
        cs.slots = slots;
        chs_[t] = cs;
      }
    } else {
      b.F = take(r2 * cin_max(l));
    }
  }
  if (d.kind == "unet") {
    gn_scale_ = take((size_t)max_batch * 1024);
    gn_shift_ = take((size_t)max_batch * 1024);
    gn_part_ = (double*)take((size_t)max_batch * 16 * d.groups * 2 * 2);
  }
  TD_CHECK((size_t)(p - (char*)ws_) <= bytes, -2, "workspace layout overflow");
  ws_batch_ = max_batch;
}

void Model::gn(hipStream_t st, const float* s0, int c0, int up0, const float* s1, int c1, int nb, int lh, int lw,
               const float* g, const float* b) {
  GnArgs a;
  a.src0 = s0;
  a.src1 = s1;
  a.c0 = c0;
  a.c1 = c1;
  a.up0 = up0;
  a.nb = nb;
  a.lh = lh;
  a.lw = lw;
  a.groups = d.groups;
  a.eps = d.gn_eps;
  a.gamma = g;
  a.beta = b;
  a.partial = gn_part_;
  a.scale = gn_scale_;
  a.shift = gn_shift_;
  launch_gn(st, a);
}

Model::ChStats* Model::chstats_of(const float* t) {
  auto it = chs_.find(t);
  return it == chs_.end() ? nullptr : &it->second;
}

void Model::gn_stats(hipStream_t st, const float* s0, int c0, int up0, const float* s1, int c1, int nb, int lh,
                     int lw, const float* g, const float* b) {
  const ChStats* a0 = chstats_of(s0);
  const ChStats* a1 = s1 ? chstats_of(s1) : nullptr;
  const bool have = a0 && a0->valid && a0->C == c0 && (!s1 || (a1 && a1->valid && a1->C == c1));
  if (!have) {
    gn(st, s0, c0, up0, s1, c1, nb, lh, lw, g, b);
    return;
  }
  GnArgs a{};
  a.c0 = c0;
  a.c1 = c1;
  a.up0 = up0;
  a.nb = nb;
  a.lh = lh;
  a.lw = lw;
  a.groups = d.groups;
  a.eps = d.gn_eps;
  a.gamma = g;
  a.beta = b;
  a.scale = gn_scale_;
  a.shift = gn_shift_;
  launch_gn_finalize_ch(st, a, a0->buf, a0->slots, s1 ? a1->buf : nullptr, s1 ? a1->slots : 0);
}

// GroupNorm of a conv input followed by its apply (act 1 affine, 2 + SiLU),
// written as BF16 (out) or FP32 (out32): one pass per window when the
// window's input fits in a workgroup, else statistics, then apply.
void Model::gn_apply(hipStream_t st, const float* s0, int c0, int up0, const float* s1, int c1, int nb, int lr,
                     const float* g, const float* b, int act, uint16_t* out, float* out32) {
  if (gn_apply_window_fits(lr, lr, c0, c1, up0, d.groups)) {
    GnArgs a{};
    a.src0 = s0;
    a.src1 = s1;
    a.c0 = c0;
    a.c1 = c1;
    a.up0 = up0;
    a.nb = nb;
    a.lh = lr;
    a.lw = lr;
    a.groups = d.groups;
    a.eps = d.gn_eps;
    a.gamma = g;
    a.beta = b;
    launch_gn_apply_window(st, a, act, out, out32);
    return;
  }
  gn_stats(st, s0, c0, up0, s1, c1, nb, lr, lr, g, b);
  apply(st, s0, c0, up0, s1, c1, act, nb, lr, out, out32);
}

void Model::conv_lp(hipStream_t st, const uint16_t* act, int cin, int nb, int lr, int cout, int taps,
                    const uint16_t* wt, const uint8_t* w8, const float* w8s, int kp, const float* bias,
                    const float* res, float* out, const uint16_t* wfrag, bool track, const float* act_scale,
                    const float* act_shift) {
  ConvLpArgs a{};
  a.act_scale = act_scale;
  a.act_shift = act_shift;
  if (prec_ == 2) {
    a.wt = w8;
    a.w8 = 1;
    a.wscale = w8s;
  } else {
    a.wt = wt;
    a.wfrag = wfrag;
  }
  a.act = act;
  a.cin = cin;
  a.nb = nb;
  a.lh = lr;
  a.lw = lr;
  a.cout = cout;
  a.taps = taps;
  a.kp = kp;
  a.bias = bias;
  a.res = res;
  a.out = out;
  ChStats* cs = track ? chstats_of(out) : nullptr;
  if (cs) {
    a.chstats = cs->buf;
    if (!conv_lp_fused_ok(a) || conv_lp_stat_slots(2 * lr) != cs->slots) a.chstats = nullptr;
  }
  launch_conv_lp(st, a);
  if (cs) {
    cs->valid = a.chstats != nullptr;
    cs->C = cout;
  }
}

bool Model::conv1_fused(hipStream_t st, const ResBlockW& w, const uint16_t* act, int nb, int lr, const float* bias,
                        uint16_t* out16) {
  if (prec_ != 1 || !w.w1_fr) return false;
  ConvLpArgs a{};
  a.act = act;
  a.cin = w.cin;
  a.nb = nb;
  a.lh = lr;
  a.lw = lr;
  a.cout = w.cout;
  a.taps = 9;
  a.kp = w.kp1;
  a.wt = w.w1_lp;
  a.wfrag = w.w1_fr;
  a.bias = bias;
  a.out16 = out16;
  a.stats = gn_part_;
  a.groups = d.groups;
  if (!conv_lp_fused_ok(a)) return false;
  launch_conv_lp(st, a);
  GnArgs g{};
  g.c0 = w.cout;
  g.nb = nb;
  g.lh = lr;
  g.lw = lr;
  g.groups = d.groups;
  g.eps = d.gn_eps;
  g.gamma = w.gn2_g;
  g.beta = w.gn2_b;
  g.partial = gn_part_;
  g.scale = gn_scale_;
  g.shift = gn_shift_;
  launch_gn_finalize(st, g, conv_lp_stat_slots(2 * lr));
  return true;
}

bool Model::conv2_act_ok(const ResBlockW& w, int nb, int lr) const {
  if (prec_ != 1 || !w.w2_fr || w.has_skip) return false;
  ConvLpArgs a{};   // the shape of the launch (conv_lp_fused_ok reads no data pointer but these)
  a.cin = w.cout;
  a.nb = nb;
  a.lh = lr;
  a.lw = lr;
  a.cout = w.cout;
  a.taps = 9;
  a.wfrag = w.w2_fr;
  a.act_scale = gn_scale_;
  a.act_shift = gn_shift_;
  return conv_lp_fused_ok(a);
}

bool Model::conv2_skip_fused(hipStream_t st, const ResBlockW& w, const uint16_t* act, const uint16_t* act2, int nb,
                             int lr, float* out) {
  if (prec_ != 1 || !w.w2s_fr) return false;
  ConvLpArgs a{};
  a.act = act;
  a.cin = w.cout;
  a.act2 = act2;
  a.cin2 = w.cin;
  a.nb = nb;
  a.lh = lr;
  a.lw = lr;
  a.cout = w.cout;
  a.taps = 9;
  a.kp = conv_lp_kp(9, w.cout);
  a.wt = w.w2_lp;
  a.wfrag = w.w2s_fr;
  a.bias = w.b2s;
  a.out = out;
  if (!conv_lp_fused_ok(a)) return false;
  ChStats* cs = chstats_of(out);
  if (cs) {
    a.chstats = cs->buf;
    if (!conv_lp_fused_ok(a) || conv_lp_stat_slots(2 * lr) != cs->slots) a.chstats = nullptr;
  }
  launch_conv_lp(st, a);
  if (cs) {
    cs->valid = a.chstats != nullptr;
    cs->C = w.cout;
  }
  return true;
}

void Model::apply(hipStream_t st, const float* s0, int c0, int up0, const float* s1, int c1, int act, int nb, int lr,
                  uint16_t* out, float* out32, uint16_t* raw) {
  ApplyArgs a{};
  a.src0 = s0;
  a.src1 = s1;
  a.c0 = c0;
  a.c1 = c1;
  a.up0 = up0;
  a.scale = gn_scale_;
  a.shift = gn_shift_;
  a.act = act;
  a.nb = nb;
  a.lh = lr;
  a.lw = lr;
  a.out = out;
  a.out32 = out32;
  a.raw = raw;
  launch_apply(st, a);
}

// 3x3 convolution of an already activated dense FP32 input
void Model::conv3_f32(hipStream_t st, const float* in, int cin, int nb, int lr, int cout, const float* wt,
                      const float* bias, const float* res, float* out, double* stats) {
  ConvArgs a{};
  a.stats = stats;
  a.groups = d.groups;
  a.src0 = in;
  a.c0 = cin;
  a.nb = nb;
  a.lh = lr;
  a.lw = lr;
  a.cout = cout;
  a.taps = 9;
  a.wt = wt;
  a.bias = bias;
  a.res = res;
  a.out = out;
  launch_conv(st, a);
}

void Model::resblock(hipStream_t st, const ResBlockW& w, int k, const float* s0, int c0, int up0, const float* s1,
                     int c1, int nb, int lvl, float* out) {
  const int lr = ilog2(d.H >> lvl);
  LevelBufs& B = lb_[lvl];
  TD_CHECK(c0 + c1 == w.cin, -5, "resblock: channel mismatch");
  if (prec_) {
    const float* bias1 = bias_eff_ + w.bias_off + (size_t)k * w.cout;
    // with a 1x1 skip, the statistics pass's apply also writes the skip
    // conv's BF16 operand from the same read of the input
    const bool raw_in_apply = w.has_skip && !gn_apply_window_fits(lr, lr, c0, c1, up0, d.groups);
    if (raw_in_apply) {
      gn_stats(st, s0, c0, up0, s1, c1, nb, lr, lr, w.gn1_g, w.gn1_b);
      apply(st, s0, c0, up0, s1, c1, 2, nb, lr, B.A, nullptr, B.A0);
    } else {
      gn_apply(st, s0, c0, up0, s1, c1, nb, lr, w.gn1_g, w.gn1_b, 2, B.A, nullptr);
    }
    // conv1's output goes to GroupNorm 2 only: stored as BF16 with its
    // statistics from the epilogue where the halo-staged kernel applies
    uint16_t* T16 = reinterpret_cast<uint16_t*>(B.T);
    const bool fused = conv1_fused(st, w, B.A, nb, lr, bias1, T16);
    if (!fused) conv_lp(st, B.A, w.cin, nb, lr, w.cout, 9, w.w1_lp, w.w1_8, w.s1_8, w.kp1, bias1, nullptr, B.T, w.w1_fr);
    const float* res = s0;
    if (w.has_skip) {
      if (!raw_in_apply) apply(st, s0, c0, up0, s1, c1, 0, nb, lr, B.A0);
    } else {
      TD_CHECK(c1 == 0 && !up0, -5, "identity skip needs a plain input");
    }
    // GroupNorm 2 + SiLU: staged by conv2 itself where the halo-staged kernel
    // allows (an identity skip, windows of side 32 or 64), else a pass into B.A
    const bool act_staged = fused && conv2_act_ok(w, nb, lr);
    if (act_staged) {
      conv_lp(st, T16, w.cout, nb, lr, w.cout, 9, w.w2_lp, w.w2_8, w.s2_8, w.kp2, w.b2, res, out, w.w2_fr, true,
              gn_scale_, gn_shift_);
      return;
    }
    if (fused) launch_apply_bf16(st, T16, w.cout, gn_scale_, gn_shift_, 2, nb, lr, lr, B.A);
    else gn_apply(st, B.T, w.cout, 0, nullptr, 0, nb, lr, w.gn2_g, w.gn2_b, 2, B.A, nullptr);
    // with a 1x1 skip: conv2 and the skip projection in one launch where the
    // halo-staged kernel applies (no skip output and no residual read)
    if (w.has_skip && conv2_skip_fused(st, w, B.A, B.A0, nb, lr, out)) return;
    if (w.has_skip) {
      conv_lp(st, B.A0, w.cin, nb, lr, w.cout, 1, w.wskip_lp, w.wskip_8, w.sskip_8, w.kps, w.bskip, nullptr, B.R,
              w.wskip_fr);
      res = B.R;
    }
    conv_lp(st, B.A, w.cout, nb, lr, w.cout, 9, w.w2_lp, w.w2_8, w.s2_8, w.kp2, w.b2, res, out, w.w2_fr, true);
    return;
  }
  // FP32: GroupNorm + SiLU are applied once per input element into F, not
  // once per tap inside the 3x3 conv's staging
  gn_apply(st, s0, c0, up0, s1, c1, nb, lr, w.gn1_g, w.gn1_b, 2, nullptr, B.F);
  // conv1's output feeds GroupNorm 2 only: its statistics come from the
  // conv's epilogue where the shape allows (C_out % 128 == 0)
  const bool fused = w.cout % 128 == 0 && w.cout % d.groups == 0 && 2 * lr >= 6 && w.cin <= kConvDenseMaxCin;
  conv3_f32(st, B.F, w.cin, nb, lr, w.cout, w.w1, bias_eff_ + w.bias_off + (size_t)k * w.cout, nullptr, B.T,
            fused ? gn_part_ : nullptr);
  const float* res = s0;
  if (w.has_skip) {
    ConvArgs s{};
    s.src0 = s0;
    s.src1 = s1;
    s.c0 = c0;
    s.c1 = c1;
    s.up0 = up0;
    s.nb = nb;
    s.lh = lr;
    s.lw = lr;
    s.cout = w.cout;
    s.taps = 1;
    s.wt = w.wskip;
    s.bias = w.bskip;
    s.out = B.R;
    launch_conv(st, s);
    res = B.R;
  } else {
    TD_CHECK(c1 == 0 && !up0, -5, "identity skip needs a plain input");
  }
  if (fused) {
    GnArgs g{};
    g.c0 = w.cout;
    g.nb = nb;
    g.lh = lr;
    g.lw = lr;
    g.groups = d.groups;
    g.eps = d.gn_eps;
    g.gamma = w.gn2_g;
    g.beta = w.gn2_b;
    g.partial = gn_part_;
    g.scale = gn_scale_;
    g.shift = gn_shift_;
    launch_gn_finalize(st, g, conv_stat_slots(2 * lr));
    apply(st, B.T, w.cout, 0, nullptr, 0, 2, nb, lr, nullptr, B.F);
  } else {
    gn_apply(st, B.T, w.cout, 0, nullptr, 0, nb, lr, w.gn2_g, w.gn2_b, 2, nullptr, B.F);
  }
  conv3_f32(st, B.F, w.cout, nb, lr, w.cout, w.w2, w.b2, res, out);
}

void Model::attention(hipStream_t st, const AttnW& w, const float* in, int nb, int lvl, float* out) {
  const int lr = ilog2(d.H >> lvl);
  LevelBufs& B = lb_[lvl];
  if (prec_) {
    gn_apply(st, in, w.C, 0, nullptr, 0, nb, lr, w.gn_g, w.gn_b, 1, B.A, nullptr);
    conv_lp(st, B.A, w.C, nb, lr, 3 * w.C, 1, w.wqkv_lp, w.wqkv_8, w.sqkv_8, w.kpq, w.bqkv, nullptr, B.Q, w.wqkv_fr);
    launch_attention(st, B.Q, B.O, nb, 1 << (2 * lr), w.C, d.heads);
    apply(st, B.O, w.C, 0, nullptr, 0, 0, nb, lr, B.A);
    conv_lp(st, B.A, w.C, nb, lr, w.C, 1, w.wproj_lp, w.wproj_8, w.sproj_8, w.kpp, w.bproj, in, out, w.wproj_fr,
            true);
    return;
  }
  gn(st, in, w.C, 0, nullptr, 0, nb, lr, lr, w.gn_g, w.gn_b);
  ConvArgs q{};
  q.src0 = in;
  q.c0 = w.C;
  q.gn_scale = gn_scale_;
  q.gn_shift = gn_shift_;
  q.act = 1;
  q.nb = nb;
  q.lh = lr;
  q.lw = lr;
  q.cout = 3 * w.C;
  q.taps = 1;
  q.wt = w.wqkv;
  q.bias = w.bqkv;
  q.out = B.Q;
  launch_conv(st, q);
  launch_attention(st, B.Q, B.O, nb, 1 << (2 * lr), w.C, d.heads);
  ConvArgs p{};
  p.src0 = B.O;
  p.c0 = w.C;
  p.nb = nb;
  p.lh = lr;
  p.lw = lr;
  p.cout = w.C;
  p.taps = 1;
  p.wt = w.wproj;
  p.bias = w.bproj;
  p.res = in;
  p.out = out;
  launch_conv(st, p);
}

void Model::run_level(hipStream_t st, const WindowBatch& wb, int t) {
  TD_CHECK(t >= 0 && t < d.T, -1, "blend level out of range");
  const int k0 = d.points[d.T - t - 1], k1 = d.points[d.T - t];
  if (k1 - k0 == 1) {
    run_batch(st, wb, k0);
    return;
  }
  TD_CHECK(state_ && wb.n <= ws_batch_, -1, "window state buffer missing");
  for (int k = k0; k < k1; ++k) {
    WindowBatch s = wb;
    if (k > k0) {   // later steps read the window state of the previous step
      s.canvas = state_;
      s.canvas_w = d.H;
      s.d_origins = state_origins_;
    }
    if (k + 1 < k1) {
      s.mode = 2;
      s.dout = state_;
    }
    run_batch(st, s, k);
  }
}

void Model::run_batch(hipStream_t st, const WindowBatch& wb, int k) {
  TD_CHECK(k >= 0 && k < d.K + (int)extra_sigma_.size(), -1, "sigma index out of range");
  TD_CHECK(k < d.K || wb.mode == 1, -1, "off-schedule noise levels give raw estimates only");
  if (judge_ && d.consistency && wb.mode == 0) {
    // student and teacher estimates side by side, then the per-window choice
    TD_CHECK(wb.n <= ws_batch_, -1, "batch larger than workspace");
    WindowBatch s = wb;
    s.mode = 1;
    s.dout = judge_s_;
    run_net(st, s, k);
    WindowBatch t = wb;
    t.mode = 1;
    t.dout = judge_t_;
    if (judge_->d.Cc != d.Cc) t.cond = nullptr;
    judge_->ensure_workspace(std::max(judge_->max_batch(), wb.n));
    judge_->run_batch(st, t, judge_->sigma_slot(st, d.sched[k]));
    launch_judge(st, judge_s_, judge_t_, wb.n, d.H, d.C, judge_thr_, judge_flags_, judge_count_);
    // a flagged window takes the teacher's plain sample J_0 on its region
    std::vector<int> flags(wb.n), pos(wb.n, -1);
    std::vector<FallbackReq> req;
    TD_HIP(hipMemcpyAsync(flags.data(), judge_flags_, (size_t)wb.n * sizeof(int), hipMemcpyDeviceToHost, st));
    TD_HIP(hipStreamSynchronize(st));
    for (int b = 0; b < wb.n; ++b)
      if (flags[b]) {
        TD_CHECK(wb.h_widx, -6, "internal: judged batch without host window indices");
        pos[b] = (int)req.size();
        req.push_back(FallbackReq{wb.h_seeds ? wb.h_seeds[b] : wb.seed, wb.h_widx[2 * b], wb.h_widx[2 * b + 1]});
      }
    TD_HIP(hipMemcpy(judge_pos_, pos.data(), pos.size() * sizeof(int), hipMemcpyHostToDevice));
    if (!req.empty()) {
      TD_CHECK(fallback_, -6, "internal: judged model without a fallback sampler");
      fallback_(fallback_user_, req.data(), (int)req.size(), judge_t_, st);
    }
    launch_select(st, judge_s_, judge_t_, judge_pos_, wb.n, d.H, d.C, w1d_, wb.d_slots);
    return;
  }
  run_net(st, wb, k);
}

void Model::run_net(hipStream_t st, const WindowBatch& wb, int k, double sigma_next_override) {
  const double sigma = sigma_of(k);
  const double sigma_next = sigma_next_override >= 0 ? sigma_next_override : (k < d.K ? d.sched[k + 1] : 0.0);
  const double sd = d.sigma_data;
  const double s2 = sigma * sigma + sd * sd;
  const float c_skip = (float)(sd * sd / s2), c_out = (float)(sigma * sd / std::sqrt(s2));
  const float c_in = (float)(1.0 / std::sqrt(s2)), c_euler = (float)((sigma_next - sigma) / sigma);
  const int direct = d.consistency ? 1 : 0;   // Phi = D (re-noising happens at the blend)
  WinGeom g{d.H, d.S, d.C};
  TD_CHECK(d.Cc == 0 || wb.cond, -6, "conditioned model run without its conditioning windows");
  if (d.kind == "linear_gaussian") {
    launch_lg_step(st, g, wb.canvas, wb.canvas_w, wb.d_origins, wb.d_widx, wb.cond, d.Cc, wb.n, d.prior_std,
                   sigma, c_euler, direct, w1d_, wb.d_slots, wb.mode, wb.dout);
    return;
  }
  TD_CHECK(wb.n <= ws_batch_, -1, "batch larger than workspace");
  const int nl = (int)d.ch.size();
  for (auto& kv : chs_) kv.second.valid = false;   // no buffer holds this run's tensors yet
  // (mode 2 writes Phi into dout; the output kernel reads x at the same
  //  element before writing it, so dout may alias the canvas)
  const int nb = wb.n;
  LevelBufs& L0 = lb_[0];
  launch_conv_in(st, wb.canvas, wb.canvas_w, wb.d_origins, nb, d.H, d.C, wb.cond, d.Cc, d.ch[0], c_in, conv_in_w_,
                 conv_in_b_, L0.X);
  const float* h = L0.X;
  int hc = d.ch[0];
  for (int l = 0; l < nl; ++l) {
    LevelBufs& B = lb_[l];
    if (l > 0) {
      int r = d.H >> (l - 1);
      launch_avgpool(st, h, B.P, nb, r, r, hc);
      h = B.P;
    }
    for (int j = 0; j < d.nres; ++j) {
      std::string p = "enc." + std::to_string(l) + "." + std::to_string(j) + ".";
      const ResBlockW& w = rb_.at(p);
      if (d.attn_at(l)) {
        resblock(st, w, k, h, hc, 0, nullptr, 0, nb, l, B.X);
        attention(st, at_.at(p + "attn."), B.X, nb, l, B.S[j]);
      } else {
        resblock(st, w, k, h, hc, 0, nullptr, 0, nb, l, B.S[j]);
      }
      h = B.S[j];
      hc = w.cout;
    }
  }
  {
    LevelBufs& B = lb_[nl - 1];
    resblock(st, rb_.at("mid.0."), k, h, hc, 0, nullptr, 0, nb, nl - 1, B.X);
    const float* m = B.X;
    if (d.mid_attn) {
      attention(st, at_.at("mid.attn."), B.X, nb, nl - 1, B.Y);
      m = B.Y;
    }
    float* o = (m == B.X) ? B.Y : B.X;
    resblock(st, rb_.at("mid.1."), k, m, hc, 0, nullptr, 0, nb, nl - 1, o);
    h = o;
  }
  int hl = nl - 1;  // level h lives at
  for (int l = nl - 1; l >= 0; --l) {
    LevelBufs& B = lb_[l];
    for (int j = 0; j < d.nres; ++j) {
      std::string p = "dec." + std::to_string(l) + "." + std::to_string(j) + ".";
      const ResBlockW& w = rb_.at(p);
      const float* skip = B.S[d.nres - 1 - j];
      int up0 = hl != l ? 1 : 0;
      float* o = (h == B.X) ? B.Y : B.X;
      if (d.attn_at(l)) {
        float* tmp = (o == B.X) ? B.Y : B.X;
        // attention input must not alias its output: resblock -> o, attention o -> tmp
        resblock(st, w, k, h, hc, up0, skip, w.cin - hc, nb, l, o);
        attention(st, at_.at(p + "attn."), o, nb, l, tmp);
        h = tmp;
      } else {
        resblock(st, w, k, h, hc, up0, skip, w.cin - hc, nb, l, o);
        h = o;
      }
      hc = w.cout;
      hl = l;
    }
  }
  gn_stats(st, h, hc, 0, nullptr, 0, nb, ilog2(d.H), ilog2(d.H), out_gn_g_, out_gn_b_);
  OutArgs oa{};
  oa.h = h;
  oa.gn_scale = gn_scale_;
  oa.gn_shift = gn_shift_;
  oa.nb = nb;
  oa.H = d.H;
  oa.c0 = hc;
  oa.cimg = d.C;
  oa.wt = out_w_;
  oa.bias = out_b_;
  oa.canvas = wb.canvas;
  oa.canvas_w = wb.canvas_w;
  oa.origins = wb.d_origins;
  oa.c_skip = c_skip;
  oa.c_out = c_out;
  oa.c_euler = c_euler;
  oa.direct = direct;
  oa.w1d = w1d_;
  oa.slots = wb.d_slots;
  oa.mode = wb.mode;
  oa.dout = wb.dout;
  launch_conv_out(st, oa);
}

}  // namespace td
