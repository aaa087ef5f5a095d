// TDW1 weight-file parsing and validation (host only).
#include "header.h"

#include <cmath>
#include <cstring>

#include "json.h"
#include "td_error.h"

namespace td {

int ilog2(int v) {
  int l = 0;
  while (l < 30 && (1 << l) < v) ++l;
  return (1 << l) == v ? l : -1;
}

namespace {

std::vector<double> edm_sigmas(int K, double smax, double smin, double rho) {
  std::vector<double> s;
  if (K == 1) {
    s = {smax, 0.0};
    return s;
  }
  double a = std::pow(smax, 1.0 / rho), b = std::pow(smin, 1.0 / rho);
  for (int k = 0; k < K; ++k) s.push_back(std::pow(a + (double)k / (K - 1) * (b - a), rho));
  s.push_back(0.0);
  return s;
}

}  // namespace

void parse_weight_file(const std::string& raw, const std::string& path, WeightFile* out) {
  ModelDesc& d = out->d;
  d = ModelDesc{};
  auto& host = out->host;
  auto& shapes = out->shapes;
  host.clear();
  shapes.clear();
  TD_CHECK(raw.size() >= 8 && raw.compare(0, 4, "TDW1") == 0, -5, "not a TDW1 weight file: " + path);
  uint32_t n = 0;
  std::memcpy(&n, raw.data() + 4, 4);
  TD_CHECK((size_t)n + 8 <= raw.size(), -5, "weight file header truncated");
  std::string htxt = raw.substr(8, n);
  Json h = JsonParser(htxt).parse();
  size_t data_start = (8 + (size_t)n + 63) / 64 * 64;

  const Json& dn = h.at("denoiser");
  d.kind = dn.at("kind").str();
  d.C = (int)dn.at("in_channels").integer();
  const Json& sp = h.at("sampler");
  d.K = (int)sp.at("steps").integer();
  d.consistency = sp.has("kind") && sp.at("kind").str() == "consistency";
  if (sp.has("kind"))
    TD_CHECK(d.consistency || sp.at("kind").str() == "edm", -5, "weight header: unknown sampler kind");
  if (d.consistency) {
    const auto& sg = sp.at("sigmas").arr();
    TD_CHECK((int)sg.size() == d.K && d.K >= 1, -5, "weight header: consistency sigmas must number steps");
    d.sched.clear();
    for (const Json& v : sg) d.sched.push_back(v.num());
    for (int k = 0; k < d.K; ++k)
      TD_CHECK(d.sched[k] > 0 && std::isfinite(d.sched[k]) && (k == 0 || d.sched[k] < d.sched[k - 1]), -5,
               "weight header: consistency sigmas must be positive and decreasing");
    d.sched.push_back(0.0);
    d.smax = d.sched[0];
    d.smin = d.sched[d.K - 1];
    d.rho = 1;
    TD_CHECK(!sp.has("blend"), -5, "weight header: consistency sampling blends every step");
  } else {
    d.smax = sp.at("sigma_max").num();
    d.smin = sp.at("sigma_min").num();
    d.rho = sp.at("rho").num();
  }
  d.sigma_data = sp.at("sigma_data").num();
  d.noise_step = 0;
  if (sp.has("noise_step")) {
    const int64_t ns = sp.at("noise_step").integer();
    TD_CHECK(ns >= 0 && ns <= 0xffffffffLL, -5, "weight header: noise_step must be a 32-bit counter word");
    d.noise_step = (uint32_t)ns;
  }
  d.Cc = d.cond_factor = 0;
  if (h.has("cond")) {
    const Json& cj = h.at("cond");
    d.Cc = (int)cj.at("channels").integer();
    d.cond_factor = (int)cj.at("factor").integer();
    TD_CHECK(d.Cc >= 1 && d.Cc <= 4 && d.cond_factor >= 1 && d.cond_factor <= 64, -5,
             "weight header: conditioning needs 1..4 channels and a factor in 1..64");
  }
  const Json& wn = h.at("window");
  d.H = (int)wn.at("size").integer();
  d.S = (int)wn.at("stride").integer();
  d.O = (int)wn.at("offset").integer();
  d.win_eps = wn.at("eps").num();
  const Json& dc = h.at("decode");
  d.factor = (int)dc.at("factor").integer();
  d.sigma_low = dc.at("sigma_low").num();
  d.sigma_res = dc.at("sigma_res").num();
  d.blur_sigma = dc.at("blur_sigma").num();
  d.blur_radius = (int)dc.at("blur_radius").integer();
  TD_CHECK(d.C >= 1 && d.K >= 1 && d.K <= 64 && d.H >= 1 && d.S >= 1 && d.H <= 4096, -5,
           "weight header: bad sampler/window constants");
  TD_CHECK(d.factor == 8 && d.blur_radius >= 0 && d.blur_radius <= 64, -5, "weight header: unsupported decode");
  TD_CHECK(d.smax > d.smin && d.smin > 0 && d.rho > 0 && d.sigma_data > 0, -5, "weight header: bad schedule");
  // comparisons already refuse NaN; infinities are refused here, and the
  // float constants that no comparison above covers get their ranges
  TD_CHECK(std::isfinite(d.smax) && std::isfinite(d.rho) && std::isfinite(d.sigma_data), -5,
           "weight header: schedule constants must be finite");
  TD_CHECK(d.win_eps >= 0 && d.win_eps <= 1, -5, "weight header: window eps must be in [0, 1]");
  TD_CHECK(d.sigma_low > 0 && std::isfinite(d.sigma_low) && d.sigma_res > 0 && std::isfinite(d.sigma_res) &&
               d.blur_sigma > 0 && std::isfinite(d.blur_sigma),
           -5, "weight header: decode scales must be positive and finite");
  if (!d.consistency) d.sched = edm_sigmas(d.K, d.smax, d.smin, d.rho);
  // a re-noised level adds noise to every pixel, which needs every pixel covered
  TD_CHECK(!d.consistency || d.S <= d.H, -5, "weight header: consistency sampling needs stride <= window size");
  d.points.clear();
  if (sp.has("blend")) {
    for (const Json& b : sp.at("blend").arr()) d.points.push_back((int)b.integer());
  } else {
    for (int k = 0; k <= d.K; ++k) d.points.push_back(k);
  }
  TD_CHECK(d.points.size() >= 2 && d.points.front() == 0 && d.points.back() == d.K, -5,
           "weight header: blend points must run from 0 to steps");
  for (size_t i = 1; i < d.points.size(); ++i)
    TD_CHECK(d.points[i] > d.points[i - 1], -5, "weight header: blend points must increase");
  d.T = (int)d.points.size() - 1;

  // tensors
  if (h.has("tensors")) {
    for (const Json& e : h.at("tensors").arr()) {
      std::vector<int> shp;
      size_t cnt = 1;
      for (const Json& x : e.at("shape").arr()) {
        long long v = x.integer();
        TD_CHECK(v >= 1 && v < (1LL << 31), -5, "weight header: bad tensor shape");
        TD_CHECK(cnt <= ((size_t)1 << 32) / (size_t)v, -5, "weight header: tensor too large");
        shp.push_back((int)v);
        cnt *= (size_t)v;
      }
      long long off = e.at("offset").integer();
      TD_CHECK(off >= 0 && data_start + (size_t)off + cnt * 4 <= raw.size(), -5,
               "weight file truncated at tensor " + e.at("name").str());
      std::vector<float> v(cnt);
      std::memcpy(v.data(), raw.data() + data_start + off, cnt * 4);
      host[e.at("name").str()] = std::move(v);
      shapes[e.at("name").str()] = shp;
      d.params += cnt;
    }
  }

  if (d.kind == "linear_gaussian") {
    d.prior_std = dn.at("prior_std").num();
    TD_CHECK(d.prior_std > 0 && std::isfinite(d.prior_std), -5, "weight header: prior_std must be positive");
  } else if (d.kind == "unet") {
    for (const Json& c : dn.at("channels").arr()) d.ch.push_back((int)c.integer());
    d.nres = (int)dn.at("num_res_blocks").integer();
    for (const Json& a : dn.at("attn_levels").arr()) d.attn_levels.push_back((int)a.integer());
    d.mid_attn = dn.at("mid_attn").boolean();
    d.heads = (int)dn.at("num_heads").integer();
    d.groups = (int)dn.at("gn_groups").integer();
    d.gn_eps = (float)dn.at("gn_eps").num();
    d.emb_mult = (int)dn.at("emb_mult").integer();
    d.pe_max_period = dn.at("pe_max_period").num();
    TD_CHECK(!d.ch.empty() && d.nres >= 1 && d.heads >= 1 && d.groups >= 1, -5, "weight header: bad UNet");
    TD_CHECK(d.gn_eps > 0 && std::isfinite(d.gn_eps) && d.pe_max_period > 0 && std::isfinite(d.pe_max_period), -5,
             "weight header: gn_eps and pe_max_period must be positive and finite");
    TD_CHECK(d.ch.size() <= 8 && d.nres <= 16 && d.heads <= 64 && d.groups <= 1024 && d.emb_mult >= 1 &&
                 d.emb_mult <= 16,
             -5, "weight header: UNet sizes out of range");
    for (int c : d.ch) TD_CHECK(c >= 1 && c <= 8192, -5, "weight header: UNet widths must be in [1, 8192]");
    for (int a : d.attn_levels)
      TD_CHECK(a >= 0 && a < (int)d.ch.size(), -5, "weight header: attention level out of range");
    const int lh = ilog2(d.H);
    TD_CHECK(lh >= 4 && (int)d.ch.size() - 1 <= lh, -5,
             "UNet windows must be a power of two >= 16 and divisible by 2^(levels-1)");
  } else {
    throw Error{-5, "unknown denoiser kind: " + d.kind};
  }
}

}  // namespace td
