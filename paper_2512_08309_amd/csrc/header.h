// Weight-file header: the model's constants (ModelDesc) and its tensors,
// read from a TDW1 file image and validated.  Host code only, no HIP: the
// parser also builds on its own for sanitizer checks.
#pragma once

#include <cstddef>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

namespace td {

struct ModelDesc {
  std::string kind;        // "unet" or "linear_gaussian"
  int C = 0;               // latent channels
  // UNet
  std::vector<int> ch;
  int nres = 0;
  std::vector<int> attn_levels;
  bool mid_attn = false;
  int heads = 1, groups = 1, emb_mult = 4;
  float gn_eps = 1e-5f;
  double pe_max_period = 10000.0;
  // analytic denoiser
  double prior_std = 0.5;
  // hierarchy: conditioning channels read from a parent model's final
  // latent, nearest-upsampled by cond_factor (0 channels: unconditioned)
  int Cc = 0, cond_factor = 0;
  uint32_t noise_step = 0;    // counter word of this model's J_T noise
  // sampler: EDM Euler, or few-step consistency sampling (Phi = D, the
  // next level re-noised with G on counter word k + 1 at the blend)
  bool consistency = false;
  int K = 0;
  double smax = 80, smin = 0.002, rho = 7, sigma_data = 0.5;
  std::vector<double> sched;  // sigma_0..sigma_{K-1}, 0
  std::vector<int> points;    // blend points b_0 = 0 < ... < b_T = K (schedule indices)
  int T = 0;                  // blend levels (= K unless truncated)
  // windows
  int H = 0, S = 0, O = 0;
  double win_eps = 0.01;
  // decode
  int factor = 8, blur_radius = 15;
  double sigma_low = 20, sigma_res = 2, blur_sigma = 5;
  size_t params = 0;
  bool attn_at(int l) const {
    for (int a : attn_levels)
      if (a == l) return true;
    return false;
  }
};

// A parsed weight file: constants and FP32 tensors (name -> values, shape).
struct WeightFile {
  ModelDesc d;
  std::map<std::string, std::vector<float>> host;
  std::map<std::string, std::vector<int>> shapes;
};

// Parses and validates a TDW1 file image ("TDW1", u32 header length, JSON
// header, 64-byte aligned FP32 data).  Throws td::Error with TD_E_FORMAT
// (-5) for anything malformed; `path` only names the file in messages.
void parse_weight_file(const std::string& raw, const std::string& path, WeightFile* out);

// log2 of a power of two, else -1.
int ilog2(int v);

}  // namespace td
