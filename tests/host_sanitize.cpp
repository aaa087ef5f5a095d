// Host-only checks of the weight-file parser and the window planner, built
// with AddressSanitizer and UndefinedBehaviorSanitizer by
// test_host_sanitize.py.  No HIP: header.cpp, json.h and plan.h are host
// code.  Modes:
//   kappa N SEED        kappa(R) on N random regions and window layouts
//                       (coordinates up to +-2^31) against the definition:
//                       every window in range meets R, the windows just
//                       outside do not
//   parse FILE...       one line per file: its status (0 = parsed)
//   fuzz FILE N SEED    N mutations of the file's header bytes, each parsed
// Any sanitizer report aborts the process with a non-zero status.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <random>
#include <sstream>
#include <string>

#include "header.h"
#include "plan.h"
#include "td_error.h"

namespace {

std::string read_file(const char* path) {
  std::ifstream f(path, std::ios::binary);
  std::stringstream ss;
  ss << f.rdbuf();
  return ss.str();
}

int parse_status(const std::string& raw) {
  try {
    td::WeightFile wf;
    td::parse_weight_file(raw, "<memory>", &wf);
    return 0;
  } catch (const td::Error& e) {
    return e.status;
  }
}

// Does window ix (origin ix S + O, size H) meet [x0, x0 + w)?
bool meets(int64_t ix, int64_t x0, int64_t w, int64_t H, int64_t S, int64_t O) {
  const int64_t a = ix * S + O;
  return a < x0 + w && a + H > x0;
}

int run_kappa(long n, unsigned seed) {
  std::mt19937_64 rng(seed);
  auto uni = [&](int64_t lo, int64_t hi) { return std::uniform_int_distribution<int64_t>(lo, hi)(rng); };
  const int64_t lim = (1LL << 31) - (1LL << 22);
  long nonempty = 0;
  for (long i = 0; i < n; ++i) {
    const int64_t H = uni(1, 96), S = uni(1, 128), O = uni(-64, 64);
    const int64_t w = uni(1, 1 << 12), h = uni(1, 1 << 12);
    const int64_t x0 = (i & 1) ? uni(-lim + 1, lim - w - 1) : uni(-300, 300);
    const int64_t y0 = (i & 2) ? uni(-lim + 1, lim - h - 1) : uni(-300, 300);
    const td::Kappa k = td::kappa(td::Region{x0, y0, w, h}, H, S, O);
    // the range is exactly the meeting windows: its ends meet, their
    // outer neighbours do not (the windows meeting an interval are a run)
    const bool any_x = meets(td::floordiv64(x0 + w - 1 - O, S), x0, w, H, S, O);
    const bool any_y = meets(td::floordiv64(y0 + h - 1 - O, S), y0, h, H, S, O);
    if (k.empty != !(any_x && any_y)) {
      std::printf("kappa emptiness wrong at case %ld\n", i);
      return 1;
    }
    if (k.empty) continue;
    ++nonempty;
    if (!meets(k.ix0, x0, w, H, S, O) || !meets(k.ix1, x0, w, H, S, O) || meets(k.ix0 - 1, x0, w, H, S, O) ||
        meets(k.ix1 + 1, x0, w, H, S, O) || !meets(k.iy0, y0, h, H, S, O) || !meets(k.iy1, y0, h, H, S, O) ||
        meets(k.iy0 - 1, y0, h, H, S, O) || meets(k.iy1 + 1, y0, h, H, S, O)) {
      std::printf("kappa range wrong at case %ld\n", i);
      return 1;
    }
    if (k.count() <= 0) return 1;
  }
  std::printf("kappa ok %ld (%ld non-empty)\n", n, nonempty);
  return 0;
}

int run_fuzz(const char* path, long n, unsigned seed) {
  const std::string good = read_file(path);
  if (good.size() < 8) return 2;
  uint32_t hl = 0;
  std::memcpy(&hl, good.data() + 4, 4);
  std::mt19937_64 rng(seed);
  auto uni = [&](int64_t lo, int64_t hi) { return std::uniform_int_distribution<int64_t>(lo, hi)(rng); };
  const char* tokens[] = {"1e309", "-1", "0", "1e30", "NaN", "null", "true", "[]", "{}", "\"\"", "9223372036854775807",
                          "-9223372036854775808", "1.5", "[[[[[[", "\"\\u0000\"", "4294967296", "2147483648"};
  long ok = 0, refused = 0;
  for (long i = 0; i < n; ++i) {
    std::string raw = good;
    const int kind = (int)uni(0, 5);
    const size_t pos = 8 + (size_t)uni(0, hl ? hl - 1 : 0);
    if (kind == 0) {                       // flip a header byte
      raw[pos] = (char)(raw[pos] ^ (1 << uni(0, 7)));
    } else if (kind == 1) {                // replace a header byte with a JSON-significant one
      const char c[] = "{}[]\",:-.e0123456789";
      raw[pos] = c[uni(0, sizeof(c) - 2)];
    } else if (kind == 2) {                // overwrite a run with a token (header length kept)
      const char* t = tokens[uni(0, sizeof(tokens) / sizeof(tokens[0]) - 1)];
      for (size_t j = 0; t[j] && pos + j < 8 + (size_t)hl; ++j) raw[pos + j] = t[j];
    } else if (kind == 3) {                // truncate anywhere
      raw.resize((size_t)uni(0, (int64_t)raw.size()));
    } else if (kind == 4) {                // a wrong header length
      const uint32_t v = (uint32_t)uni(0, (int64_t)raw.size() + 64);
      std::memcpy(&raw[4], &v, 4);
    } else {                               // drop a header byte (the rest shifts)
      raw.erase(pos, 1);
    }
    (parse_status(raw) == 0 ? ok : refused)++;
  }
  std::printf("fuzz ok %ld parsed %ld refused %ld\n", n, ok, refused);
  return 0;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc >= 4 && !std::strcmp(argv[1], "kappa")) return run_kappa(std::atol(argv[2]), (unsigned)std::atol(argv[3]));
  if (argc >= 5 && !std::strcmp(argv[1], "fuzz"))
    return run_fuzz(argv[2], std::atol(argv[3]), (unsigned)std::atol(argv[4]));
  if (argc >= 3 && !std::strcmp(argv[1], "parse")) {
    for (int i = 2; i < argc; ++i) std::printf("%d\n", parse_status(read_file(argv[i])));
    return 0;
  }
  std::fprintf(stderr, "usage: host_sanitize kappa N SEED | parse FILE... | fuzz FILE N SEED\n");
  return 2;
}
