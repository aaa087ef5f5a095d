// Window planning of the lazy sampler: the windows kappa(R) whose extent
// meets a region (the window-range algorithm of the formal appendix, with
// mathematical floor and ceiling on int64).  Host code only, no HIP.
#pragma once

#include <cstdint>

namespace td {

inline int64_t floordiv64(int64_t a, int64_t b) {
  int64_t q = a / b;
  return (q * b > a) ? q - 1 : q;
}
inline int64_t ceildiv64(int64_t a, int64_t b) { return -floordiv64(-a, b); }

struct Region {
  int64_t x0, y0, w, h;
};

struct Kappa {
  bool empty = true;
  int64_t ix0 = 0, ix1 = -1, iy0 = 0, iy1 = -1;
  int64_t nx() const { return ix1 - ix0 + 1; }
  int64_t ny() const { return iy1 - iy0 + 1; }
  int64_t count() const { return empty ? 0 : nx() * ny(); }
};

inline Kappa kappa(const Region& r, int64_t H, int64_t S, int64_t O) {
  Kappa k;
  if (r.w <= 0 || r.h <= 0) return k;
  k.ix0 = ceildiv64(r.x0 - O - H + 1, S);
  k.ix1 = floordiv64(r.x0 + r.w - 1 - O, S);
  k.iy0 = ceildiv64(r.y0 - O - H + 1, S);
  k.iy1 = floordiv64(r.y0 + r.h - 1 - O, S);
  k.empty = k.ix0 > k.ix1 || k.iy0 > k.iy1;
  return k;
}

}  // namespace td
