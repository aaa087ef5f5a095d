// Known-answer source for the oracle's Philox4x32-10: rocRAND's own
// host-callable engine (the public rocrand_philox4x32_10.h header), used only
// by tests/test_oracle_noise.py to pin the oracle.  Neither the oracle nor the
// library includes or links this file or rocRAND.
//
// stdin: lines "seed c0 c1 c2 c3" (decimal; c* are 32-bit counter words).
// stdout: the four 32-bit output words of Philox4x32-10 with
// key = (lo32(seed), hi32(seed)) and counter = (c0, c1, c2, c3).
//
// rocRAND seeds its state with key = (lo32, hi32) of the seed and counter
// (offset / 4 as words 0-1, subsequence as words 2-3): a subsequence of
// c2 | c3 << 32 sets words 2-3, and skipping ahead by 4 * (c0 | c1 << 32)
// numbers sets words 0-1.  The skip is taken in pieces of at most 2^61
// blocks so that 4 * piece stays below 2^64; their sum stays below 2^64, so
// nothing carries into words 2-3.
#include <cstdint>
#include <cstdio>

#include <rocrand/rocrand_philox4x32_10.h>

int main() {
  unsigned long long seed, c0, c1, c2, c3;
  while (std::scanf("%llu %llu %llu %llu %llu", &seed, &c0, &c1, &c2, &c3) == 5) {
    rocrand_state_philox4x32_10 st;
    rocrand_init(seed, c2 | (c3 << 32), 0, &st);
    unsigned long long blocks = c0 | (c1 << 32);
    while (blocks != 0) {
      const unsigned long long piece = blocks < (1ull << 61) ? blocks : (1ull << 61);
      skipahead(4ull * piece, &st);
      blocks -= piece;
    }
    const uint4 r = rocrand4(&st);
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
