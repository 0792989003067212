// Philox4x32-10 blocks of rocRAND's engine (an implementation independent of
// the oracle's) for counters and keys read from stdin, one block per line:
// "c0 c1 c2 c3 k0 k1" in hex in, "r0 r1 r2 r3" in hex out.  Host code only;
// built by tests/test_oracle_philox.py as a known-answer check of the
// oracle's Philox4x32-10 (its multipliers and Weyl constants).
#include <cstdio>
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
struct Open : rocrand_device::philox4x32_10_engine {
  static uint4 block(uint4 c, uint2 k) { return Open().ten_rounds(c, k); }
};
int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint4 r = Open::block(uint4{c0, c1, c2, c3}, uint2{k0, k1});
    std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
