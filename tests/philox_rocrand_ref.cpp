// Host-side reference for the oracle's Philox4x32-10: reads lines
// "c0 c1 c2 c3 k0 k1" (hex) on stdin and prints rocRAND's ten-round output
// block for each, so the oracle can be compared with an independent
// library implementation.  Built and run on the CPU only.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

struct Engine : rocrand_device::philox4x32_10_engine {
  uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  Engine e;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint4 r = e.block(uint4{c0, c1, c2, c3}, uint2{k0, k1});
    std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
