// Host-side reference for the Philox4x32-10 bijection, taken from rocRAND's
// own implementation (header rocrand/rocrand_philox4x32_10.h).  Test helper
// only: reads lines "c0 c1 c2 c3 k0 k1" (hex) on stdin and prints the four
// output words (hex) of the ten-round bijection for each.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct RocrandPhilox : rocrand_device::philox4x32_10_engine {
    uint4 bijection(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    RocrandPhilox e;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = e.bijection(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
