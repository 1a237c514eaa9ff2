// Host-side Philox4x32-10 blocks from rocRAND's implementation, used by the
// CPU tests as an independent reference for the oracle's Philox (the library
// routine, not this project's code).  Reads lines "c0 c1 c2 c3 k0 k1" (hex)
// from stdin and prints "x0 x1 x2 x3" (hex) for each.
#include <cstdio>

#include <rocrand/rocrand_philox4x32_10.h>

struct Exposed : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
    Exposed e;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 c;
        c.x = c0;
        c.y = c1;
        c.z = c2;
        c.w = c3;
        uint2 k;
        k.x = k0;
        k.y = k1;
        const uint4 r = e.block(c, k);
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
