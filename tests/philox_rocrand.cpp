// Host-side reference for the oracle's Philox4x32-10: reads lines
// "ctr0 ctr1 ctr2 ctr3 key0 key1" (hex) on stdin and prints the four output
// words of rocRAND's philox4x32_10 engine for each.  Test helper only.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct Engine : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main()
{
    Engine e;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = e.block(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
