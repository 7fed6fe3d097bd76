// Host-only dump of rocRAND's Philox4x32-10 block function, used to pin the
// oracle's own Philox against an independent implementation (a library's
// source header, compiled here for the host; no GPU code is involved).
// Reads lines "c0 c1 c2 c3 k0 k1" (hex) on stdin, prints "o0 o1 o2 o3".
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

struct Exposed : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main()
{
    Exposed e;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 o = e.block(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%08x %08x %08x %08x\n", o.x, o.y, o.z, o.w);
    }
    return 0;
}
