// Independent Philox4x32-10 implementation for cross-checking the oracle:
// rocRAND's engine, called on the host through its ten-round block function.
// Reads "c0 c1 c2 c3 k0 k1" lines (hex) on stdin, prints the 4 output words.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

struct probe : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
    probe p;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 o = p.block(make_uint4(c0, c1, c2, c3), make_uint2(k0, k1));
        std::printf("%08x %08x %08x %08x\n", o.x, o.y, o.z, o.w);
    }
    return 0;
}
