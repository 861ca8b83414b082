// Test helper: evaluates the Philox4x32-10 bijection through rocRAND's own,
// independently written engine, so that the oracle's generator is checked
// against a second implementation.  Reads lines "c0 c1 c2 c3 k0 k1" (hex) on
// stdin and prints the four output words.  Host code only.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

namespace {
struct Bijection : rocrand_device::philox4x32_10_engine {
    uint4 apply(uint4 counter, uint2 key) { return ten_rounds(counter, key); }
};
}  // namespace

int main() {
    Bijection engine;
    unsigned v[6];
    while (std::scanf("%x %x %x %x %x %x", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5]) == 6) {
        uint4 c = {v[0], v[1], v[2], v[3]};
        uint2 k = {v[4], v[5]};
        uint4 r = engine.apply(c, k);
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
