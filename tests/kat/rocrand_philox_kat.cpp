// Independent Philox4x32-10 reference for the CPU tests: rocRAND's
// open-source engine, evaluated on the host.  Reads lines
// "c0 c1 c2 c3 k0 k1" (hex) on stdin, prints the four output words.
// Counter words (c0, c1) are reached through the engine's offset and
// (c2, c3) through its subsequence, which is how the engine maps them.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main() {
    unsigned c[4], k[2];
    while (std::scanf("%x %x %x %x %x %x", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
        const unsigned long long seed = (unsigned long long)k[1] << 32 | k[0];
        const unsigned long long subseq = (unsigned long long)c[3] << 32 | c[2];
        const unsigned long long offset = 4ull * ((unsigned long long)c[1] << 32 | c[0]);
        rocrand_device::philox4x32_10_engine e(seed, subseq, offset);
        const uint4 r = e.next4();
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
