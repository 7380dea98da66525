// Host-side reference for the Philox4x32-10 pin: evaluates rocRAND's own
// host-callable ten_rounds() (rocrand_philox4x32_10.h) for (counter, key)
// tuples read from stdin, one "c0 c1 c2 c3 k0 k1" line each, and prints the
// four output words. Test infrastructure only.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

// ten_rounds() is a protected member: a derived class makes it callable.
struct philox_ref : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    philox_ref eng;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 c = {c0, c1, c2, c3};
        uint2 k = {k0, k1};
        uint4 r = eng.block(c, k);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
