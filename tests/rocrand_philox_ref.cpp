// Host-side reference for the Philox4x32-10 pin: evaluates rocRAND's
// independent implementation of the published Philox4x32-10 block function
// (rocrand_device::philox4x32_10_engine::ten_rounds) for counter/key lines
// read from stdin ("c0 c1 c2 c3 k0 k1" as decimal) and prints the 4 output
// words.  Test helper only; it is compiled by the tests into a temporary
// directory and never linked into the library.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

// ten_rounds is a protected member; a derived class makes it callable.
struct philox_block : rocrand_device::philox4x32_10_engine {
    using rocrand_device::philox4x32_10_engine::ten_rounds;
};

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    philox_block eng;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 ctr = {c0, c1, c2, c3};
        uint2 key = {k0, k1};
        uint4 out = eng.ten_rounds(ctr, key);
        std::printf("%u %u %u %u\n", out.x, out.y, out.z, out.w);
    }
    return 0;
}
