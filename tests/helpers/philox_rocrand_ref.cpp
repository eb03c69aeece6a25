// Reference Philox4x32-10 outputs from rocRAND's header implementation
// (independent of the oracle), run on the host CPU only.
// stdin: lines "key_lo key_hi c0 c1 c2 c3" (hex); stdout: 4 hex words per line.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned k0, k1, c0, c1, c2, c3;
    while (std::scanf("%x %x %x %x %x %x", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        unsigned long long key = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long lo = (unsigned long long)c0 | ((unsigned long long)c1 << 32);
        unsigned long long hi = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        // the engine's counter is (offset / 4) in words x,y and the subsequence in z,w
        rocrand_device::philox4x32_10_engine e(key, hi, lo * 4ull);
        unsigned a = e.next(), b = e.next(), c = e.next(), d = e.next();
        std::printf("%08x %08x %08x %08x\n", a, b, c, d);
    }
    return 0;
}
