// Host-only driver around rocRAND's Philox4x32-10 engine (a library routine,
// compiled here from the installed rocRAND headers and run on the CPU).
// Reads lines "seed c0 c1 c2 c3" (decimal) on stdin and prints the four output
// words of that counter under that key, in hex.
//
// rocRAND keys the engine with (seed low word, seed high word); the upper 64
// counter bits are its "subsequence" and the lower 64 bits are its "offset"
// divided by four, so the engine positioned at (subsequence, 4 * offset)
// returns exactly the block for counter (c0, c1, c2, c3).
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_kernel.h>
#include <cstdio>

int main() {
    unsigned long long seed, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu", &seed, &c0, &c1, &c2, &c3) == 5) {
        unsigned long long offset = (c0 | (c1 << 32)) * 4ULL;
        unsigned long long subseq = c2 | (c3 << 32);
        rocrand_device::philox4x32_10_engine e(seed, subseq, offset);
        unsigned int w0 = e(), w1 = e(), w2 = e(), w3 = e();
        std::printf("%08x %08x %08x %08x\n", w0, w1, w2, w3);
    }
    return 0;
}
