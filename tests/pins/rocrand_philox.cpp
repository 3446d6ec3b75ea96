// Host-side evaluation of rocRAND's Philox4x32-10 engine, used only as an
// independent pin for the oracle's generator.  Reads a binary request
// (uint64 seed, uint64 n, then n x uint32[4] counters with c1 < 2^30) from
// argv[1] and writes n x uint32[4] outputs to argv[2].  The counter
// (c0, c1, c2, c3) is reached as rocrand_init(seed, subsequence = c2 | c3<<32,
// offset = 4 * (c0 | c1<<32)), whose first four draws are the block's words.
#include <rocrand/rocrand_kernel.h>

#include <cstdint>
#include <cstdio>
#include <vector>

int main(int argc, char** argv)
{
    if (argc != 3) return 2;
    FILE* f = std::fopen(argv[1], "rb");
    if (!f) return 3;
    uint64_t seed = 0, n = 0;
    if (std::fread(&seed, 8, 1, f) != 1 || std::fread(&n, 8, 1, f) != 1) return 4;
    std::vector<uint32_t> ctr(4 * n), out(4 * n);
    if (std::fread(ctr.data(), 4, 4 * n, f) != 4 * n) return 5;
    std::fclose(f);
    for (uint64_t j = 0; j < n; ++j) {
        const uint32_t* c = &ctr[4 * j];
        unsigned long long sub = (unsigned long long)c[2] | ((unsigned long long)c[3] << 32);
        unsigned long long off = 4ull * ((unsigned long long)c[0] | ((unsigned long long)c[1] << 32));
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, sub, off, &st);
        for (int w = 0; w < 4; ++w) out[4 * j + w] = rocrand(&st);
    }
    FILE* g = std::fopen(argv[2], "wb");
    if (!g) return 6;
    std::fwrite(out.data(), 4, 4 * n, g);
    std::fclose(g);
    return 0;
}
