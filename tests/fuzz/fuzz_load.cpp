// Mutation fuzzing of ac_load's blob parser on the host (built with the
// host compiler's address and undefined-behaviour sanitizers).  Every
// mutated blob must be answered with a status: AC_ERR_FORMAT, or -- when the
// mutation leaves a well-formed blob -- the device error of this GPU-less
// build.  Any crash or sanitizer report fails the run.
//   fuzz_load <blob file> <iterations> <seed>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "qkc.h"

int main(int argc, char **argv) {
    if (argc != 4) return 2;
    FILE *f = std::fopen(argv[1], "rb");
    if (!f) return 2;
    std::vector<uint8_t> blob;
    for (int c; (c = std::fgetc(f)) != EOF;) blob.push_back(static_cast<uint8_t>(c));
    std::fclose(f);
    const long iters = std::atol(argv[2]);
    std::mt19937_64 rng(std::strtoull(argv[3], nullptr, 10));
    long n_format = 0, n_device = 0, n_other = 0;
    const uint32_t edge[] = {0u, 1u, 2u, 7u, 0x7fffffffu, 0x80000000u, 0xfffffffeu, 0xffffffffu, 0x3fffffffu, 64u, 65u};
    for (long it = 0; it < iters; ++it) {
        std::vector<uint8_t> b = blob;
        const int kind = static_cast<int>(rng() % 5);
        if (kind == 0) {                                   // truncation
            b.resize(rng() % b.size());
        } else if (kind == 1) {                            // bit flips anywhere
            const int n = 1 + static_cast<int>(rng() % 8);
            for (int i = 0; i < n; ++i) b[rng() % b.size()] ^= static_cast<uint8_t>(1u << (rng() % 8));
        } else if (kind == 2) {                            // a header field set to an edge value
            const size_t at = 8 + 4 * (rng() % 14);
            const uint32_t v = edge[rng() % (sizeof(edge) / sizeof(edge[0]))];
            std::memcpy(&b[at], &v, 4);
        } else if (kind == 3) {                            // a random aligned word set to an edge value
            const size_t at = (rng() % (b.size() / 4)) * 4;
            const uint32_t v = edge[rng() % (sizeof(edge) / sizeof(edge[0]))];
            std::memcpy(&b[at], &v, 4);
        } else {                                           // random bytes appended or a random byte run
            const size_t at = rng() % b.size(), len = 1 + rng() % 64;
            for (size_t i = 0; i < len && at + i < b.size(); ++i) b[at + i] = static_cast<uint8_t>(rng());
        }
        ac_graph *g = nullptr;
        const ac_status st = ac_load(b.empty() ? nullptr : b.data(), b.size(), 0, &g);
        if (g) ac_free(g);
        if (st == AC_ERR_FORMAT || st == AC_ERR_INVALID_ARG) ++n_format;
        else if (st == AC_ERR_DEVICE) ++n_device;
        else ++n_other;
    }
    std::printf("format %ld device %ld other %ld\n", n_format, n_device, n_other);
    return n_other == 0 ? 0 : 1;
}
