// Driver of the host layout planner for the sanitizer test (tests/test_sanitizers.py):
// reads one problem's observation indices from a binary file and runs ba_plan_validate,
// which plans the HBM layout (and the multidirectional layouts for the given N) exactly
// as the library's build does and checks every invariant the kernels index by.
//
// File layout (little endian): int32 n_cams, int32 n_lms, int64 n_obs, int32 cam[n_obs],
// int32 lm[n_obs].  Arguments: file max_slots max_tiles N...
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "ba.h"

int main(int argc, char **argv) {
    if (argc < 4) {
        std::fprintf(stderr, "usage: %s file max_slots max_tiles [N...]\n", argv[0]);
        return 2;
    }
    FILE *f = std::fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t nc = 0, nl = 0;
    int64_t m = 0;
    if (std::fread(&nc, 4, 1, f) != 1 || std::fread(&nl, 4, 1, f) != 1 || std::fread(&m, 8, 1, f) != 1) return 2;
    std::vector<int32_t> cam((size_t)m), lm((size_t)m);
    if (std::fread(cam.data(), 4, (size_t)m, f) != (size_t)m || std::fread(lm.data(), 4, (size_t)m, f) != (size_t)m)
        return 2;
    std::fclose(f);
    std::vector<int32_t> Ns;
    for (int i = 4; i < argc; ++i) Ns.push_back(std::atoi(argv[i]));
    std::vector<int64_t> stats(4 + 3 * Ns.size());
    const ba_status st = ba_plan_validate(nc, nl, m, cam.data(), lm.data(), std::atoi(argv[2]), std::atoi(argv[3]),
                                          Ns.data(), (int32_t)Ns.size(), stats.data());
    std::printf("status %d tiles %lld chunks %lld %s\n", (int)st, (long long)stats[0], (long long)stats[1],
                st == BA_OK ? "" : ba_plan_validate_error());
    return st == BA_OK ? 0 : 1;
}
