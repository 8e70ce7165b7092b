// Host driver of the library's lattice builder for the sanitizer build (test
// infrastructure): builds sparse pore lattices and their pull tables from
// random masks with every z treatment, side periodicity and reservoir
// setting, checks the pull table's bijection and the compact forms' decoding
// against it (the library's own host checks), and exercises code limits
// that send tiles to every form. Built with -fsanitize=address,undefined by
// tests/test_host_sanitizers.py; exits non-zero when a check fails.
#include <cstdio>
#include <cstdint>
#include <random>
#include <string>
#include <vector>

#include "../../paper_1806_10589_amd/csrc/lattice.h"
#include "../../paper_1806_10589_amd/csrc/pull_format.h"

int main()
{
    std::mt19937 gen(1234);
    int fails = 0;
    const int shapes[][3] = {{7, 6, 5}, {33, 5, 9}, {16, 16, 12}, {40, 31, 6}};
    for (const auto &sh : shapes)
        for (int z_mode = 0; z_mode < 3; ++z_mode)
            for (int per = 0; per < 4; ++per)
                for (int res = 0; res < 2; ++res) {
                    flbm::LatticeSpec spec;
                    spec.nx = sh[0];
                    spec.ny = sh[1];
                    spec.nz = sh[2];
                    spec.periodic_x = per & 1;
                    spec.periodic_y = (per >> 1) & 1;
                    spec.z_mode = z_mode;
                    spec.reservoir_layers = res;
                    std::vector<uint8_t> mask((size_t)sh[0] * sh[1] * sh[2]);
                    std::bernoulli_distribution solid(0.3);
                    for (auto &m : mask) m = solid(gen) ? 1 : 0;
                    for (int i = 0; i < sh[0] * sh[1]; ++i) mask[i] = 0;  // an open inlet plane
                    flbm::Lattice L;
                    int code = 0;
                    std::string e = flbm::build_lattice(mask.data(), spec, L, code);
                    if (!e.empty()) {
                        std::printf("build_lattice: %s\n", e.c_str());
                        ++fails;
                        continue;
                    }
                    e = flbm::check_pull_bijection(L, spec);
                    if (!e.empty()) {
                        std::printf("bijection: %s\n", e.c_str());
                        ++fails;
                    }
                    const int32_t limits[][2] = {{(int32_t)flbm::PULL_MAX_CODE, (int32_t)flbm::PULL_MAX_BYTE},
                                                 {40, 6},
                                                 {(int32_t)flbm::PULL_MAX_CODE, 0}};
                    for (const auto &lim : limits) {
                        flbm::CompactPull cp;
                        e = flbm::build_compact_pull(L, 512, lim[0], lim[1], cp);
                        if (e.empty()) e = flbm::check_compact_pull(L, cp);
                        if (!e.empty()) {
                            std::printf("compact (%d, %d): %s\n", lim[0], lim[1], e.c_str());
                            ++fails;
                        }
                    }
                }
    // a mask the builder must refuse: no pore site on the inlet plane
    {
        flbm::LatticeSpec spec;
        spec.nx = spec.ny = 4;
        spec.nz = 5;
        std::vector<uint8_t> mask(80, 0);
        for (int i = 0; i < 16; ++i) mask[i] = 1;
        flbm::Lattice L;
        int code = 0;
        if (flbm::build_lattice(mask.data(), spec, L, code).empty()) ++fails;
    }
    std::printf("lattice driver: %d failures\n", fails);
    return fails ? 1 : 0;
}
