// Host-only probe of the library's starting shapes (no HIP call is made):
//   shapes_probe nc ne nv N [nc ne nv N ...]  -> the 7 shapes of a launch set
//                                               over those instances
//   shapes_probe w max_lds N [N ...]          -> columns per block of the
//                                               level-parallel column for N levels
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "nhdc_host.h"

int main(int argc, char **argv) {
    if (argc > 2 && std::strcmp(argv[1], "w") == 0) {
        const int max_lds = std::atoi(argv[2]);
        for (int i = 3; i < argc; ++i) std::printf("%d ", nhdc::stg_width(std::atoi(argv[i]), max_lds));
        std::printf("\n");
        return 0;
    }
    if (argc < 5 || (argc - 1) % 4 != 0) return 2;
    std::vector<nhdc::Grid> g((argc - 1) / 4);
    std::vector<const nhdc::Grid *> p;
    for (size_t i = 0; i < g.size(); ++i) {
        g[i].nc = std::atoll(argv[1 + 4 * i]);
        g[i].ne = std::atoll(argv[2 + 4 * i]);
        g[i].nv = std::atoll(argv[3 + 4 * i]);
        g[i].N = std::atoi(argv[4 + 4 * i]);
        p.push_back(&g[i]);
    }
    int s[7];
    nhdc::tune_shapes(nhdc::default_tune(p.data(), int(p.size())), s);
    for (int v : s) std::printf("%d ", v);
    std::printf("\n");
    return 0;
}
