// Host driver of the STL reader for sanitizer builds: reads every file named
// on the command line and prints one line per file: "ok V T" or
// "err STATUS message".  Exit 0 unless the reader misbehaves (an ok result
// with inconsistent sizes).
#include <cstdio>
#include <vector>

#include "../../include/hra.h"

int main(int argc, char **argv) {
    for (int i = 1; i < argc; ++i) {
        hra_stl *m = nullptr;
        int64_t nv = 0, nt = 0;
        const hra_status st = hra_stl_read(argv[i], &m, &nv, &nt);
        if (st != HRA_OK) {
            std::printf("err %d %s\n", (int)st, hra_stl_error());
            if (m) return 1;
            continue;
        }
        std::vector<float> v(3 * (size_t)nv);
        std::vector<int32_t> t(3 * (size_t)nt);
        if (hra_stl_copy(m, v.data(), t.data()) != HRA_OK) return 1;
        for (int32_t x : t)
            if (x < 0 || x >= nv) return 1;
        hra_stl_free(m);
        std::printf("ok %lld %lld\n", (long long)nv, (long long)nt);
    }
    return 0;
}
