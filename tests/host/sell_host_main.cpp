// Host-only harness for the library's SELL-C-sigma build (sell.hpp): reads a
// CSR pattern and (C, sigma) from a text file, runs build_sell exactly as
// skr_matrix_create does, and writes the layout as text.  Plain C++, no GPU.
//
// Input:  n nnz C sigma / rp[n+1] / ci[nnz]
// Output: "ok" or "too_large", then cptr, clen, row, ci, idx (one line each)
#include <cstdio>
#include <vector>

#include "sell.hpp"

using namespace skr;

static void line(const std::vector<int>& v) {
    for (int x : v) std::printf("%d ", x);
    std::printf("\n");
}

int main(int argc, char** argv) {
    if (argc < 2) return 2;
    FILE* f = std::fopen(argv[1], "r");
    if (!f) return 2;
    int n, nnz, C, sigma;
    if (std::fscanf(f, "%d %d %d %d", &n, &nnz, &C, &sigma) != 4) return 2;
    std::vector<int> rp(n + 1), ci(nnz);
    for (int& v : rp)
        if (std::fscanf(f, "%d", &v) != 1) return 2;
    for (int& v : ci)
        if (std::fscanf(f, "%d", &v) != 1) return 2;
    std::fclose(f);
    HostSell h;
    if (!build_sell(n, rp, ci, C, sigma, h)) {
        std::printf("too_large\n");
        return 0;
    }
    std::printf("ok\n");
    line(h.cptr);
    line(h.clen);
    line(h.row);
    line(h.ci);
    line(h.idx);
    return 0;
}
