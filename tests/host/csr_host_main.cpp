// Host-only harness for the library's CSR set-up (csr_host.hpp): reads n, nnz,
// row_ptr (int64) and columns from a text file, validates them and builds the
// A^H index structure exactly as skr_matrix_create does.  Plain C++, no GPU.
//
// Input:  n nnz / row_ptr[n+1] / ci[nnz]
// Output: "ERROR <reason>", or "ok" then rpH, ciH, perm (one line each)
#include <cstdio>
#include <vector>

#include "csr_host.hpp"

using namespace skr;

int main(int argc, char** argv) {
    if (argc < 2) return 2;
    FILE* f = std::fopen(argv[1], "r");
    if (!f) return 2;
    int n;
    long long nnz;
    if (std::fscanf(f, "%d %lld", &n, &nnz) != 2) return 2;
    std::vector<int64_t> rp64(n + 1);
    std::vector<int> ci(nnz);
    for (auto& v : rp64) {
        long long x;
        if (std::fscanf(f, "%lld", &x) != 1) return 2;
        v = x;
    }
    for (int& v : ci)
        if (std::fscanf(f, "%d", &v) != 1) return 2;
    std::fclose(f);
    std::vector<int> rp, rpH, ciH, perm;
    if (const char* why = validate_csr(n, nnz, rp64, ci, rp)) {
        std::printf("ERROR %s\n", why);
        return 0;
    }
    adjoint_pattern(n, rp, ci, rpH, ciH, perm);
    std::printf("ok\n");
    for (const auto* v : {&rpH, &ciH, &perm}) {
        for (int x : *v) std::printf("%d ", x);
        std::printf("\n");
    }
    return 0;
}
