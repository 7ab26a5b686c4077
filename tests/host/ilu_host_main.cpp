// Host-only harness for the library's ILU(0) set-up code (ilu.hpp): reads a
// CSR matrix from a text file, runs the factorisation, the conjugate
// transposes and the level schedules exactly as skr_matrix_ilu0 does, and
// writes the four triangular operators as text.  Used by the CPU test suite;
// it calls no HIP runtime function and needs no GPU.
//
// Input:  n nnz complex(0|1) / rp[n+1] / ci[nnz] / values (re [im]) per entry
// Output: for each of L, U, UH, LH: "name nnz nlev", rp, ci, values, diagonal
//         (or "-"), rows (level order), level offsets; then the same for their
//         level-order copies (Lo, Uo, UHo, LHo: rp, values and diagonal indexed
//         by position).  "ERROR msg" on failure.
#include <cstdio>
#include <vector>

#include "ilu.hpp"

using namespace skr;

template <class T>
static void put(const T& v) {
    if constexpr (std::is_same<T, c64>::value) std::printf("%.17g %.17g ", v.x, v.y);
    else std::printf("%.17g ", v);
}

template <class T>
static void dump(const char* name, const TriHost<T>& t, int n) {
    std::printf("%s %d %d\n", name, t.rp[n], (int)t.lvl.size() - 1);
    for (int v : t.rp) std::printf("%d ", v);
    std::printf("\n");
    for (int v : t.ci) std::printf("%d ", v);
    std::printf("\n");
    for (const T& v : t.va) put(v);
    std::printf("\n");
    if (t.dg.empty()) std::printf("-");
    for (const T& v : t.dg) put(v);
    std::printf("\n");
    for (int v : t.rows) std::printf("%d ", v);
    std::printf("\n");
    for (int v : t.lvl) std::printf("%d ", v);
    std::printf("\n");
}

template <class T>
static int run(int n, const std::vector<int>& rp, const std::vector<int>& ci, const std::vector<T>& va) {
    TriHost<T> L, U, UH, LH;
    try {
        ilu0_factor<T>(n, rp, ci, va, L, U);
    } catch (const IluError& e) {
        std::printf("ERROR %s\n", e.what.c_str());
        return 0;
    }
    tri_adjoint(U, n, UH);
    tri_adjoint(L, n, LH);
    tri_levels(L, n, true);
    tri_levels(U, n, false);
    tri_levels(UH, n, true);
    tri_levels(LH, n, false);
    dump("L", L, n);
    dump("U", U, n);
    dump("UH", UH, n);
    dump("LH", LH, n);
    const TriHost<T>* ops[4] = {&L, &U, &UH, &LH};
    const char* names[4] = {"Lo", "Uo", "UHo", "LHo"};
    for (int k = 0; k < 4; ++k) {   // the level-order copies the device solves use
        TriHost<T> o;
        tri_level_order(*ops[k], n, o);
        dump(names[k], o, n);
    }
    return 0;
}

int main(int argc, char** argv) {
    if (argc < 2) return 2;
    FILE* f = std::fopen(argv[1], "r");
    if (!f) return 2;
    int n, nnz, cplx;
    if (std::fscanf(f, "%d %d %d", &n, &nnz, &cplx) != 3) return 2;
    std::vector<int> rp(n + 1), ci(nnz);
    for (auto& v : rp)
        if (std::fscanf(f, "%d", &v) != 1) return 2;
    for (auto& v : ci)
        if (std::fscanf(f, "%d", &v) != 1) return 2;
    if (cplx) {
        std::vector<c64> va(nnz);
        for (auto& v : va)
            if (std::fscanf(f, "%lf %lf", &v.x, &v.y) != 2) return 2;
        return run<c64>(n, rp, ci, va);
    }
    std::vector<double> va(nnz);
    for (auto& v : va)
        if (std::fscanf(f, "%lf", &v) != 1) return 2;
    return run<double>(n, rp, ci, va);
}
