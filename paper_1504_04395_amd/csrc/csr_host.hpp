// Host-side set-up of a CSR matrix at skr_matrix_create: validation of the
// caller's arrays, int32 row pointers, and the index structure of the explicit
// conjugate transpose A^H with the permutation that maps each A^H entry to its
// A entry (A^H values are gathered through it on the device, also after a
// value refresh).
//
// Plain C++: the library and the CPU test harness both build it.
#pragma once

#include <cstdint>
#include <vector>

namespace skr {

// Checks row_ptr[0] = 0, row_ptr[n] = nnz, non-decreasing row pointers,
// columns in [0, n) and strictly increasing within a row.  Returns nullptr and
// fills rp (int32 row pointers) when valid, else the reason.
inline const char* validate_csr(int n, int64_t nnz, const std::vector<int64_t>& rp64, const std::vector<int>& ci,
                                std::vector<int>& rp) {
    if (rp64[0] != 0 || rp64[n] != nnz) return "row_ptr[0] must be 0 and row_ptr[n] = nnz";
    rp.assign(n + 1, 0);
    for (int i = 0; i < n; ++i) {
        if (rp64[i + 1] < rp64[i]) return "row_ptr must be non-decreasing";
        rp[i] = (int)rp64[i];
        for (int64_t k = rp64[i]; k < rp64[i + 1]; ++k) {
            const int col = ci[k];
            if (col < 0 || col >= n) return "column index out of range";
            if (k > rp64[i] && col <= ci[k - 1]) return "column indices must be strictly increasing within a row";
        }
    }
    rp[n] = (int)nnz;
    return nullptr;
}

// A^H index structure by a stable counting sort on the column: row j of A^H
// lists the rows i of A with a_ij stored, in increasing i, and perm[p] is the
// A position of A^H entry p.
inline void adjoint_pattern(int n, const std::vector<int>& rp, const std::vector<int>& ci, std::vector<int>& rpH,
                            std::vector<int>& ciH, std::vector<int>& perm) {
    const int nnz = rp[n];
    rpH.assign(n + 1, 0);
    ciH.assign(nnz, 0);
    perm.assign(nnz, 0);
    for (int k = 0; k < nnz; ++k) rpH[ci[k] + 1]++;
    for (int i = 0; i < n; ++i) rpH[i + 1] += rpH[i];
    std::vector<int> next(rpH.begin(), rpH.end() - 1);
    for (int i = 0; i < n; ++i)
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            const int p = next[ci[k]]++;
            ciH[p] = i;
            perm[p] = k;
        }
}

}  // namespace skr
