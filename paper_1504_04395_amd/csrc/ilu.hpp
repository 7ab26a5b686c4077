// Right no-fill ILU preconditioning (Section 5.2 uses a right ILU without fill
// for Examples 1-3).
//
// Set-up (host, once per matrix): ILU(0) by row-wise Gaussian elimination that
// keeps only updates inside A's sparsity pattern (Saad, Section 10.3.2), so
// that (L U)_ij = a_ij on the pattern; L is unit lower, U upper triangular.
// The four triangular operators a right-preconditioned method needs --
// L and U for A M^-1, U^H and L^H for M^-H A^H -- are stored as CSR of their
// strictly triangular parts plus the diagonal, with their rows grouped into
// dependency levels: the rows of one level depend only on earlier levels.
//
// Apply (device): thread (row, column) of the n x s block computes
// y_i = (z_i - sum_j t_ij y_j) [/ t_ii], level after level: one launch per
// level, or one workgroup that sweeps all levels when they hold little work.
// A level's rows read only rows of earlier levels, so in-place solves
// (Y == Z) are race-free.
#pragma once

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "common.hpp"

namespace skr {

struct IluError {
    std::string what;
};

// A triangular operator in level order: position p = 0..n-1 runs over the rows
// level by level; rows[p] is the row at p, and rp[p]..rp[p+1] its strictly
// triangular entries (ci, va), dg[p] its diagonal.  The row index, the entry
// range and the diagonal of a position are independent loads, and the entries
// of one level are contiguous.
template <class T>
struct TriOp {
    const int* rp;
    const int* ci;
    const T* va;
    const T* dg;       // nullptr = unit diagonal
    const int* rows;
};

__device__ inline double tdiv(double a, double b) { return a / b; }
__device__ inline c64 tdiv(c64 a, c64 b) { return cdiv(a, b); }

template <class T>
__global__ __launch_bounds__(kBlock) void k_trsv_level(const Ctl* ctl, TriOp<T> F, int l0, int cnt, int s,
                                                       const T* Z, T* Y) {
    if (stopped(ctl)) return;
    const long long g = (long long)blockIdx.x * kBlock + threadIdx.x;
    const int q = (int)(g / s);
    if (q >= cnt) return;
    const int c = (int)(g - (long long)q * s);
    const int p = l0 + q, i = F.rows[p];
    T acc = Z[(size_t)i * s + c];
    for (int k = F.rp[p]; k < F.rp[p + 1]; ++k) acc = fma_(-F.va[k], Y[(size_t)F.ci[k] * s + c], acc);
    Y[(size_t)i * s + c] = F.dg ? tdiv(acc, F.dg[p]) : acc;
}

// All levels in one workgroup (levels with little work): the workgroup sweeps
// the levels in order with a barrier between them, which makes each level's
// rows visible to the next.  lvl: nlev + 1 level offsets on the device.
constexpr int kTrsvWg = 1024;
template <class T>
__global__ __launch_bounds__(kTrsvWg) void k_trsv_wg(const Ctl* ctl, TriOp<T> F, const int* __restrict__ lvl,
                                                     int nlev, int s, const T* Z, T* Y) {
    if (stopped(ctl)) return;
    for (int l = 0; l < nlev; ++l) {
        const int l0 = lvl[l], work = (lvl[l + 1] - l0) * s;
        for (int g = threadIdx.x; g < work; g += kTrsvWg) {
            const int q = g / s, c = g - q * s;
            const int p = l0 + q, i = F.rows[p];
            T acc = Z[(size_t)i * s + c];
            for (int k = F.rp[p]; k < F.rp[p + 1]; ++k) acc = fma_(-F.va[k], Y[(size_t)F.ci[k] * s + c], acc);
            Y[(size_t)i * s + c] = F.dg ? tdiv(acc, F.dg[p]) : acc;
        }
        __syncthreads();
    }
}

// The same sweep, software-pipelined, when every level fits one pass of the
// workgroup (rows x s <= kTrsvWg): thread t owns item t of each level (row
// t / s of the level, column t % s).  While level l is solved, the row index,
// entry range and diagonal of level l + 2 and the first kTrsvK entries and the
// right-hand side of level l + 1 are already loading, so a level waits on one
// round of memory (the gathers of solved rows) instead of three.  Prefetched
// values are only of the operator and of Z; Z's row i is not written before
// row i itself is solved (in-place solves included).
constexpr int kTrsvK = 4;
template <class T>
struct TrsvItem {
    bool on;
    int i, kb, ke;
    T d;
};
template <class T>
__device__ inline TrsvItem<T> trsv_stage_a(const TriOp<T>& F, const int* __restrict__ lvl, int nlev, int l, int s,
                                           int t) {
    TrsvItem<T> it{false, 0, 0, 0, zero<T>()};
    if (l >= nlev) return it;
    const int l0 = lvl[l];
    if (t >= (lvl[l + 1] - l0) * s) return it;
    const int p = l0 + t / s;
    it.on = true;
    it.i = F.rows[p];
    it.kb = F.rp[p];
    it.ke = F.rp[p + 1];
    if (F.dg) it.d = F.dg[p];
    return it;
}
template <class T>
__global__ __launch_bounds__(kTrsvWg) void k_trsv_wgp(const Ctl* ctl, TriOp<T> F, const int* __restrict__ lvl,
                                                      int nlev, int s, const T* Z, T* Y) {
    if (stopped(ctl)) return;
    const int t = threadIdx.x, c = t % s;
    int cc0[kTrsvK], cc1[kTrsvK];
    T vv0[kTrsvK], vv1[kTrsvK], z0 = zero<T>(), z1 = zero<T>();
    auto stage_b = [&](const TrsvItem<T>& it, int (&cc)[kTrsvK], T (&vv)[kTrsvK], T& z) {
#pragma unroll
        for (int k = 0; k < kTrsvK; ++k) {
            const bool ok = it.on && it.kb + k < it.ke;
            cc[k] = ok ? F.ci[it.kb + k] : 0;
            vv[k] = ok ? F.va[it.kb + k] : zero<T>();
        }
        if (it.on) z = Z[(size_t)it.i * s + c];
    };
    TrsvItem<T> a0 = trsv_stage_a(F, lvl, nlev, 0, s, t);
    stage_b(a0, cc0, vv0, z0);
    TrsvItem<T> a1 = trsv_stage_a(F, lvl, nlev, 1, s, t);
    for (int l = 0; l < nlev; ++l) {
        stage_b(a1, cc1, vv1, z1);                                  // level l + 1
        const TrsvItem<T> a2 = trsv_stage_a(F, lvl, nlev, l + 2, s, t);   // level l + 2
        if (a0.on) {                                                // level l
            T acc = z0;
#pragma unroll
            for (int k = 0; k < kTrsvK; ++k)
                if (a0.kb + k < a0.ke) acc = fma_(-vv0[k], Y[(size_t)cc0[k] * s + c], acc);
            for (int k = a0.kb + kTrsvK; k < a0.ke; ++k) acc = fma_(-F.va[k], Y[(size_t)F.ci[k] * s + c], acc);
            Y[(size_t)a0.i * s + c] = F.dg ? tdiv(acc, a0.d) : acc;
        }
        __syncthreads();
        a0 = a1;
        a1 = a2;
        z0 = z1;
#pragma unroll
        for (int k = 0; k < kTrsvK; ++k) {
            cc0[k] = cc1[k];
            vv0[k] = vv1[k];
        }
    }
}

// ------------------------------------------------------------------ host side
inline bool hzero(double v) { return v == 0.0; }
inline bool hzero(c64 v) { return v.x == 0.0 && v.y == 0.0; }
inline bool hfinite(double v) { return std::isfinite(v); }
inline bool hfinite(c64 v) { return std::isfinite(v.x) && std::isfinite(v.y); }
inline double hdiv(double a, double b) { return a / b; }
inline c64 hdiv(c64 a, c64 b) { return cdiv(a, b); }
inline double hconj(double a) { return a; }
inline c64 hconj(c64 a) { return conj_(a); }

// One triangular operator: host arrays while building, device arrays after upload.
template <class T>
struct TriHost {
    std::vector<int> rp, ci, rows, lvl;
    std::vector<T> va, dg;
};

struct TriDev {
    int *rp = nullptr, *ci = nullptr, *rows = nullptr, *dlvl = nullptr;
    void *va = nullptr, *dg = nullptr;
    std::vector<int> lvl;   // level offsets into rows (host copy, drives the launches; dlvl on the device)
    int maxrows = 0;        // rows of the widest level
    size_t bytes = 0;
};

struct Ilu {
    int dtype = 0;
    TriDev L, U, UH, LH;
};

// Level of each row: forward (lower operators, row i needs rows j < i) or
// backward (upper operators, row i needs rows j > i); rows sorted by level.
template <class T>
void tri_levels(TriHost<T>& t, int n, bool forward) {
    std::vector<int> lev(n, 0);
    int nlev = 0;
    for (int q = 0; q < n; ++q) {
        const int i = forward ? q : n - 1 - q;
        int l = 0;
        for (int k = t.rp[i]; k < t.rp[i + 1]; ++k) l = std::max(l, lev[t.ci[k]] + 1);
        lev[i] = l;
        nlev = std::max(nlev, l + 1);
    }
    t.lvl.assign(nlev + 1, 0);
    for (int i = 0; i < n; ++i) ++t.lvl[lev[i] + 1];
    for (int l = 0; l < nlev; ++l) t.lvl[l + 1] += t.lvl[l];
    std::vector<int> fill(t.lvl.begin(), t.lvl.end() - 1);
    t.rows.assign(n, 0);
    for (int i = 0; i < n; ++i) t.rows[fill[lev[i]]++] = i;
}

// The level-order copy of a row-ordered operator (after tri_levels): entry
// range, entries and diagonal of the row at each position of t.rows.
template <class T>
void tri_level_order(const TriHost<T>& t, int n, TriHost<T>& out) {
    out.rp.assign(n + 1, 0);
    out.ci.clear();
    out.va.clear();
    out.ci.reserve(t.ci.size());
    out.va.reserve(t.va.size());
    if (!t.dg.empty()) out.dg.resize(n);
    for (int p = 0; p < n; ++p) {
        const int i = t.rows[p];
        for (int k = t.rp[i]; k < t.rp[i + 1]; ++k) {
            out.ci.push_back(t.ci[k]);
            out.va.push_back(t.va[k]);
        }
        out.rp[p + 1] = (int)out.ci.size();
        if (!t.dg.empty()) out.dg[p] = t.dg[i];
    }
    out.rows = t.rows;
    out.lvl = t.lvl;
}

// Conjugate transpose of a strictly triangular CSR (counting sort by column).
template <class T>
void tri_adjoint(const TriHost<T>& a, int n, TriHost<T>& out) {
    const int nnz = a.rp[n];
    out.rp.assign(n + 1, 0);
    for (int k = 0; k < nnz; ++k) ++out.rp[a.ci[k] + 1];
    for (int i = 0; i < n; ++i) out.rp[i + 1] += out.rp[i];
    std::vector<int> fill(out.rp.begin(), out.rp.end() - 1);
    out.ci.assign(nnz, 0);
    out.va.assign(nnz, T{});
    for (int i = 0; i < n; ++i)
        for (int k = a.rp[i]; k < a.rp[i + 1]; ++k) {
            const int d = fill[a.ci[k]]++;
            out.ci[d] = i;
            out.va[d] = hconj(a.va[k]);
        }
    if (!a.dg.empty()) {
        out.dg.resize(n);
        for (int i = 0; i < n; ++i) out.dg[i] = hconj(a.dg[i]);
    }
}

// ILU(0) of the CSR (rp, ci sorted within rows, a) into L (strict lower, unit
// diagonal) and U (strict upper + diagonal).  Throws IluError for a missing
// diagonal entry or a zero / non-finite pivot.
template <class T>
void ilu0_factor(int n, const std::vector<int>& rp, const std::vector<int>& ci, std::vector<T> a, TriHost<T>& L,
                 TriHost<T>& U) {
    std::vector<int> dpos(n, -1), pos(n, -1);
    for (int i = 0; i < n; ++i)
        for (int k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] == i) dpos[i] = k;
    for (int i = 0; i < n; ++i)
        if (dpos[i] < 0) throw IluError{"ILU(0): row " + std::to_string(i) + " has no diagonal entry"};
    for (int i = 0; i < n; ++i) {
        for (int k = rp[i]; k < rp[i + 1]; ++k) pos[ci[k]] = k;
        for (int e = rp[i]; e < rp[i + 1] && ci[e] < i; ++e) {
            const int kk = ci[e];
            const T lik = hdiv(a[e], a[dpos[kk]]);
            a[e] = lik;
            for (int f = dpos[kk] + 1; f < rp[kk + 1]; ++f)
                if (pos[ci[f]] >= 0) a[pos[ci[f]]] = a[pos[ci[f]]] - lik * a[f];
        }
        if (hzero(a[dpos[i]]) || !hfinite(a[dpos[i]]))
            throw IluError{"ILU(0): zero or non-finite pivot in row " + std::to_string(i)};
        for (int k = rp[i]; k < rp[i + 1]; ++k) pos[ci[k]] = -1;
    }
    L.rp.assign(n + 1, 0);
    U.rp.assign(n + 1, 0);
    U.dg.resize(n);
    for (int i = 0; i < n; ++i) {
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            if (ci[k] < i) {
                L.ci.push_back(ci[k]);
                L.va.push_back(a[k]);
            } else if (ci[k] > i) {
                U.ci.push_back(ci[k]);
                U.va.push_back(a[k]);
            }
        }
        U.dg[i] = a[dpos[i]];
        L.rp[i + 1] = (int)L.ci.size();
        U.rp[i + 1] = (int)U.ci.size();
    }
}

// Y = T^-1 Z for one triangular operator, level by level (Y may equal Z).
// When the levels are narrow -- on average at most 256 rows (each a few
// scattered cache lines that one CU must fetch) and at most two passes of one
// workgroup (rows x s <= 2048) -- a single workgroup sweeps them all;
// otherwise each level is its own launch over as many workgroups as it needs.
template <class T>
void tri_solve(hipStream_t st, const TriDev& t, int s, const T* Z, T* Y, const Ctl* ctl) {
    const TriOp<T> op{t.rp, t.ci, (const T*)t.va, (const T*)t.dg, t.rows};
    const int nlev = (int)t.lvl.size() - 1;
    if (nlev < 1) return;
    const long long rows = t.lvl[nlev];
    if (rows <= 256LL * nlev && rows * s <= 2LL * kTrsvWg * nlev) {
        if ((long long)t.maxrows * s <= kTrsvWg)
            k_trsv_wgp<T><<<1, kTrsvWg, 0, st>>>(ctl, op, t.dlvl, nlev, s, Z, Y);
        else
            k_trsv_wg<T><<<1, kTrsvWg, 0, st>>>(ctl, op, t.dlvl, nlev, s, Z, Y);
        return;
    }
    for (size_t l = 0; l + 1 < t.lvl.size(); ++l) {
        const int l0 = t.lvl[l], cnt = t.lvl[l + 1] - l0;
        const long long threads = (long long)cnt * s;
        const int grid = (int)((threads + kBlock - 1) / kBlock);
        k_trsv_level<T><<<grid, kBlock, 0, st>>>(ctl, op, l0, cnt, s, Z, Y);
    }
}

}  // namespace skr
