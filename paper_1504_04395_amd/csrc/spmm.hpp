// Sparse matrix x block products Y = A X for row-major n x s blocks.
//
// CSR: a group of L lanes owns one row; each lane owns columns lane + L*j
// (j < J) of the block, so every stored nonzero a_ij is read once for all s
// right-hand sides and the s values X[j, :] are one contiguous read: the
// memory-traffic saving that motivates the simultaneous methods (Section 1).
//
// SELL-C-sigma: rows are sorted by length inside windows of sigma rows and cut
// into chunks of C rows; a chunk stores its entries column-major (slot k of all
// C rows together), padded to the chunk's longest row.  16 lanes own one row
// (k_spmm_sell16); the padding entries have value 0 and column = row.
//
// Epilogues fold the reductions the solvers need right after the product into
// the same pass (the output row is still in registers): traces tr(Z^H Y),
// eGl's sum(z^H Y) and s x s Gram matrices (MFMA, tile-16 layout).
#pragma once

#include "common.hpp"

#include <type_traits>

namespace skr {

template <class T>
struct CsrOp {
    int n;
    const int* __restrict__ rp;
    const int* __restrict__ ci;
    const T* __restrict__ va;
};

template <class T>
struct SellOp {
    int n;
    int C;                          // chunk height (rows)
    const int* __restrict__ cptr;   // chunk start offsets (nchunks + 1), in entries
    const int* __restrict__ clen;   // chunk width (slots)
    const int* __restrict__ row;    // sorted position -> original row
    const int* __restrict__ ci;     // column of each slot
    const T* __restrict__ va;       // value of each slot (0 for padding)
};

struct Layout {
    int s;      // block width
    int L;      // lanes per row (power of two, <= 16)
    int lgL;
};

// ------------------------------------------------------------------ epilogues
struct EpiNone {
    struct St {};
    __device__ void init(St&) {}
    template <class T, int J>
    __device__ void row(St&, int, bool, int, const Layout&, const T (&)[J]) {}
    __device__ void finish(St&, int) {}
};

// part[block] = sum_rows sum_c conj(Z[i,c]) * Y[i,c]   (tr(Z^H Y))
template <class T>
struct EpiTrace {
    const T* __restrict__ Z;
    c64* part;
    struct St { c64 acc[1]; };
    __device__ void init(St& st) { st.acc[0] = {0.0, 0.0}; }
    template <int J>
    __device__ void row(St& st, int i, bool valid, int lane, const Layout& ly, const T (&y)[J]) {
        if (!valid) return;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            int c = lane + ly.L * j;
            if (c < ly.s) dot_acc(st.acc[0], Z[(size_t)i * ly.s + c], y[j]);
        }
    }
    __device__ void finish(St& st, int b) { block_reduce_store<1>(st.acc, part + (size_t)b); }
};

// part[block] = sum_i conj(z_i) sum_c Y[i,c]   (sum(z^H Y), economic variants)
template <class T>
struct EpiVecSum {
    const T* __restrict__ z;
    c64* part;
    struct St { c64 acc[1]; };
    __device__ void init(St& st) { st.acc[0] = {0.0, 0.0}; }
    template <int J>
    __device__ void row(St& st, int i, bool valid, int lane, const Layout& ly, const T (&y)[J]) {
        if (!valid) return;
        T zi = z[i];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            int c = lane + ly.L * j;
            if (c < ly.s) dot_acc(st.acc[0], zi, y[j]);
        }
    }
    __device__ void finish(St& st, int b) { block_reduce_store<1>(st.acc, part + (size_t)b); }
};

// part[block] = (tr(Y^H Z), tr(Y^H Y))  -- BiCGStab's omega step with Y = A S, Z = S
template <class T>
struct EpiTraceOmega {
    const T* __restrict__ Z;
    c64* part;
    struct St { c64 acc[2]; };
    __device__ void init(St& st) { st.acc[0] = {0.0, 0.0}; st.acc[1] = {0.0, 0.0}; }
    template <int J>
    __device__ void row(St& st, int i, bool valid, int lane, const Layout& ly, const T (&y)[J]) {
        if (!valid) return;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            int c = lane + ly.L * j;
            if (c < ly.s) {
                dot_acc(st.acc[0], y[j], Z[(size_t)i * ly.s + c]);
                dot_acc(st.acc[1], y[j], y[j]);
            }
        }
    }
    __device__ void finish(St& st, int b) { block_reduce_store<2>(st.acc, part + (size_t)b * 2); }
};

// part[block] = Z^H Y (s x s), requires L = 16 (tile-16 layout)
template <class T, int J>
struct EpiGram {
    const T* __restrict__ Z;
    c64* part;
    struct St { GramAcc<J, Tr<T>::cplx> g; };
    __device__ void init(St& st) { st.g.clear(); }
    __device__ void row(St& st, int i, bool valid, int lane, const Layout& ly, const T (&y)[J]) {
        c64 zv[J], yv[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            int c = lane + 16 * j;
            bool ok = valid && c < ly.s;
            zv[j] = ok ? up(Z[(size_t)i * ly.s + c]) : c64{0.0, 0.0};
            yv[j] = ok ? up(y[j]) : c64{0.0, 0.0};
        }
        st.g.add(zv, yv);
    }
    __device__ void finish(St& st, int b, int s) {
        __shared__ c64 lds[(16 * J) * (16 * J)];
        st.g.store(s, lds, part + (size_t)b * s * s);
    }
};

// part[block] = (Y^H Z, Y^H Y) as two s x s matrices -- Bl-BiCGStab-rQ omega step
template <class T, int J>
struct EpiGramOmega {
    const T* __restrict__ Z;
    c64* part;
    struct St { GramAcc<J, Tr<T>::cplx> g1, g2; };
    __device__ void init(St& st) { st.g1.clear(); st.g2.clear(); }
    __device__ void row(St& st, int i, bool valid, int lane, const Layout& ly, const T (&y)[J]) {
        c64 zv[J], yv[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            int c = lane + 16 * j;
            bool ok = valid && c < ly.s;
            zv[j] = ok ? up(Z[(size_t)i * ly.s + c]) : c64{0.0, 0.0};
            yv[j] = ok ? up(y[j]) : c64{0.0, 0.0};
        }
        st.g1.add(yv, zv);
        st.g2.add(yv, yv);
    }
    __device__ void finish(St& st, int b, int s) {
        __shared__ c64 lds[(16 * J) * (16 * J)];
        st.g1.store(s, lds, part + (size_t)b * 2 * s * s);
        st.g2.store(s, lds, part + (size_t)b * 2 * s * s + s * s);
    }
};

template <class E> struct EpiIsGram { static constexpr bool value = false; };
template <class T, int J> struct EpiIsGram<EpiGram<T, J>> { static constexpr bool value = true; };
template <class T, int J> struct EpiIsGram<EpiGramOmega<T, J>> { static constexpr bool value = true; };

template <class E, int J>
__device__ inline void epi_finish(E& e, typename E::St& st, int b, int s) {
    if constexpr (EpiIsGram<E>::value) e.finish(st, b, s);
    else e.finish(st, b);
}

// ------------------------------------------------------------------ kernels
// 32-bit broadcast of lane N of each 16-lane row (DPP row_newbcast).
template <int N>
__device__ inline int rbc32(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x150 + N, 0xF, 0xF, false); }
template <int N>
__device__ inline double rbc64(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), 0x150 + N, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x150 + N, 0xF, 0xF, false);
    return __builtin_bit_cast(double, (long long)(unsigned)lo | ((long long)hi << 32));
}
template <int N>
__device__ inline float rbc64(float v) { return __builtin_bit_cast(float, rbc32<N>(__builtin_bit_cast(int, v))); }
template <int N>
__device__ inline c64 rbc64(c64 v) { return {rbc64<N>(v.x), rbc64<N>(v.y)}; }
template <int N>
__device__ inline c32 rbc64(c32 v) { return {rbc64<N>(v.x), rbc64<N>(v.y)}; }

template <int A, int END, class F>
__device__ inline void sfor(F&& f) {
    if constexpr (A < END) {
        f(std::integral_constant<int, A>{});
        sfor<A + 1, END>(f);
    }
}

// Row mapping: XCD x (= workgroup index mod 8; workgroups are dispatched
// round-robin over the 8 XCDs) owns one contiguous region of rows, and the
// XCD's workgroups sweep that region together, one pass of RP*16 rows each per
// step.  The rows an XCD works on at any moment, and the block rows they gather
// (neighbours in a stencil ordering), then stay within a window that fits its
// L2.  Layout: 16 lanes per row (a DPP row), lane owning columns lane + 16 j.
// The row's (column, value) pairs are loaded cooperatively, 8 at a time (lane
// u & 7 loads entry u), and handed to the whole row by DPP broadcasts, so each
// nonzero costs one block-row read per lane and no per-lane index loads.
template <class T, int J, class Epi>
__global__ __launch_bounds__(kBlock) void k_spmm_csr(const Ctl* ctl, CsrOp<T> A, Layout ly, int rows_per_xcd,
                                                      const T* __restrict__ X, T* __restrict__ Y, Epi epi) {
    if (stopped(ctl)) return;
    constexpr int RP = J == 1 ? 2 : 1;
    constexpr int U = 8;
    const int lane = threadIdx.x & 15;
    const int grp = threadIdx.x >> 4;
    const int xcd = blockIdx.x & 7, q = blockIdx.x >> 3, nq = gridDim.x >> 3;
    const int r0 = xcd * rows_per_xcd;
    const int r1 = min(A.n, r0 + rows_per_xcd);
    const int s = ly.s;
    int col[J];
#pragma unroll
    for (int j = 0; j < J; ++j) col[j] = min(lane + 16 * j, s - 1);
    typename Epi::St st;
    epi.init(st);
    for (int base = r0 + q * RP * 16; base < r1; base += nq * RP * 16) {
        int i[RP], k0[RP], k1[RP];
        bool valid[RP];
#pragma unroll
        for (int p = 0; p < RP; ++p) {
            i[p] = base + p * 16 + grp;
            valid[p] = i[p] < r1;
            const int ii = min(i[p], A.n - 1);      // unconditional loads: no wait at a branch join
            const int a0 = A.rp[ii], a1 = A.rp[ii + 1];
            k0[p] = valid[p] ? a0 : 0;
            k1[p] = valid[p] ? a1 : 0;
        }
        T acc[RP][J];
#pragma unroll
        for (int p = 0; p < RP; ++p)
#pragma unroll
            for (int j = 0; j < J; ++j) acc[p][j] = zero<T>();
        for (int off = 0;; off += U) {
            int mc[RP];
            T ma[RP];
            bool more = false;
#pragma unroll
            for (int p = 0; p < RP; ++p) {
                const int k = k0[p] + off + (lane & (U - 1));
                const int kc = max(0, min(k, k1[p] - 1));   // clamped: always a valid entry
                mc[p] = A.ci[kc];
                const T v = A.va[kc];
                ma[p] = k < k1[p] ? v : zero<T>();
                more |= k0[p] + off + U < k1[p];
            }
#pragma unroll
            for (int p = 0; p < RP; ++p) {
                sfor<0, U>([&](auto ic) {
                    constexpr int u = decltype(ic)::value;
                    const int c = rbc32<u>(mc[p]);
                    const T a = rbc64<u>(ma[p]);
                    const T* __restrict__ xr = X + (size_t)c * s;
#pragma unroll
                    for (int j = 0; j < J; ++j) acc[p][j] = fma_(a, xr[col[j]], acc[p][j]);
                });
            }
            if (!more) break;
        }
#pragma unroll
        for (int p = 0; p < RP; ++p) {
            if (valid[p]) {
#pragma unroll
                for (int j = 0; j < J; ++j)
                    if (lane + 16 * j < s) Y[(size_t)i[p] * s + lane + 16 * j] = acc[p][j];
            }
        }
#pragma unroll
        for (int p = 0; p < RP; ++p) epi.row(st, i[p], valid[p], lane, ly, acc[p]);
    }
    epi_finish<Epi, J>(epi, st, blockIdx.x, s);
}

// Real blocks with even s <= 16: 8 lanes per row, lane l holding columns 2l and
// 2l + 1 (one 16-byte load of X per nonzero for FP64).  A group of 16 lanes
// carries two matrix rows; the entries of both are loaded 8 at a time (lane u
// of each half loads entry u) and staged in LDS, from where the 8 lanes of the
// row read each entry back (one address per half: an LDS broadcast).  The
// column indices are read back before the X gathers are issued and each value
// just before its FMA, so no lane holds the 8 broadcast entries in registers
// while the gathers are in flight; that keeps the FP64 kernel at 3 waves per
// SIMD.  A wave owns 16 consecutive rows per pass (two groups of 8); products
// are accumulated in FP64 also for FP32 data.  The matrix stream (indices,
// values) is read and Y is written with non-temporal hints, so that L2 keeps
// the X rows that neighbouring matrix rows gather again.  Epilogues see the
// tile-16 layout: the wave's 16 x 16 result tile goes through LDS and each
// lane then holds column (lane % 16) of rows 4v + lane / 16.
template <class T> struct Pair;
template <> struct Pair<double> { using type = double2; };
template <> struct Pair<float> { using type = float2; };

template <class T, class Epi>
__global__ __launch_bounds__(kBlock) void k_spmm_csr8(const Ctl* ctl, CsrOp<T> A, Layout ly, int rows_per_xcd,
                                                       const T* __restrict__ X, T* __restrict__ Y, Epi epi) {
    if (stopped(ctl)) return;
    using P2 = typename Pair<T>::type;
    constexpr int U = 8;
    constexpr bool EPI = !std::is_same<Epi, EpiNone>::value;
    constexpr bool G1 = std::is_same<Epi, EpiGram<T, 1>>::value;        // Z^H Y
    constexpr bool G2 = std::is_same<Epi, EpiGramOmega<T, 1>>::value;   // (Y^H Z, Y^H Y)
    constexpr bool TR = std::is_same<Epi, EpiTrace<T>>::value;          // tr(Z^H Y)
    constexpr bool TO = std::is_same<Epi, EpiTraceOmega<T>>::value;     // (tr(Y^H Z), tr(Y^H Y))
    constexpr bool VS = std::is_same<Epi, EpiVecSum<T>>::value;         // z^H Y 1
    const int s = ly.s;
    const int lane = threadIdx.x & 15, half = lane >> 3, l8 = lane & 7;
    const int w = threadIdx.x >> 6, g = (threadIdx.x >> 4) & 3;
    const int xcd = blockIdx.x & 7, q = blockIdx.x >> 3, nq = gridDim.x >> 3;
    const int r0 = xcd * rows_per_xcd;
    const int r1 = min(A.n, r0 + rows_per_xcd);
    const int step = nq * 64;
    constexpr bool DIRECT = TR || TO || VS;   // sums over rows: taken in the product's own lane layout
    constexpr bool TILE = EPI && !DIRECT;     // the Grams read the result back as 16 x 16 tiles
    const bool colok = 2 * l8 < s;          // s is even: both of the lane's columns exist, or neither
    const int cofs = colok ? 2 * l8 : 0;
    __shared__ T tiles[TILE ? kWaves : 1][TILE ? 16 * 17 : 1];
    __shared__ __align__(16) int ecol[kWaves][16][U];   // staged entries: [wave][row of the pass][slot]
    __shared__ __align__(16) T eval[kWaves][16][U];
    typename Epi::St st;
    epi.init(st);
    const int tc = threadIdx.x & 15, tq = (threadIdx.x >> 4) & 3;   // tile-16 layout of the epilogue
    // Software pipeline over the wave's 16-row steps: the next step's row
    // pointers, and then its first U entries per row, are loaded while this
    // step's X gathers are in flight, so a step waits on one round of memory
    // instead of three.  Rows, entries and the order of the sums are those of
    // the plain sweep, so the result is the same to the bit.
    // The row pointers are loaded unconditionally (rows past the end read the
    // last row's, then discarded): a load under a branch makes the compiler wait
    // for it at the branch's end, which would put one more memory round into
    // every step.
    auto rows_of = [&](int base, int (&i)[2], bool (&valid)[2], int (&k0)[2], int (&k1)[2]) {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            i[p] = base + 16 * w + 8 * p + 2 * g + half;
            valid[p] = i[p] < r1;
            const int ii = min(i[p], A.n - 1);
            const int a0 = A.rp[ii], a1 = A.rp[ii + 1];
            k0[p] = valid[p] ? a0 : 0;
            k1[p] = valid[p] ? a1 : 0;
        }
    };
    auto entries = [&](const int (&k0)[2], const int (&k1)[2], int off, int (&mc)[2], T (&ma)[2]) {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const int k = k0[p] + off + l8;
            const int kc = max(0, min(k, k1[p] - 1));   // clamped: always a valid entry
            mc[p] = __builtin_nontemporal_load(&A.ci[kc]);
            const T v = __builtin_nontemporal_load(&A.va[kc]);
            ma[p] = k < k1[p] ? v : T(0);
        }
    };
    int i[2], k0[2], k1[2], mc[2];
    bool valid[2];
    T ma[2];
    int base = r0 + q * 64;
    rows_of(base, i, valid, k0, k1);
    entries(k0, k1, 0, mc, ma);
    for (; base < r1; base += step) {
        const int wb = base + 16 * w;
        // The epilogue's second operand is loaded before the product, so that its
        // latency hides behind the gathers; rows past the end read row `base`
        // (< r1) instead and are zeroed.  Grams: at the tile entry
        // (wb + 4v + tq, tc).  Row sums: at the lane's own rows and columns.
        T zp[4] = {T(0), T(0), T(0), T(0)};
        if constexpr (G1 || G2) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = wb + 4 * v + tq;
                const bool ok = r < r1 && tc < s;
                const T zz = epi.Z[(size_t)(ok ? r : base) * s + (ok ? tc : 0)];
                zp[v] = ok ? zz : T(0);
            }
        }
        P2 zd[2];
        if constexpr (DIRECT) {
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const bool ok = valid[p] && colok;
                const int r = ok ? i[p] : base;
                if constexpr (VS) {
                    const T zz = epi.z[r];
                    zd[p].x = ok ? zz : T(0);
                } else {
                    const P2 zz = *reinterpret_cast<const P2*>(epi.Z + (size_t)r * s + cofs);
                    zd[p].x = ok ? zz.x : T(0);
                    zd[p].y = ok ? zz.y : T(0);
                }
            }
        }
        int ni[2], nk0[2], nk1[2], nmc[2];
        bool nvalid[2];
        T nma[2];
        rows_of(base + step, ni, nvalid, nk0, nk1);       // next step's row pointers
        double ax[2] = {0.0, 0.0}, ay[2] = {0.0, 0.0};   // FP64 accumulation, also for FP32 data
        for (int off = 0;; off += U) {
            int more = 0;
#pragma unroll
            for (int p = 0; p < 2; ++p) more |= k0[p] + off + U < k1[p];
            more = __any(more);
            // stage this round's entries: row 8p + 2g + half of the wave, slot l8
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                ecol[w][8 * p + 2 * g + half][l8] = mc[p];
                eval[w][8 * p + 2 * g + half][l8] = ma[p];
            }
            __builtin_amdgcn_wave_barrier();
            int cc[2][U];
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const int4* cr = reinterpret_cast<const int4*>(&ecol[w][8 * p + 2 * g + half][0]);
                const int4 c03 = cr[0], c47 = cr[1];
                cc[p][0] = c03.x; cc[p][1] = c03.y; cc[p][2] = c03.z; cc[p][3] = c03.w;
                cc[p][4] = c47.x; cc[p][5] = c47.y; cc[p][6] = c47.z; cc[p][7] = c47.w;
            }
            P2 xv[2][U];
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int u = 0; u < U; ++u) xv[p][u] = *reinterpret_cast<const P2*>(X + (size_t)cc[p][u] * s + cofs);
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const T* er = &eval[w][8 * p + 2 * g + half][0];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const T a = er[u];
                    ax[p] = fma((double)a, (double)xv[p][u].x, ax[p]);
                    ay[p] = fma((double)a, (double)xv[p][u].y, ay[p]);
                }
            }
            if (off == 0) entries(nk0, nk1, 0, nmc, nma);   // next step's first entries
            if (!more) break;
            __builtin_amdgcn_wave_barrier();                 // every read of this round precedes the next writes
            entries(k0, k1, off + U, mc, ma);                // rows longer than U: the rest in place
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            if (valid[p] && colok) {
                T* yr = Y + (size_t)i[p] * s + 2 * l8;
                __builtin_nontemporal_store((T)ax[p], yr);
                __builtin_nontemporal_store((T)ay[p], yr + 1);
            }
        }
        if constexpr (DIRECT) {
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                if (valid[p] && colok) {
                    const T y0 = (T)ax[p], y1 = (T)ay[p];   // the stored (rounded) values
                    if constexpr (VS) {
                        dot_acc(st.acc[0], zd[p].x, y0);
                        dot_acc(st.acc[0], zd[p].x, y1);
                    } else if constexpr (TR) {
                        dot_acc(st.acc[0], zd[p].x, y0);
                        dot_acc(st.acc[0], zd[p].y, y1);
                    } else {
                        dot_acc(st.acc[0], y0, zd[p].x);
                        dot_acc(st.acc[1], y0, y0);
                        dot_acc(st.acc[0], y1, zd[p].y);
                        dot_acc(st.acc[1], y1, y1);
                    }
                }
            }
        }
        if constexpr (TILE) {
            T* tw = tiles[w];
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const int lr = 8 * p + 2 * g + half;
                tw[lr * 17 + 2 * l8] = colok ? (T)ax[p] : T(0);       // the stored (rounded) values
                tw[lr * 17 + 2 * l8 + 1] = colok ? (T)ay[p] : T(0);
            }
            __builtin_amdgcn_wave_barrier();
            const Layout l16{s, 16, 4};
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int lr = 4 * v + tq;
                if constexpr (G1) {
                    const double zv[1] = {(double)zp[v]}, yv[1] = {(double)tw[lr * 17 + tc]};
                    st.g.add(zv, yv);
                } else if constexpr (G2) {
                    const double zv[1] = {(double)zp[v]}, yv[1] = {(double)tw[lr * 17 + tc]};
                    st.g1.add(yv, zv);
                    st.g2.add(yv, yv);
                } else {
                    const T y[1] = {tw[lr * 17 + tc]};
                    epi.row(st, wb + lr, wb + lr < r1, tc, l16, y);
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            i[p] = ni[p];
            valid[p] = nvalid[p];
            k0[p] = nk0[p];
            k1[p] = nk1[p];
            mc[p] = nmc[p];
            ma[p] = nma[p];
        }
    }
    epi_finish<Epi, 1>(epi, st, blockIdx.x, s);
}

__device__ inline double shfl_xor_v(double v, int off) { return __shfl_xor(v, off, 64); }
__device__ inline float shfl_xor_v(float v, int off) { return __shfl_xor(v, off, 64); }
__device__ inline c64 shfl_xor_v(c64 v, int off) { return {__shfl_xor(v.x, off, 64), __shfl_xor(v.y, off, 64)}; }
__device__ inline c32 shfl_xor_v(c32 v, int off) { return {__shfl_xor(v.x, off, 64), __shfl_xor(v.y, off, 64)}; }


// Single vector (s = 1): y = A x with 8 lanes per row.  Lane e of a row's group
// takes entries k0 + e, k0 + e + 8, ... and the 8 partial sums are added by a
// butterfly inside the group, in FP64 whatever the storage precision.  Same
// per-XCD row sweep as k_spmm_csr, software-pipelined like k_spmm_csr8: the
// next pass's row pointers (loaded unconditionally, clamped) and first entries
// are in flight while this pass's x gathers are; the order of the sums is that
// of the plain sweep.  (Two rows per 8-lane group and pass were measured too:
// no faster.)
template <class T>
__global__ __launch_bounds__(kBlock) void k_spmv_csr(const Ctl* ctl, CsrOp<T> A, int rows_per_xcd,
                                                      const T* __restrict__ x, T* __restrict__ y) {
    if (stopped(ctl)) return;
    using W = Val<T>;   // double or c64
    const int sub = threadIdx.x & 7;
    const int grp = threadIdx.x >> 3;                     // 32 rows per workgroup pass
    const int xcd = blockIdx.x & 7, q = blockIdx.x >> 3, nq = gridDim.x >> 3;
    const int r0 = xcd * rows_per_xcd;
    const int r1 = min(A.n, r0 + rows_per_xcd);
    const int step = nq * 32;
    auto row_of = [&](int base, int& i, bool& valid, int& k0, int& k1) {
        i = base + grp;
        valid = i < r1;                                   // uniform inside the 8-lane group
        const int ii = min(i, A.n - 1);
        const int a0 = A.rp[ii], a1 = A.rp[ii + 1];
        k0 = valid ? a0 : 0;
        k1 = valid ? a1 : 0;
    };
    auto first = [&](int k0, int k1, int& c, T& a) {     // the lane's first entry (a = 0 past the row's end)
        const int k = k0 + sub;
        const int kc = max(0, min(k, k1 - 1));
        c = A.ci[kc];
        const T v = A.va[kc];
        a = k < k1 ? v : zero<T>();
    };
    int base = r0 + q * 32;
    if (base >= r1) return;
    int i, k0, k1, c;
    bool valid;
    T a;
    row_of(base, i, valid, k0, k1);
    first(k0, k1, c, a);
    for (; base < r1; base += step) {
        int ni, nk0, nk1, nc;
        bool nvalid;
        T na;
        row_of(base + step, ni, nvalid, nk0, nk1);
        const W p0 = vfma(vup(a), vup(x[c]), vzero<W>());
        W acc = k0 + sub < k1 ? p0 : vzero<W>();   // a lane past the row's end adds nothing
        for (int k = k0 + sub + 8; k < k1; k += 8) acc = vfma(vup(A.va[k]), vup(x[A.ci[k]]), acc);
        first(nk0, nk1, nc, na);
        acc = acc + shfl_xor_v(acc, 4);
        acc = acc + shfl_xor_v(acc, 2);
        acc = acc + shfl_xor_v(acc, 1);
        if (valid && sub == 0) y[i] = vdown<T>(acc);
        i = ni;
        valid = nvalid;
        k0 = nk0;
        k1 = nk1;
        c = nc;
        a = na;
    }
}

// Non-temporal load of one stored value (complex values as a 2-vector).
template <class T> __device__ inline T nt_value(const T* p) { return __builtin_nontemporal_load(p); }
template <> __device__ inline c64 nt_value<c64>(const c64* p) {
    typedef double v2 __attribute__((ext_vector_type(2)));
    const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
    return {v.x, v.y};
}
template <> __device__ inline c32 nt_value<c32>(const c32* p) {
    typedef float v2 __attribute__((ext_vector_type(2)));
    const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
    return {v.x, v.y};
}

// SELL-C-sigma product with the CSR kernels' techniques.  16 lanes per row
// (lane l holds columns l + 16 j, j < J); a workgroup takes 16 consecutive
// sorted positions of a chunk per pass (4 per wave) and walks its chunks in
// order.  A chunk stores slot k of its rows contiguously, so the entries of a
// wave's 4 rows for 8 slots are 32 loads of consecutive words (lanes 0..31),
// staged in LDS and read back by the 16 lanes of each row (an LDS broadcast).
// The sweep is software-pipelined: the next round's entries (next 8 slots,
// or the first 8 of the next pass) are loaded while this round's X gathers
// are in flight.  Padding slots (value 0, the row's own column) are gathered
// and multiplied like stored entries; their terms are exact zeros.  Y is
// written at the original row of each sorted position.
template <class T, int J, class Epi>
__global__ __launch_bounds__(kBlock) void k_spmm_sell16(const Ctl* ctl, SellOp<T> A, Layout ly, int chunks_per_block,
                                                         const T* __restrict__ X, T* __restrict__ Y, Epi epi) {
    if (stopped(ctl)) return;
    constexpr int U = 8;
    const int lane = threadIdx.x & 15, rr = (threadIdx.x >> 4) & 3, w = threadIdx.x >> 6, lw = threadIdx.x & 63;
    const int s = ly.s, C = A.C;
    const int nchunks = (A.n + C - 1) / C;
    const int cb = xcd_chunk(blockIdx.x, gridDim.x) * chunks_per_block;
    const int ce = min(nchunks, cb + chunks_per_block);
    __shared__ __align__(16) int ecol[kWaves][U][4];
    __shared__ __align__(16) T eval[kWaves][U][4];
    int col[J];
#pragma unroll
    for (int j = 0; j < J; ++j) col[j] = min(lane + 16 * j, s - 1);
    typename Epi::St st;
    epi.init(st);
    // a round: chunk ch, pass r0 (rows r0 .. r0 + 15 of the chunk), slots k .. k + U - 1
    struct Round { int ch, r0, k, width, e0; };
    auto chunk_round = [&](int ch) {
        Round q{ch, 0, 0, 0, 0};
        if (ch < ce) {
            q.width = A.clen[ch];
            q.e0 = A.cptr[ch];
        }
        return q;
    };
    auto next_round = [&](Round q) {
        q.k += U;
        if (q.k >= q.width) {
            q.k = 0;
            q.r0 += 16;
            if (q.r0 >= C) q = chunk_round(q.ch + 1);
        }
        return q;
    };
    // lane lw < 32 loads slot k + lw / 4 of row r0 + 4 w + lw % 4; other lanes and
    // slots past the chunk's width read slot 0 of the array (always allocated)
    // with value 0
    auto load_round = [&](const Round& q, int& mc, T& ma) {
        const int kk = q.k + (lw >> 2);
        const bool ok = q.ch < ce && lw < 32 && kk < q.width;
        const int e = ok ? q.e0 + kk * C + q.r0 + 4 * w + (lw & 3) : 0;
        mc = __builtin_nontemporal_load(&A.ci[e]);
        const T v = nt_value(&A.va[e]);
        ma = ok ? v : zero<T>();
    };
    Round cur = chunk_round(cb);
    while (cur.ch < ce && cur.width == 0) {   // chunks of empty rows: write zeros
        for (int r0 = 0; r0 < C; r0 += 16) {
            const int pos = cur.ch * C + r0 + 4 * w + rr;
            const bool valid = pos < A.n;
            T acc[J];
#pragma unroll
            for (int j = 0; j < J; ++j) acc[j] = zero<T>();
            const int i = valid ? A.row[pos] : 0;
            if (valid) {
#pragma unroll
                for (int j = 0; j < J; ++j)
                    if (lane + 16 * j < s) Y[(size_t)i * s + lane + 16 * j] = acc[j];
            }
            epi.row(st, i, valid, lane, ly, acc);
        }
        cur = chunk_round(cur.ch + 1);
    }
    int mc = 0;
    T ma = zero<T>();
    if (cur.ch < ce) load_round(cur, mc, ma);
    T acc[J];
#pragma unroll
    for (int j = 0; j < J; ++j) acc[j] = zero<T>();
    while (cur.ch < ce) {
        if (lw < 32) {                            // lanes 0..31 hold this round's entries
            ecol[w][lw >> 2][lw & 3] = mc;
            eval[w][lw >> 2][lw & 3] = ma;
        }
        __builtin_amdgcn_wave_barrier();
        int cc[U];
        T av[U];
#pragma unroll
        for (int u = 0; u < U; ++u) cc[u] = ecol[w][u][rr];
        T xv[U][J];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < J; ++j) xv[u][j] = X[(size_t)cc[u] * s + col[j]];
        Round nxt = next_round(cur);
        int nmc = 0;
        T nma = zero<T>();
        if (nxt.ch < ce) load_round(nxt, nmc, nma);     // next round's entries, behind the gathers
#pragma unroll
        for (int u = 0; u < U; ++u) av[u] = eval[w][u][rr];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < J; ++j) acc[j] = fma_(av[u], xv[u][j], acc[j]);
        __builtin_amdgcn_wave_barrier();                 // every read of this round precedes the next writes
        if (nxt.ch != cur.ch || nxt.r0 != cur.r0) {      // the pass ends: store its rows
            const int pos = cur.ch * C + cur.r0 + 4 * w + rr;
            const bool valid = pos < A.n;
            const int i = valid ? A.row[pos] : 0;
            if (valid) {
#pragma unroll
                for (int j = 0; j < J; ++j)
                    if (lane + 16 * j < s) Y[(size_t)i * s + lane + 16 * j] = acc[j];
            }
            epi.row(st, i, valid, lane, ly, acc);
#pragma unroll
            for (int j = 0; j < J; ++j) acc[j] = zero<T>();
            // chunks of empty rows after this one
            while (nxt.ch < ce && nxt.width == 0) {
                for (int r0 = 0; r0 < C; r0 += 16) {
                    const int p2 = nxt.ch * C + r0 + 4 * w + rr;
                    const bool v2 = p2 < A.n;
                    T z[J];
#pragma unroll
                    for (int j = 0; j < J; ++j) z[j] = zero<T>();
                    const int i2 = v2 ? A.row[p2] : 0;
                    if (v2) {
#pragma unroll
                        for (int j = 0; j < J; ++j)
                            if (lane + 16 * j < s) Y[(size_t)i2 * s + lane + 16 * j] = z[j];
                    }
                    epi.row(st, i2, v2, lane, ly, z);
                }
                nxt = chunk_round(nxt.ch + 1);
                if (nxt.ch < ce) load_round(nxt, nmc, nma);
            }
        }
        cur = nxt;
        mc = nmc;
        ma = nma;
    }
    epi_finish<Epi, J>(epi, st, blockIdx.x, s);
}

}  // namespace skr
