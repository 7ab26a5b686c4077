// Kernels of the block family with QR of the block residuals: Bl-BiCG-rQ
// (Algorithm 5, eqs. (newalpha)-(newbetahat)) and Bl-BiCGStab-rQ (Section 4,
// closing paragraph), plus the thin QR they rely on.
//
// Layout ("tile-16"): a workgroup handles 16 rows per pass, 16 lanes per row,
// lane l owning columns l + 16 j (j < J, J = ceil(s/16)).  Block updates with
// an s x s coefficient matrix M (Out = A + B M, the BLAS3 updates the paper
// notes after Proposition 1) stage the 16 x s row tile of B in LDS and read M
// from LDS.  Gram matrices (Y^H X, s x s) are accumulated with FP64 MFMA in the
// same pass that produces their operands.
//
// Thin QR (Section 4: R = Q C with Q^H Q = I) is CholeskyQR2: G = Z^H Z = S1^H S1,
// Q1 = Z S1^{-1}, G1 = Q1^H Q1 = S2^H S2, Q = Q1 S2^{-1}, C = S2 S1.  If the
// first Cholesky factorisation fails, the first pass is repeated with the shift
// 11 (n s + s(s+1)) u tr(G) (shifted CholeskyQR, Fukaya et al. 2020) and one
// more unshifted pass is added (CholeskyQR3).  Q1 is never stored: each pass
// recomputes the rows Z S1^{-1} S2^{-1} ... with the same sequence of row x
// triangle products, so every Gram matrix is taken from exactly the rows the
// next factor corrects.
#pragma once

#include "common.hpp"
#include "glk.hpp"
#include "small.hpp"

#include <type_traits>

namespace skr {

// ---------------------------------------------------------------- mats slots
// Every block method keeps its s x s matrices in one device array `mats`
// (slot k at mats + k*s*s, complex FP64).
enum {
    M_C = 0, M_CH, M_M, M_G, M_ALPHA, M_ALPHAH, M_ALPHAC, M_BETA, M_BETAH,
    M_S1, M_S1INV, M_S12, M_S2INV, M_S, M_S3INV,          // QR slot 0 work (M_S: R factor)
    M_T1, M_T1INV, M_T12, M_T2INV, M_T, M_T3INV,          // QR slot 1 work (M_T: R factor)
    M_N, M_A, M_AC, M_WC, M_B, M_RB, M_TMP,
    M_G1, M_RR, M_RHR, M_RT, M_W, M_MW,                   // plain Bl-BiCG / Bl-BiCGStab / Li-BiCG
    // Li-QMR: per-column scalars on the diagonals, the identity and its negative
    M_QRHO, M_QXI, M_QDELTA, M_QEPS, M_QBETA, M_QGAMMA, M_QTHETA, M_QETA, M_QF,
    M_QRHON, M_QXIN, M_QDELTAN, M_QIRHO, M_QIXI, M_QMB, M_QMBC, M_QMCP, M_QMCQ,
    M_QVV, M_QWW, M_QWV, M_ID, M_MID,
    M_COUNT
};
enum { SC_GAMMA = 40, SC_OMEGA = 41, SC_PIV = 48 };   // scalars / pivots inside sc[]

struct Tile16 {
    int n, s, rpc;
};

#define SKR_TILE_LOOP(tl)                                                              \
    const int lane = threadIdx.x & 15;                                                 \
    const int grp = threadIdx.x >> 4;                                                  \
    const int r0_ = xcd_chunk(blockIdx.x, gridDim.x) * (tl).rpc;                       \
    const int r1_ = min((tl).n, r0_ + (tl).rpc);                                       \
    for (int base_ = r0_; base_ < r1_; base_ += 16)

// Row passes handled together by one lane group in the streaming block kernels
// (their loads are issued before any is used, to keep loads in flight).
template <class T, int J> struct RowPasses { static constexpr int value = Tr<T>::cplx ? (J == 1 ? 2 : 1) : (J == 1 ? 4 : 2); };

#define SKR_TILE_LOOP_RP(tl, RP)                                                       \
    const int lane = threadIdx.x & 15;                                                 \
    const int grp = threadIdx.x >> 4;                                                  \
    const int r0_ = xcd_chunk(blockIdx.x, gridDim.x) * (tl).rpc;                       \
    const int r1_ = min((tl).n, r0_ + (tl).rpc);                                       \
    for (int base_ = r0_; base_ < r1_; base_ += 16 * (RP))

__device__ inline double vmul(c64 a, double b) { return a.x * b; }
__device__ inline c64 vmul(c64 a, c64 b) { return a * b; }
__device__ inline double vfrom(c64 a, double) { return a.x; }
__device__ inline c64 vfrom(c64 a, c64) { return a; }

// Loads are unconditional (row 0 / column s-1 stand in for out-of-range
// positions) and the value is zeroed afterwards, so no branch separates them.
template <class T, int J>
__device__ inline void load_row(const T* P, int i, bool valid, int lane, int s, Val<T> (&v)[J]) {
    const size_t ib = (size_t)(valid ? i : 0) * s;
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int c = lane + 16 * j;
        const Val<T> x = vup(P[ib + min(c, s - 1)]);
        v[j] = (valid && c < s) ? x : vzero<Val<T>>();
    }
}
template <class T, int J>
__device__ inline void store_row(T* P, int i, bool valid, int lane, int s, const Val<T> (&v)[J]) {
    if (!valid) return;
#pragma unroll
    for (int j = 0; j < J; ++j) {
        int c = lane + 16 * j;
        if (c < s) P[(size_t)i * s + c] = vdown<T>(v[j]);
    }
}
// tile[grp][:] = v (this lane's entries)
template <class Vt, int J>
__device__ inline void put_tile(Vt* tile, int grp, int lane, int s, const Vt (&v)[J]) {
#pragma unroll
    for (int j = 0; j < J; ++j) {
        int c = lane + 16 * j;
        if (c < s) tile[grp * s + c] = v[j];
    }
}
// an s x s FP64 coefficient matrix (complex FP64 in device memory) copied into LDS
template <class Vt>
__device__ inline void lds_load_mat(Vt* dst, const c64* __restrict__ src, int s) {
    for (int e = threadIdx.x; e < s * s; e += kBlock) dst[e] = vfrom(src[e], Vt{});
}

// Broadcast of lane N of each 16-lane row (DPP row_newbcast, gfx90a and later):
// inside a tile-16 row group this hands every lane the row's entry of column N
// without LDS or a barrier.
template <int N>
__device__ inline double rbc(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), 0x150 + N, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x150 + N, 0xF, 0xF, false);
    return __builtin_bit_cast(double, (long long)(unsigned)lo | ((long long)hi << 32));
}
template <int N>
__device__ inline c64 rbc(c64 v) { return {rbc<N>(v.x), rbc<N>(v.y)}; }

// value of lane `src` of this lane's 16-lane row group
__device__ inline double shfl16(double v, int src) { return __shfl(v, src, 16); }
__device__ inline c64 shfl16(c64 v, int src) { return {__shfl(v.x, src, 16), __shfl(v.y, src, 16)}; }

template <int A, int END, class F>
__device__ inline void static_for(F&& f) {
    if constexpr (A < END) {
        f(std::integral_constant<int, A>{});
        static_for<A + 1, END>(f);
    }
}

// Row x coefficient matrix: out[j] += sum_a x_a M[a][lane + 16 j], where x_a is
// column a of this lane's row, held by lane a % 16 of the row group in
// register a / 16 (padding columns are zero).  Real blocks with s <= 16 keep
// this lane's column of M in registers; otherwise M is read from LDS.  Output
// padding columns are set to zero.
template <class T, int J>
struct Coef {
    using VV = Val<T>;
    static constexpr bool REG = !Tr<T>::cplx && J == 1;
    double m[REG ? 16 : 1];
    const VV* M;
    int s;
    __device__ inline void load(const VV* Mlds, int s_, int lane) {
        M = Mlds;
        s = s_;
        if constexpr (REG) {
#pragma unroll
            for (int a = 0; a < 16; ++a) m[a] = (a < s && lane < s) ? (double)Mlds[a * s + lane] : 0.0;
        }
    }
    __device__ inline void apply(const VV (&x)[J], int lane, VV (&out)[J]) const {
        if constexpr (REG) {
            double acc = out[0];
            static_for<0, 16>([&](auto ic) {
                constexpr int a = decltype(ic)::value;
                acc = fma(rbc<a>(x[0]), m[a], acc);
            });
            out[0] = acc;
        } else {
            // rolled loop over the s coefficients (a full unroll of 16 J
            // broadcasts would keep too many values live); column a of the row
            // comes from lane a % 16 of the row group by a lane shuffle
            int cc[J];
#pragma unroll
            for (int j = 0; j < J; ++j) cc[j] = min(lane + 16 * j, s - 1);
            for (int a = 0; a < s; ++a) {
                const VV xa = shfl16((J == 1 || a < 16) ? x[0] : x[J - 1], a & 15);
                const int ar = a * s;
#pragma unroll
                for (int j = 0; j < J; ++j) out[j] = vfma(xa, M[ar + cc[j]], out[j]);
            }
#pragma unroll
            for (int j = 0; j < J; ++j)
                if (lane + 16 * j >= s) out[j] = vzero<VV>();
        }
    }
};

// ---------------------------------------------------------------- Gram
// part[b] = L^H R over this workgroup's rows
template <class T, int J>
__global__ __launch_bounds__(kBlock) void k_bl_gram(const Ctl* ctl, Tile16 tl, const T* __restrict__ Lm,
                                                    const T* __restrict__ Rm, c64* part, int pstride = 0,
                                                    int poff = 0) {
    if (stopped(ctl)) return;
    constexpr int RP = RowPasses<T, J>::value;
    GramAcc<J, Tr<T>::cplx> g;
    g.clear();
    SKR_TILE_LOOP_RP(tl, RP) {
        Val<T> l[RP][J], r[RP][J];
#pragma unroll
        for (int p = 0; p < RP; ++p) {
            const int i = base_ + 16 * p + grp;
            load_row<T, J>(Lm, i, i < r1_, lane, tl.s, l[p]);
            load_row<T, J>(Rm, i, i < r1_, lane, tl.s, r[p]);
        }
#pragma unroll
        for (int p = 0; p < RP; ++p) g.add(l[p], r[p]);
    }
    __shared__ c64 lds[(16 * J) * (16 * J)];
    g.store(tl.s, lds, part + (size_t)blockIdx.x * (pstride > 0 ? pstride : tl.s * tl.s) + poff);
}

// Second reduction stage: per-workgroup partials [np][E] -> out[E].  One wave
// per element: lane l sums partials l, l + 64, l + 128, ... into eight
// independent accumulators (so eight loads are in flight), then the wave sums
// its lanes by a butterfly.  The order is fixed, so results are reproducible.
__global__ __launch_bounds__(kBlock) void k_reduce_parts(const Ctl* ctl, int cond_slot, const c64* __restrict__ part,
                                                         int np, int E, c64* __restrict__ out) {
    if (stopped(ctl)) return;
    if (cond_slot >= 0 && !ctl->qr_shift[cond_slot]) return;
    const int e = blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (e >= E) return;   // uniform per wave
    const int l = threadIdx.x & 63;
    c64 a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = {0.0, 0.0};
    int b = l;
    for (; b + 7 * 64 < np; b += 8 * 64) {
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = a[u] + part[(size_t)(b + 64 * u) * E + e];
    }
    for (; b < np; b += 64) a[0] = a[0] + part[(size_t)b * E + e];
    c64 t = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    t.x = wave_sum(t.x);
    t.y = wave_sum(t.y);
    if (l == 0) out[e] = t;
}

// final sum of the stage-2 partials into LDS
__device__ inline void gram_final(const c64* __restrict__ part2, int p2, int E, c64* dst) {
    for (int e = threadIdx.x; e < E; e += blockDim.x) {
        c64 acc = part2[e];
        for (int y = 1; y < p2; ++y) acc = acc + part2[(size_t)y * E + e];
        dst[e] = acc;
    }
    __syncthreads();
}

// ---------------------------------------------------------------- triangular pass
enum { TRI_WRITE = 1, TRI_G_OUT_OUT = 2, TRI_G_OTHER_OUT = 4, TRI_G_OUT_OTHER = 8 };

// ------------------------------------------------ real s <= 16: MFMA row tiles
// A wave owns 16 consecutive rows.  Lane L = c + 16 q holds, in register v, the
// element (row 4v + q, column c) of the tile: four coalesced 16-column loads,
// and also the layout of an MFMA f64 16x16x4 result, D[4v + q][c] in lane
// c + 16 q, register v.  The product of the tile with an s x s matrix M is
// four MFMAs whose A operand (lane c + 16 q: tile[c][4t + q]) is read back
// transposed through a per-wave LDS tile, and whose B operand (lane c + 16 q:
// M[4t + q][c]) stays in registers.  Padding rows and columns are zero.
constexpr int kTileLd = 17;   // padded LDS row: transposed reads are bank-spread

// B operand of M (complex FP64 storage, real part) for the four k-slabs
__device__ inline void mfma_bop(const c64* __restrict__ Mg, int s, int c, int q, double (&m)[4]) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int k = 4 * t + q;
        m[t] = (k < s && c < s) ? Mg[k * s + c].x : 0.0;
    }
}
// returns X M for the wave's tile X (x[v] = X[4v + q][c]); tw: this wave's LDS tile
__device__ inline d4 mfma_apply(const double (&x)[4], const double (&m)[4], double* tw, int c, int q) {
#pragma unroll
    for (int v = 0; v < 4; ++v) tw[(4 * v + q) * kTileLd + c] = x[v];
    __builtin_amdgcn_wave_barrier();
    d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < 4; ++t) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(tw[c * kTileLd + 4 * t + q], m[t], acc, 0, 0, 0);
    __builtin_amdgcn_wave_barrier();
    return acc;
}
// the wave's tile rows of P (row stride s) as x[v] = P[b + 4v + q][c]; zero
// outside rows [b, r1) and columns [0, s).  Loads are clamped, not branched.
template <class T>
__device__ inline void tile_load(const T* P, int b, int r1, int s, int c, int q, double (&x)[4]) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = b + 4 * v + q;
        const bool ok = i < r1 && c < s;
        const double val = (double)ld_nt(&P[(size_t)(ok ? i : b) * s + (ok ? c : 0)]);
        x[v] = ok ? val : 0.0;
    }
}
template <class T>
__device__ inline void tile_store(T* P, int b, int r1, int s, int c, int q, const d4& x) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = b + 4 * v + q;
        if (i < r1 && c < s) P[(size_t)i * s + c] = (T)x[v];
    }
}

// CholeskyQR triangular pass, real blocks with s <= 16: out = Z S1^{-1} S2^{-1}
// [S3^{-1}], the first `nchain` inverse factors of QR slot `slot` applied one
// after the other, plus S3^{-1} when `add_shift` and the slot used the shifted
// first pass; cond: run only when the shifted pass was used; mode: write out
// (TRI_WRITE) and/or accumulate a Gram of out (TRI_G_*).  Out may alias Z (each
// tile is read before it is written, by the same lanes).  NC: the
// most inverse factors this instance applies (1 or 3); OTH: whether the Gram's
// second operand is another block (fewer live registers when it is not).
template <class T, int NC, bool OTH>
__global__ __launch_bounds__(kBlock) void k_bl_tri16(const Ctl* ctl, int slot, int cond, int nchain, int add_shift,
                                                     Tile16 tl, int mode, const c64* __restrict__ mats, const T* Z,
                                                     T* Out, const T* __restrict__ Other, c64* part) {
    if (stopped(ctl)) return;
    const int shifted = ctl->qr_shift[slot];
    if (cond && !shifted) return;
    const int nc = nchain + (add_shift && shifted ? 1 : 0);
    const int s = tl.s, ss = s * s;
    const int base = slot == 0 ? M_S1 : M_T1;
    const int L = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int c = L & 15, q = L >> 4;
    double m0[4], m1[NC > 1 ? 4 : 1], m2[NC > 1 ? 4 : 1];
    mfma_bop(mats + (size_t)(base + 1) * ss, s, c, q, m0);
    if constexpr (NC > 1) {
        mfma_bop(mats + (size_t)(base + 3) * ss, s, c, q, m1);
        mfma_bop(mats + (size_t)(base + 5) * ss, s, c, q, m2);
    }
    __shared__ double tiles[kWaves][16 * kTileLd];
    __shared__ c64 glds[256];
    double* tw = tiles[w];
    GramAcc<1, false> g;
    g.clear();
    const int r0 = xcd_chunk(blockIdx.x, gridDim.x) * tl.rpc;
    const int r1 = min(tl.n, r0 + tl.rpc);
    // software pipelining: the next tile's loads are issued before this tile's MFMAs
    constexpr bool oth = OTH;
    double xn[4], otn[4] = {0.0, 0.0, 0.0, 0.0};
    int b = r0 + 16 * w;
    if (b < r1) {
        tile_load<T>(Z, b, r1, s, c, q, xn);
        if (oth) tile_load<T>(Other, b, r1, s, c, q, otn);
    }
    for (; b < r1; b += 16 * kWaves) {
        double x[4], ot[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            x[v] = xn[v];
            ot[v] = otn[v];
        }
        const int bn = b + 16 * kWaves;
        if (bn < r1) {
            tile_load<T>(Z, bn, r1, s, c, q, xn);
            if (oth) tile_load<T>(Other, bn, r1, s, c, q, otn);
        }
        d4 o = mfma_apply(x, m0, tw, c, q);
        if constexpr (NC > 1) {
            if (nc > 1) {
                double y[4] = {o[0], o[1], o[2], o[3]};
                o = mfma_apply(y, m1, tw, c, q);
            }
            if (nc > 2) {
                double y[4] = {o[0], o[1], o[2], o[3]};
                o = mfma_apply(y, m2, tw, c, q);
            }
        }
        if (mode & TRI_WRITE) tile_store<T>(Out, b, r1, s, c, q, o);
        if (mode & (TRI_G_OUT_OUT | TRI_G_OTHER_OUT | TRI_G_OUT_OTHER)) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double ov[1] = {o[v]};
                if (!OTH) {
                    g.add(ov, ov);
                } else {
                    const double tv[1] = {ot[v]};
                    if (mode & TRI_G_OTHER_OUT) g.add(tv, ov);
                    else g.add(ov, tv);
                }
            }
        }
    }
    if (mode & (TRI_G_OUT_OUT | TRI_G_OTHER_OUT | TRI_G_OUT_OTHER)) {
        __syncthreads();
        g.store(s, glds, part + (size_t)blockIdx.x * s * s);
    }
}

// Out = A + (B + gamma C) M [+ part = Out^H Out] for real blocks with s <= 16;
// A or C may be null; Out may alias A or B.
template <class T, bool GRAM>
__global__ __launch_bounds__(kBlock) void k_bl_axpm16(const Ctl* ctl, Tile16 tl, const c64* __restrict__ mats,
                                                      int mslot, const c64* __restrict__ sc, int gslot, const T* A,
                                                      const T* B, const T* __restrict__ Cm, T* Out, c64* part) {
    if (stopped(ctl)) return;
    const int s = tl.s;
    const int L = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int c = L & 15, q = L >> 4;
    double m[4];
    mfma_bop(mats + (size_t)mslot * s * s, s, c, q, m);
    const double gamma = Cm ? sc[gslot].x : 0.0;
    __shared__ double tiles[kWaves][16 * kTileLd];
    __shared__ c64 glds[256];
    double* tw = tiles[w];
    GramAcc<1, false> g;
    g.clear();
    const int r0 = xcd_chunk(blockIdx.x, gridDim.x) * tl.rpc;
    const int r1 = min(tl.n, r0 + tl.rpc);
    // software pipelining of the B stream (Out may alias B: a tile is loaded
    // one iteration before it is written, and later tiles are never written early)
    double xn[4];
    int b = r0 + 16 * w;
    if (b < r1) tile_load<T>(B, b, r1, s, c, q, xn);
    for (; b < r1; b += 16 * kWaves) {
        double x[4], a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int v = 0; v < 4; ++v) x[v] = xn[v];
        if (b + 16 * kWaves < r1) tile_load<T>(B, b + 16 * kWaves, r1, s, c, q, xn);
        if (Cm) {
            double y[4];
            tile_load<T>(Cm, b, r1, s, c, q, y);
#pragma unroll
            for (int v = 0; v < 4; ++v) x[v] = fma(gamma, y[v], x[v]);
        }
        if (A) tile_load<T>(A, b, r1, s, c, q, a);
        d4 o = mfma_apply(x, m, tw, c, q);
#pragma unroll
        for (int v = 0; v < 4; ++v) o[v] += a[v];
        tile_store<T>(Out, b, r1, s, c, q, o);
        if (GRAM) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double ov[1] = {o[v]};
                g.add(ov, ov);
            }
        }
    }
    if (GRAM) {
        __syncthreads();
        g.store(s, glds, part + (size_t)blockIdx.x * s * s);
    }
}

// Bl-BiCG-rQ, real blocks with s <= 16: X += V (alpha C); Z = Q - W alpha;
// part = Z^H Z.  mats holds -alpha.
template <class T>
__global__ __launch_bounds__(kBlock) void k_blrq_updz16(const Ctl* ctl, Tile16 tl, const c64* __restrict__ mats,
                                                        T* __restrict__ X, const T* __restrict__ Vb,
                                                        const T* __restrict__ Q, const T* __restrict__ W,
                                                        T* __restrict__ Z, c64* part) {
    if (stopped(ctl)) return;
    const int s = tl.s;
    const int L = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int c = L & 15, q = L >> 4;
    double ma[4], mac[4];
    mfma_bop(mats + (size_t)M_ALPHA * s * s, s, c, q, ma);     // -alpha
    mfma_bop(mats + (size_t)M_ALPHAC * s * s, s, c, q, mac);   // alpha C
    __shared__ double tiles[kWaves][16 * kTileLd];
    __shared__ c64 glds[256];
    double* tw = tiles[w];
    GramAcc<1, false> g;
    g.clear();
    const int r0 = xcd_chunk(blockIdx.x, gridDim.x) * tl.rpc;
    const int r1 = min(tl.n, r0 + tl.rpc);
    for (int b = r0 + 16 * w; b < r1; b += 16 * kWaves) {
        double v[4], wv[4], x[4], z[4];
        tile_load<T>(Vb, b, r1, s, c, q, v);
        tile_load<T>(W, b, r1, s, c, q, wv);
        tile_load<T>(X, b, r1, s, c, q, x);
        tile_load<T>(Q, b, r1, s, c, q, z);
        d4 xo = mfma_apply(v, mac, tw, c, q);
        d4 zo = mfma_apply(wv, ma, tw, c, q);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            xo[u] += x[u];
            zo[u] += z[u];
        }
        tile_store<T>(X, b, r1, s, c, q, xo);
        tile_store<T>(Z, b, r1, s, c, q, zo);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double zv[1] = {zo[u]};
            g.add(zv, zv);
        }
    }
    __syncthreads();
    g.store(s, glds, part + (size_t)blockIdx.x * s * s);
}

// Bl-BiCGStab-rQ, real blocks with s <= 16: X += U (a C) + S~ (omega C);
// Z = S~ - omega T~; part = Z^H Z.
template <class T>
__global__ __launch_bounds__(kBlock) void k_blst_upd16(const Ctl* ctl, Tile16 tl, const c64* __restrict__ mats,
                                                       const c64* __restrict__ sc, T* __restrict__ X,
                                                       const T* __restrict__ U, const T* __restrict__ St,
                                                       const T* __restrict__ Tt, T* __restrict__ Z, c64* part) {
    if (stopped(ctl)) return;
    const int s = tl.s;
    const int L = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int c = L & 15, q = L >> 4;
    double mac[4], mwc[4];
    mfma_bop(mats + (size_t)M_AC * s * s, s, c, q, mac);   // a C
    mfma_bop(mats + (size_t)M_WC * s * s, s, c, q, mwc);   // omega C
    const double mw = -sc[SC_OMEGA].x;
    __shared__ double tiles[kWaves][16 * kTileLd];
    __shared__ c64 glds[256];
    double* tw = tiles[w];
    GramAcc<1, false> g;
    g.clear();
    const int r0 = xcd_chunk(blockIdx.x, gridDim.x) * tl.rpc;
    const int r1 = min(tl.n, r0 + tl.rpc);
    for (int b = r0 + 16 * w; b < r1; b += 16 * kWaves) {
        double u[4], st[4], tt[4], x[4];
        tile_load<T>(U, b, r1, s, c, q, u);
        tile_load<T>(St, b, r1, s, c, q, st);
        tile_load<T>(Tt, b, r1, s, c, q, tt);
        tile_load<T>(X, b, r1, s, c, q, x);
        d4 xa = mfma_apply(u, mac, tw, c, q);
        d4 xb = mfma_apply(st, mwc, tw, c, q);
        d4 z;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            xa[v] = (x[v] + xa[v]) + xb[v];
            z[v] = fma(mw, tt[v], st[v]);
        }
        tile_store<T>(X, b, r1, s, c, q, xa);
        tile_store<T>(Z, b, r1, s, c, q, z);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const double zv[1] = {z[v]};
            g.add(zv, zv);
        }
    }
    __syncthreads();
    g.store(s, glds, part + (size_t)blockIdx.x * s * s);
}

// ---------------------------------------------------------------- coefficient kernels
// Dynamic LDS: 6 s x s matrices.
__device__ inline void set_bd(Ctl* c) { set_breakdown(c); }

// CholeskyQR factor kernels for QR slot `slot` (reduced Gram in part2):
// pass 1: G = Z^H Z -> S1 (shifted if the plain factorisation fails), S1^{-1};
// pass 2: G = Q1^H Q1 -> S2, S2^{-1}; S12 = S2 S1, the R factor S = S12 unless shifted;
// pass 3 (shifted case only): G = Q2^H Q2 -> S3, S3^{-1}; S = S3 S12.
// `u` is the unit roundoff of the stored blocks (2^-53 for FP64, 2^-24 for the
// FP32 inner solves).  The Gram itself is always accumulated in FP64, so the
// shift that makes the Cholesky factorisation succeed is Fukaya et al.'s
// 11 (ns + s(s+1)) 2^-53 tr(G); it is raised to 1e3 u tr(G) where that is
// larger, so that the shifted Q1 (condition number <= (1e3 u)^{-1/2}) is still
// orthonormal enough, in the stored precision, for the two passes after it.
__global__ __launch_bounds__(kCoefThreads) void k_qr_chol(Ctl* c, int slot, int pass, int n, int s, const c64* __restrict__ part2, int p2,
                          c64* __restrict__ mats, double u) {
    if (stopped(c)) return;
    if (pass == 3 && !c->qr_shift[slot]) return;
    extern __shared__ c64 dyn[];
    __shared__ int flag;
    const int ss = s * s;
    c64* G = dyn;
    c64* A = dyn + ss;
    c64* B = dyn + 2 * ss;
    c64* D = dyn + 3 * ss;
    const int base = slot == 0 ? M_S1 : M_T1;
    c64* mS1 = mats + (size_t)(base + 0) * ss;
    c64* mS1i = mats + (size_t)(base + 1) * ss;
    c64* mS12 = mats + (size_t)(base + 2) * ss;
    c64* mS2i = mats + (size_t)(base + 3) * ss;
    c64* mS = mats + (size_t)(base + 4) * ss;
    c64* mS3i = mats + (size_t)(base + 5) * ss;
    gram_final(part2, p2, ss, G);
    if (pass == 1) {
        if (threadIdx.x == 0) c->qr_shift[slot] = 0;
        sm_copy(A, G, ss);
        int ok = sm_cholesky(A, s, 0.0, &flag, 1e4 * u);
        if (!ok) {
            double trg = 0.0;
            for (int i = 0; i < s; ++i) trg += G[i * s + i].x;
            double shift = fmax(11.0 * ((double)n * s + (double)s * (s + 1)) * 0x1p-53, 1e3 * u) * trg;
            sm_copy(A, G, ss);
            ok = sm_cholesky(A, s, shift, &flag, fmax(1e2 * u, 1e-12));
            if (threadIdx.x == 0) c->qr_shift[slot] = 1;
            __syncthreads();
        }
        if (!ok) {
            if (threadIdx.x == 0) set_bd(c);
            return;
        }
        sm_tri_inv_upper(A, B, s);
        for (int e = threadIdx.x; e < ss; e += blockDim.x) {
            mS1[e] = A[e];
            mS1i[e] = B[e];
        }
        return;
    }
    sm_copy(A, G, ss);
    int ok = sm_cholesky(A, s, 0.0, &flag, fmax(1e2 * u, 1e-12));
    if (!ok) {
        if (threadIdx.x == 0) set_bd(c);
        return;
    }
    sm_tri_inv_upper(A, B, s);   // B = S_k^{-1}
    sm_copy(G, pass == 2 ? mS1 : mS12, ss);
    sm_gemm(D, A, 0, G, 0, s);   // S_k * (previous product)
    c64* oS = (pass == 2 && c->qr_shift[slot]) ? mS12 : mS;
    c64* oInv = pass == 2 ? mS2i : mS3i;
    for (int e = threadIdx.x; e < ss; e += blockDim.x) {
        oS[e] = D[e];
        oInv[e] = B[e];
        if (pass == 2) mS12[e] = D[e];
    }
}

// Bl-BiCG-rQ: G = V^^H W -> alpha = G^{-1} M, alpha^ = G^{-H} M^H, alpha C.
__global__ __launch_bounds__(kCoefThreads) void k_blrq_alpha(Ctl* c, int s, const c64* __restrict__ part2, int p2, c64* __restrict__ mats,
                             c64* __restrict__ sc) {
    if (stopped(c)) return;
    extern __shared__ c64 dyn[];
    __shared__ int flag;
    __shared__ int piv[kMaxS];
    const int ss = s * s;
    c64* G = dyn;
    c64* A = dyn + ss;
    c64* B = dyn + 2 * ss;
    c64* D = dyn + 3 * ss;
    gram_final(part2, p2, ss, G);
    if (!sm_lu(G, piv, s, &flag)) {
        if (threadIdx.x == 0) set_bd(c);
        return;
    }
    const c64* Mm = mats + (size_t)M_M * ss;
    sm_copy(A, Mm, ss);
    sm_lu_solve(G, piv, A, s, s);                         // alpha
    for (int e = threadIdx.x; e < ss; e += blockDim.x) {      // M^H
        int i = e / s, j = e - i * s;
        B[e] = conj_(Mm[j * s + i]);
    }
    __syncthreads();
    sm_lu_solve_h(G, piv, B, s, s);                       // alpha^
    sm_copy(D, mats + (size_t)M_C * ss, ss);
    sm_gemm(G, A, 0, D, 0, s);                            // alpha C (G reused)
    for (int e = threadIdx.x; e < ss; e += blockDim.x) {
        mats[(size_t)M_ALPHA * ss + e] = -A[e];           // stored negated: Z = Q + W (-alpha)
        mats[(size_t)M_ALPHAH * ss + e] = -B[e];
        mats[(size_t)M_ALPHAC * ss + e] = G[e];
    }
    (void)sc;
}

// Bl-BiCG-rQ: M' = Q^'^H Q' -> C = S C, C^ = S^ C^, stopping test on ||C||_F,
// beta = M^{-1} S^^H M', beta^ = M^{-H} S^H M'^H, M = M'.
__global__ __launch_bounds__(kCoefThreads) void k_blrq_beta(Ctl* c, double* hist, int s, const c64* __restrict__ part2, int p2,
                            c64* __restrict__ mats) {
    if (stopped(c)) return;
    extern __shared__ c64 dyn[];
    __shared__ int flag;
    __shared__ int piv[kMaxS];
    __shared__ double red;
    const int ss = s * s;
    c64* Mn = dyn;
    c64* A = dyn + ss;
    c64* B = dyn + 2 * ss;
    c64* D = dyn + 3 * ss;
    gram_final(part2, p2, ss, Mn);
    // C = S C
    sm_copy(A, mats + (size_t)M_S * ss, ss);
    sm_copy(B, mats + (size_t)M_C * ss, ss);
    sm_gemm(D, A, 0, B, 0, s);
    for (int e = threadIdx.x; e < ss; e += blockDim.x) mats[(size_t)M_C * ss + e] = D[e];
    double res2 = sm_frob2(D, ss, &red);
    // C^ = S^ C^
    sm_copy(A, mats + (size_t)M_T * ss, ss);
    sm_copy(B, mats + (size_t)M_CH * ss, ss);
    sm_gemm(D, A, 0, B, 0, s);
    for (int e = threadIdx.x; e < ss; e += blockDim.x) mats[(size_t)M_CH * ss + e] = D[e];
    if (threadIdx.x == 0) flag = end_of_iteration(c, hist, res2) ? 1 : 0;
    __syncthreads();
    if (!flag) return;
    __syncthreads();
    // beta = M^{-1} S^^H M' ; beta^ = M^{-H} S^H M'^H
    sm_copy(A, mats + (size_t)M_M * ss, ss);
    if (!sm_lu(A, piv, s, &flag)) {
        if (threadIdx.x == 0) set_bd(c);
        return;
    }
    sm_copy(B, mats + (size_t)M_T * ss, ss);   // S^
    sm_gemm(D, B, 1, Mn, 0, s);                // S^^H M'
    sm_lu_solve(A, piv, D, s, s);              // beta
    for (int e = threadIdx.x; e < ss; e += blockDim.x) mats[(size_t)M_BETA * ss + e] = D[e];
    sm_copy(B, mats + (size_t)M_S * ss, ss);   // S
    sm_gemm(D, B, 1, Mn, 1, s);                // S^H M'^H
    sm_lu_solve_h(A, piv, D, s, s);            // beta^
    for (int e = threadIdx.x; e < ss; e += blockDim.x) {
        mats[(size_t)M_BETAH * ss + e] = D[e];
        mats[(size_t)M_M * ss + e] = Mn[e];
    }
}

// Initialisation of an rQ method after the first QR (slot 0): C = S, ||C||_F
// -> control block.  copy_hat: C^ = C (shadow = R0).  Reduced Gram (if p2 > 0)
// -> mats slot `gslot` (M = Q^H Q or N = R~^H Q).
__global__ __launch_bounds__(kScalar) void k_bl_init(Ctl* c, double* hist, int s, int copy_hat, const c64* __restrict__ part2, int p2,
                          int gslot, c64* __restrict__ mats) {
    if (stopped(c)) return;
    extern __shared__ c64 dyn[];
    __shared__ double red;
    const int ss = s * s;
    c64* G = dyn;
    if (p2 > 0) {
        gram_final(part2, p2, ss, G);
        for (int e = threadIdx.x; e < ss; e += blockDim.x) mats[(size_t)gslot * ss + e] = G[e];
    }
    sm_copy(G, mats + (size_t)M_S * ss, ss);
    for (int e = threadIdx.x; e < ss; e += blockDim.x) {
        mats[(size_t)M_C * ss + e] = G[e];
        if (copy_hat) {
            mats[(size_t)M_CH * ss + e] = G[e];
            mats[(size_t)M_T * ss + e] = G[e];
        }
    }
    double nr2 = sm_frob2(G, ss, &red);
    if (threadIdx.x == 0) {
        double nr0 = sqrt(nr2);
        c->nr0 = nr0;
        c->res = nr0;
        c->iter = 0;
        c->bd_iter = -1;
        hist[0] = 1.0;
        c->status = ST_RUNNING;
        c->done = c->maxit <= 0 ? 1 : 0;
        if (!(nr0 > 0.0)) { c->status = ST_OK; c->done = 1; }
    }
}

// Bl-BiCGStab-rQ: G = R~^H W -> LU (kept), a = G^{-1} N (stored negated for S~ = Q - W a)
__global__ __launch_bounds__(kCoefThreads) void k_blst_a(Ctl* c, int s, const c64* __restrict__ part2, int p2, c64* __restrict__ mats,
                         c64* __restrict__ sc) {
    if (stopped(c)) return;
    extern __shared__ c64 dyn[];
    __shared__ int flag;
    __shared__ int piv[kMaxS];
    const int ss = s * s;
    c64* G = dyn;
    c64* A = dyn + ss;
    gram_final(part2, p2, ss, G);
    if (!sm_lu(G, piv, s, &flag)) {
        if (threadIdx.x == 0) set_bd(c);
        return;
    }
    sm_copy(A, mats + (size_t)M_N * ss, ss);
    sm_lu_solve(G, piv, A, s, s);
    for (int e = threadIdx.x; e < ss; e += blockDim.x) {
        mats[(size_t)M_A * ss + e] = A[e];
        mats[(size_t)M_TMP * ss + e] = -A[e];
        mats[(size_t)M_G * ss + e] = G[e];
    }
    for (int k = threadIdx.x; k < s; k += blockDim.x) sc[SC_PIV + k] = {(double)piv[k], 0.0};
}

// Bl-BiCGStab-rQ: (T~^H S~, T~^H T~) -> omega = tr(T~^H S~ K) / tr(T~^H T~ K), K = C C^H;
// a C and omega C for the X update.
__global__ __launch_bounds__(kCoefThreads) void k_blst_omega(Ctl* c, int s, const c64* __restrict__ part2, int p2, c64* __restrict__ mats,
                             c64* __restrict__ sc) {
    if (stopped(c)) return;
    extern __shared__ c64 dyn[];
    const int ss = s * s;
    c64* G1 = dyn;
    c64* G2 = dyn + ss;
    c64* A = dyn + 2 * ss;
    c64* K = dyn + 3 * ss;
    // the two Grams are stored back to back: entries [0, ss) and [ss, 2 ss)
    for (int e = threadIdx.x; e < 2 * ss; e += blockDim.x) {
        c64 acc = part2[e];
        for (int y = 1; y < p2; ++y) acc = acc + part2[(size_t)y * 2 * ss + e];
        if (e < ss) G1[e] = acc;
        else G2[e - ss] = acc;
    }
    __syncthreads();
    sm_copy(A, mats + (size_t)M_C * ss, ss);
    sm_gemm(K, A, 0, A, 1, s);                 // C C^H
    c64 num = {0.0, 0.0}, den = {0.0, 0.0};   // tr(G1 K), tr(G2 K)
    for (int e = threadIdx.x; e < ss; e += blockDim.x) {
        const int a = e / s, b = e - a * s;
        num = num + G1[e] * K[b * s + a];
        den = den + G2[e] * K[b * s + a];
    }
    num = {wg_sum(num.x), wg_sum(num.y)};
    den = {wg_sum(den.x), wg_sum(den.y)};
    if (threadIdx.x == 0) {
        if (bad_den(den)) {
            set_bd(c);
        } else {
            sc[SC_OMEGA] = cdiv(num, den);
        }
    }
    __syncthreads();
    if (stopped(c)) return;
    const c64 w = sc[SC_OMEGA];
    sm_copy(G2, mats + (size_t)M_A * ss, ss);
    sm_gemm(G1, G2, 0, A, 0, s);               // a C
    for (int e = threadIdx.x; e < ss; e += blockDim.x) {
        mats[(size_t)M_AC * ss + e] = G1[e];
        mats[(size_t)M_WC * ss + e] = w * A[e];
    }
}

// Bl-BiCGStab-rQ: N' = R~^H Q' -> C = Sigma C, stopping test, b = (1/omega) G^{-1} N', N = N'.
__global__ __launch_bounds__(kCoefThreads) void k_blst_b(Ctl* c, double* hist, int s, const c64* __restrict__ part2, int p2,
                         c64* __restrict__ mats, c64* __restrict__ sc) {
    if (stopped(c)) return;
    extern __shared__ c64 dyn[];
    __shared__ int flag;
    __shared__ int piv[kMaxS];
    __shared__ double red;
    const int ss = s * s;
    c64* Nn = dyn;
    c64* A = dyn + ss;
    c64* B = dyn + 2 * ss;
    c64* D = dyn + 3 * ss;
    gram_final(part2, p2, ss, Nn);
    sm_copy(A, mats + (size_t)M_S * ss, ss);
    sm_copy(B, mats + (size_t)M_C * ss, ss);
    sm_gemm(D, A, 0, B, 0, s);
    for (int e = threadIdx.x; e < ss; e += blockDim.x) mats[(size_t)M_C * ss + e] = D[e];
    double res2 = sm_frob2(D, ss, &red);
    if (threadIdx.x == 0) flag = end_of_iteration(c, hist, res2) ? 1 : 0;
    __syncthreads();
    if (!flag) return;
    __syncthreads();
    const c64 w = sc[SC_OMEGA];
    if (bad_den(w)) {
        if (threadIdx.x == 0) set_bd(c);
        return;
    }
    sm_copy(A, mats + (size_t)M_G * ss, ss);
    for (int k = threadIdx.x; k < s; k += blockDim.x) piv[k] = (int)sc[SC_PIV + k].x;
    sm_copy(B, Nn, ss);
    sm_lu_solve(A, piv, B, s, s);
    const c64 iw = cdiv(c64{1.0, 0.0}, w);
    for (int e = threadIdx.x; e < ss; e += blockDim.x) {
        mats[(size_t)M_B * ss + e] = iw * B[e];
        mats[(size_t)M_N * ss + e] = Nn[e];
    }
    if (threadIdx.x == 0) sc[SC_GAMMA] = -w;
}

}  // namespace skr
