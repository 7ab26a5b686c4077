// Block kernels on MFMA row tiles for complex storage (s <= 16 J, J = 1 or 2)
// and for real storage with 16 < s <= 32: the CholeskyQR triangular pass, the
// s x s-coefficient updates of the block methods and the Bl-BiCG-rQ /
// Bl-BiCGStab-rQ fused updates, with the same arguments and results as the
// real s <= 16 kernels in blk.hpp (k_bl_tri16, k_bl_axpm16, k_blrq_updz16,
// k_blst_upd16).  Real data carry zero imaginary parts, which
// the real instances neither load nor multiply (one MFMA per slab, not four).
//
// Tile layout: a wave owns 16 consecutive rows; lane L = c + 16 q holds, in
// register v, the element (row 4v + q, column c + 16 h) for h < J, real and
// imaginary parts apart.  These are 16-lane coalesced row loads, and also the
// layout of the MFMA f64 16x16x4 result D[4v + q][c] (lane c + 16 q,
// register v).  A product with an s x s complex matrix M is
//     X M = (Xr Mr - Xi Mi) + i (Xr Mi + Xi Mr),
// four real MFMAs per 4-column slab t of X and 16-column slab jb of M.  The A
// operand (lane c + 16 q: X[c][4t + q]) is read back transposed through a
// per-wave LDS tile; the B operand (lane c + 16 q: M[4t + q][16 jb + c]) comes
// from the workgroup's LDS copy of M, zero-padded to 16 J x 16 J.  Padding
// rows (past n) and columns (past s) are zero, so they add nothing to Grams.
#pragma once

#include "blk.hpp"

namespace skr {

template <int J>
struct CTile {
    double r[J][4], i[J][4];
};

template <int J>
constexpr int cld() { return 16 * J + 1; }   // LDS row stride in doubles (odd: spread banks)

template <int J>
__device__ inline void ctile_zero(CTile<J>& x) {
#pragma unroll
    for (int h = 0; h < J; ++h)
#pragma unroll
        for (int v = 0; v < 4; ++v) x.r[h][v] = x.i[h][v] = 0.0;
}

// rows b + 4v + q (< r1), columns c + 16h (< s) of P (row stride s); zero elsewhere
template <class T, int J>
__device__ inline void ctile_load(const T* P, int b, int r1, int s, int c, int q, CTile<J>& x) {
#pragma unroll
    for (int h = 0; h < J; ++h)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = b + 4 * v + q, col = c + 16 * h;
            const bool ok = i < r1 && col < s;
            const c64 u = up(P[(size_t)(ok ? i : b) * s + (ok ? col : 0)]);
            x.r[h][v] = ok ? u.x : 0.0;
            x.i[h][v] = ok ? u.y : 0.0;
        }
}

template <class T, int J>
__device__ inline void ctile_store(T* P, int b, int r1, int s, int c, int q, const CTile<J>& x) {
#pragma unroll
    for (int h = 0; h < J; ++h)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = b + 4 * v + q, col = c + 16 * h;
            if (i < r1 && col < s) P[(size_t)i * s + col] = down<T>(c64{x.r[h][v], x.i[h][v]});
        }
}

// the workgroup's LDS copy of the s x s matrix Mg (real and imaginary parts apart,
// zero-padded to 16J x 16J); the caller synchronises before use
template <int J>
__device__ inline void cmat_lds(double* Mr, double* Mi, const c64* __restrict__ Mg, int s) {
    constexpr int S = 16 * J, LD = cld<J>();
    for (int e = threadIdx.x; e < S * S; e += blockDim.x) {
        const int k = e / S, j = e - k * S;
        const c64 v = (k < s && j < s) ? Mg[k * s + j] : c64{0.0, 0.0};
        Mr[k * LD + j] = v.x;
        Mi[k * LD + j] = v.y;
    }
}

// o += x M for the wave's tile x; M from LDS (Mr, Mi); tw: this wave's LDS tile
// (2 * 16 * cld<J>() doubles).  C: complex arithmetic (else real parts only).
template <int J, bool C>
__device__ inline void capply(const CTile<J>& x, const double* Mr, const double* Mi, double* tw, int c, int q,
                              CTile<J>& o) {
    constexpr int LD = cld<J>();
    double* twr = tw;
    double* twi = tw + 16 * LD;
#pragma unroll
    for (int h = 0; h < J; ++h)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            twr[(4 * v + q) * LD + 16 * h + c] = x.r[h][v];
            if (C) twi[(4 * v + q) * LD + 16 * h + c] = x.i[h][v];
        }
    __builtin_amdgcn_wave_barrier();
    d4 ar[J], ai[J];
#pragma unroll
    for (int jb = 0; jb < J; ++jb) {
        ar[jb] = d4{o.r[jb][0], o.r[jb][1], o.r[jb][2], o.r[jb][3]};
        ai[jb] = d4{o.i[jb][0], o.i[jb][1], o.i[jb][2], o.i[jb][3]};
    }
#pragma unroll
    for (int t = 0; t < 4 * J; ++t) {
        const double xr = twr[c * LD + 4 * t + q];
#pragma unroll
        for (int jb = 0; jb < J; ++jb) {
            const double mr = Mr[(4 * t + q) * LD + 16 * jb + c];
            ar[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(xr, mr, ar[jb], 0, 0, 0);
            if (C) {
                const double xi = twi[c * LD + 4 * t + q], mi = Mi[(4 * t + q) * LD + 16 * jb + c];
                ar[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-xi, mi, ar[jb], 0, 0, 0);
                ai[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(xr, mi, ai[jb], 0, 0, 0);
                ai[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(xi, mr, ai[jb], 0, 0, 0);
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int jb = 0; jb < J; ++jb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            o.r[jb][v] = ar[jb][v];
            o.i[jb][v] = ai[jb][v];
        }
}

// Gram accumulation of y^H x over the tile's four row groups
template <int J, bool C>
__device__ inline void cgram_add(GramAcc<J, C>& g, const CTile<J>& y, const CTile<J>& x) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        c64 yv[J], xv[J];
#pragma unroll
        for (int h = 0; h < J; ++h) {
            yv[h] = c64{y.r[h][v], y.i[h][v]};
            xv[h] = c64{x.r[h][v], x.i[h][v]};
        }
        g.add(yv, xv);
    }
}

// the wave's tile loop over this workgroup's rows (XCD-chunked like the real kernels)
#define SKR_CTILE_RANGE(tl)                                         \
    const int L_ = threadIdx.x & 63, w_ = threadIdx.x >> 6;         \
    const int c = L_ & 15, q = L_ >> 4;                             \
    const int r0_ = xcd_chunk(blockIdx.x, gridDim.x) * (tl).rpc;    \
    const int r1_ = min((tl).n, r0_ + (tl).rpc)

// ---------------------------------------------------------------- kernels
// CholeskyQR triangular pass (as k_bl_tri16).  NC: the most inverse factors this instance
// applies (1 or 3); OTH: whether the Gram's second operand is another block.
template <class T, int J, int NC, bool OTH>
__global__ __launch_bounds__(kBlock) void k_bl_tric(const Ctl* ctl, int slot, int cond, int nchain, int add_shift,
                                                    Tile16 tl, int mode, const c64* __restrict__ mats, const T* Z,
                                                    T* Out, const T* __restrict__ Other, c64* part) {
    if (stopped(ctl)) return;
    constexpr bool C = Tr<T>::cplx;
    const int shifted = ctl->qr_shift[slot];
    if (cond && !shifted) return;
    const int nc = nchain + (add_shift && shifted ? 1 : 0);
    constexpr int S = 16 * J, LD = cld<J>();
    const int s = tl.s, ss = s * s;
    const int base = slot == 0 ? M_S1 : M_T1;
    __shared__ double Ms[NC][2][S * LD];
    __shared__ double tiles[kWaves][2 * 16 * LD];   // also the Gram's reduction buffer at the end
    cmat_lds<J>(Ms[0][0], Ms[0][1], mats + (size_t)(base + 1) * ss, s);
    if constexpr (NC > 1) {
        if (nc > 1) cmat_lds<J>(Ms[1][0], Ms[1][1], mats + (size_t)(base + 3) * ss, s);
        if (nc > 2) cmat_lds<J>(Ms[2][0], Ms[2][1], mats + (size_t)(base + 5) * ss, s);
    }
    __syncthreads();
    SKR_CTILE_RANGE(tl);
    double* tw = tiles[w_];
    GramAcc<J, C> g;
    g.clear();
    CTile<J> xn, otn;
    ctile_zero(otn);
    int b = r0_ + 16 * w_;
    if (b < r1_) {
        ctile_load<T, J>(Z, b, r1_, s, c, q, xn);
        if (OTH) ctile_load<T, J>(Other, b, r1_, s, c, q, otn);
    }
    for (; b < r1_; b += 16 * kWaves) {
        const CTile<J> x = xn, ot = otn;
        const int bn = b + 16 * kWaves;
        if (bn < r1_) {   // the next tile's loads are issued before this tile's MFMAs
            ctile_load<T, J>(Z, bn, r1_, s, c, q, xn);
            if (OTH) ctile_load<T, J>(Other, bn, r1_, s, c, q, otn);
        }
        CTile<J> o;
        ctile_zero(o);
        capply<J, C>(x, Ms[0][0], Ms[0][1], tw, c, q, o);
        if constexpr (NC > 1) {
            if (nc > 1) {
                const CTile<J> y = o;
                ctile_zero(o);
                capply<J, C>(y, Ms[1][0], Ms[1][1], tw, c, q, o);
            }
            if (nc > 2) {
                const CTile<J> y = o;
                ctile_zero(o);
                capply<J, C>(y, Ms[2][0], Ms[2][1], tw, c, q, o);
            }
        }
        if (mode & TRI_WRITE) ctile_store<T, J>(Out, b, r1_, s, c, q, o);
        if (mode & (TRI_G_OUT_OUT | TRI_G_OTHER_OUT | TRI_G_OUT_OTHER)) {
            if (!OTH) cgram_add<J, C>(g, o, o);
            else if (mode & TRI_G_OTHER_OUT) cgram_add<J, C>(g, ot, o);
            else cgram_add<J, C>(g, o, ot);
        }
    }
    if (mode & (TRI_G_OUT_OUT | TRI_G_OTHER_OUT | TRI_G_OUT_OTHER)) {
        __syncthreads();
        g.store(s, reinterpret_cast<c64*>(&tiles[0][0]), part + (size_t)blockIdx.x * ss);
    }
}

// Out = A + (B + gamma C) M [+ part = Out^H Out];
// A or C may be null; Out may alias A or B (a tile is loaded before it is
// written, by the same lanes, and later tiles are never written early).
template <class T, int J, bool GRAM>
__global__ __launch_bounds__(kBlock) void k_bl_axpmc(const Ctl* ctl, Tile16 tl, const c64* __restrict__ mats,
                                                     int mslot, const c64* __restrict__ sc, int gslot, const T* A,
                                                     const T* B, const T* __restrict__ Cm, T* Out, c64* part) {
    if (stopped(ctl)) return;
    constexpr bool C = Tr<T>::cplx;
    constexpr int S = 16 * J, LD = cld<J>();
    const int s = tl.s;
    __shared__ double Ms[2][S * LD];
    __shared__ double tiles[kWaves][2 * 16 * LD];
    cmat_lds<J>(Ms[0], Ms[1], mats + (size_t)mslot * s * s, s);
    __syncthreads();
    const c64 gamma = Cm ? sc[gslot] : c64{0.0, 0.0};
    SKR_CTILE_RANGE(tl);
    double* tw = tiles[w_];
    GramAcc<J, C> g;
    g.clear();
    CTile<J> bn_;
    int b = r0_ + 16 * w_;
    if (b < r1_) ctile_load<T, J>(B, b, r1_, s, c, q, bn_);
    for (; b < r1_; b += 16 * kWaves) {
        CTile<J> x = bn_;
        const int bn = b + 16 * kWaves;
        if (bn < r1_) ctile_load<T, J>(B, bn, r1_, s, c, q, bn_);
        if (Cm) {
            CTile<J> y;
            ctile_load<T, J>(Cm, b, r1_, s, c, q, y);
#pragma unroll
            for (int h = 0; h < J; ++h)
#pragma unroll
                for (int v = 0; v < 4; ++v) {   // x += gamma y
                    const double yr = y.r[h][v], yi = y.i[h][v];
                    x.r[h][v] = fma(gamma.x, yr, fma(-gamma.y, yi, x.r[h][v]));
                    x.i[h][v] = fma(gamma.x, yi, fma(gamma.y, yr, x.i[h][v]));
                }
        }
        CTile<J> o;
        if (A) ctile_load<T, J>(A, b, r1_, s, c, q, o);
        else ctile_zero(o);
        capply<J, C>(x, Ms[0], Ms[1], tw, c, q, o);
        ctile_store<T, J>(Out, b, r1_, s, c, q, o);
        if (GRAM) cgram_add<J, C>(g, o, o);
    }
    if (GRAM) {
        __syncthreads();
        g.store(s, reinterpret_cast<c64*>(&tiles[0][0]), part + (size_t)blockIdx.x * s * s);
    }
}

// Bl-BiCG-rQ: X += V (alpha C); Z = Q - W alpha; part = Z^H Z.
template <class T, int J>
__global__ __launch_bounds__(kBlock) void k_blrq_updzc(const Ctl* ctl, Tile16 tl, const c64* __restrict__ mats,
                                                       T* __restrict__ X, const T* __restrict__ Vb,
                                                       const T* __restrict__ Q, const T* __restrict__ W,
                                                       T* __restrict__ Z, c64* part) {
    if (stopped(ctl)) return;
    constexpr bool C = Tr<T>::cplx;
    constexpr int S = 16 * J, LD = cld<J>();
    const int s = tl.s;
    __shared__ double Ma[2][S * LD];    // -alpha
    __shared__ double Mac[2][S * LD];   // alpha C
    __shared__ double tiles[kWaves][2 * 16 * LD];
    cmat_lds<J>(Ma[0], Ma[1], mats + (size_t)M_ALPHA * s * s, s);
    cmat_lds<J>(Mac[0], Mac[1], mats + (size_t)M_ALPHAC * s * s, s);
    __syncthreads();
    SKR_CTILE_RANGE(tl);
    double* tw = tiles[w_];
    GramAcc<J, C> g;
    g.clear();
    for (int b = r0_ + 16 * w_; b < r1_; b += 16 * kWaves) {
        CTile<J> v, w, x, z;
        ctile_load<T, J>(Vb, b, r1_, s, c, q, v);
        ctile_load<T, J>(W, b, r1_, s, c, q, w);
        ctile_load<T, J>(X, b, r1_, s, c, q, x);
        ctile_load<T, J>(Q, b, r1_, s, c, q, z);
        capply<J, C>(v, Mac[0], Mac[1], tw, c, q, x);
        ctile_store<T, J>(X, b, r1_, s, c, q, x);
        capply<J, C>(w, Ma[0], Ma[1], tw, c, q, z);
        ctile_store<T, J>(Z, b, r1_, s, c, q, z);
        cgram_add<J, C>(g, z, z);
    }
    __syncthreads();
    g.store(s, reinterpret_cast<c64*>(&tiles[0][0]), part + (size_t)blockIdx.x * s * s);
}

// Bl-BiCGStab-rQ: X += U (a C) + S~ (omega C); Z = S~ - omega T~;
// part = Z^H Z.
template <class T, int J>
__global__ __launch_bounds__(kBlock) void k_blst_updc(const Ctl* ctl, Tile16 tl, const c64* __restrict__ mats,
                                                      const c64* __restrict__ sc, T* __restrict__ X,
                                                      const T* __restrict__ U, const T* __restrict__ St,
                                                      const T* __restrict__ Tt, T* __restrict__ Z, c64* part) {
    if (stopped(ctl)) return;
    constexpr bool C = Tr<T>::cplx;
    constexpr int S = 16 * J, LD = cld<J>();
    const int s = tl.s;
    __shared__ double Mac[2][S * LD];   // a C
    __shared__ double Mwc[2][S * LD];   // omega C
    __shared__ double tiles[kWaves][2 * 16 * LD];
    cmat_lds<J>(Mac[0], Mac[1], mats + (size_t)M_AC * s * s, s);
    cmat_lds<J>(Mwc[0], Mwc[1], mats + (size_t)M_WC * s * s, s);
    __syncthreads();
    const c64 mw = -sc[SC_OMEGA];
    SKR_CTILE_RANGE(tl);
    double* tw = tiles[w_];
    GramAcc<J, C> g;
    g.clear();
    for (int b = r0_ + 16 * w_; b < r1_; b += 16 * kWaves) {
        CTile<J> u, st, tt, x, z;
        ctile_load<T, J>(U, b, r1_, s, c, q, u);
        ctile_load<T, J>(St, b, r1_, s, c, q, st);
        ctile_load<T, J>(Tt, b, r1_, s, c, q, tt);
        ctile_load<T, J>(X, b, r1_, s, c, q, x);
        capply<J, C>(u, Mac[0], Mac[1], tw, c, q, x);
        capply<J, C>(st, Mwc[0], Mwc[1], tw, c, q, x);
        ctile_store<T, J>(X, b, r1_, s, c, q, x);
#pragma unroll
        for (int h = 0; h < J; ++h)
#pragma unroll
            for (int v = 0; v < 4; ++v) {   // z = st + mw tt
                const double tr = tt.r[h][v], ti = tt.i[h][v];
                z.r[h][v] = fma(mw.x, tr, fma(-mw.y, ti, st.r[h][v]));
                z.i[h][v] = fma(mw.x, ti, fma(mw.y, tr, st.i[h][v]));
            }
        ctile_store<T, J>(Z, b, r1_, s, c, q, z);
        cgram_add<J, C>(g, z, z);
    }
    __syncthreads();
    g.store(s, reinterpret_cast<c64*>(&tiles[0][0]), part + (size_t)blockIdx.x * s * s);
}

}  // namespace skr
