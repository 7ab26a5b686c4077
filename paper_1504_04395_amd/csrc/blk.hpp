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
// Q1 = Z S1^{-1}, G1 = Q1^H Q1 = S2^H S2, Q = Z (S2 S1)^{-1}, C = S2 S1.  If the
// first Cholesky factorisation fails, the first pass is repeated with the shift
// 11 (n s + s(s+1)) u tr(G) (shifted CholeskyQR, Fukaya et al. 2020) and one
// more unshifted pass is added (CholeskyQR3).  Q1 is never stored: each pass
// recomputes it from Z.
#pragma once

#include "common.hpp"
#include "glk.hpp"
#include "small.hpp"

namespace skr {

// ---------------------------------------------------------------- mats slots
// Every block method keeps its s x s matrices in one device array `mats`
// (slot k at mats + k*s*s, complex FP64).
enum {
    M_C = 0, M_CH, M_M, M_G, M_ALPHA, M_ALPHAH, M_ALPHAC, M_BETA, M_BETAH,
    M_S1, M_S1INV, M_S12, M_S12INV, M_S, M_SINV,          // QR slot 0 work
    M_T1, M_T1INV, M_T12, M_T12INV, M_T, M_TINV,          // QR slot 1 work
    M_N, M_A, M_AC, M_WC, M_B, M_RB, M_TMP,
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

template <class T, int J>
__device__ inline void load_row(const T* __restrict__ P, int i, bool valid, int lane, int s, c64 (&v)[J]) {
#pragma unroll
    for (int j = 0; j < J; ++j) {
        int c = lane + 16 * j;
        v[j] = (valid && c < s) ? up(P[(size_t)i * s + c]) : c64{0.0, 0.0};
    }
}
template <class T, int J>
__device__ inline void store_row(T* __restrict__ P, int i, bool valid, int lane, int s, const c64 (&v)[J]) {
    if (!valid) return;
#pragma unroll
    for (int j = 0; j < J; ++j) {
        int c = lane + 16 * j;
        if (c < s) P[(size_t)i * s + c] = down<T>(v[j]);
    }
}
// tile[grp][:] = v (this lane's entries)
template <int J>
__device__ inline void put_tile(c64* tile, int grp, int lane, int s, const c64 (&v)[J]) {
#pragma unroll
    for (int j = 0; j < J; ++j) {
        int c = lane + 16 * j;
        if (c < s) tile[grp * s + c] = v[j];
    }
}
// out[j] (+)= sum_a tile[grp][a] * M[a][c_j]
template <int J>
__device__ inline void tile_times(const c64* tile, const c64* M, int grp, int lane, int s, c64 (&out)[J]) {
#pragma unroll
    for (int j = 0; j < J; ++j) {
        int c = lane + 16 * j;
        if (c >= s) continue;
        c64 acc = out[j];
        for (int a = 0; a < s; ++a) {
            c64 t = tile[grp * s + a], m = M[a * s + c];
            acc.x = fma(t.x, m.x, fma(-t.y, m.y, acc.x));
            acc.y = fma(t.x, m.y, fma(t.y, m.x, acc.y));
        }
        out[j] = acc;
    }
}
__device__ inline void lds_load_mat(c64* dst, const c64* __restrict__ src, int s) {
    for (int e = threadIdx.x; e < s * s; e += kBlock) dst[e] = src[e];
}

// ---------------------------------------------------------------- Gram
// part[b] = L^H R over this workgroup's rows
template <class T, int J>
__global__ __launch_bounds__(kBlock) void k_bl_gram(const Ctl* ctl, Tile16 tl, const T* __restrict__ Lm,
                                                    const T* __restrict__ Rm, c64* part) {
    if (stopped(ctl)) return;
    GramAcc<J, Tr<T>::cplx> g;
    g.clear();
    SKR_TILE_LOOP(tl) {
        const int i = base_ + grp;
        const bool valid = i < r1_;
        c64 l[J], r[J];
        load_row<T, J>(Lm, i, valid, lane, tl.s, l);
        load_row<T, J>(Rm, i, valid, lane, tl.s, r);
        g.add(l, r);
    }
    __shared__ c64 lds[(16 * J) * (16 * J)];
    g.store(tl.s, lds, part + (size_t)blockIdx.x * tl.s * tl.s);
}

// Stage-2 reduction of per-workgroup partials [np][E] -> [gridDim.y][E]
__global__ __launch_bounds__(kBlock) void k_reduce_parts(const Ctl* ctl, int cond_slot, const c64* __restrict__ part,
                                                         int np, int E, c64* __restrict__ out) {
    if (stopped(ctl)) return;
    if (cond_slot >= 0 && !ctl->qr_shift[cond_slot]) return;
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= E) return;
    const int per = (np + gridDim.y - 1) / gridDim.y;
    const int b0 = blockIdx.y * per, b1 = min(np, b0 + per);
    c64 acc = {0.0, 0.0};
    for (int b = b0; b < b1; ++b) acc = acc + part[(size_t)b * E + e];
    out[(size_t)blockIdx.y * E + e] = acc;
}

// final sum of the stage-2 partials into LDS
__device__ inline void gram_final(const c64* __restrict__ part2, int p2, int E, c64* dst) {
    for (int e = threadIdx.x; e < E; e += kBlock) {
        c64 acc = part2[e];
        for (int y = 1; y < p2; ++y) acc = acc + part2[(size_t)y * E + e];
        dst[e] = acc;
    }
    __syncthreads();
}

// ---------------------------------------------------------------- triangular pass
enum { TRI_WRITE = 1, TRI_G_OUT_OUT = 2, TRI_G_OTHER_OUT = 4, TRI_G_OUT_OTHER = 8 };

// out = Z * Minv (Minv at mats slot `minv`).  cond_slot >= 0: run only when the
// shifted first pass was used for that QR slot.
template <class T, int J>
__global__ __launch_bounds__(kBlock) void k_bl_tri(const Ctl* ctl, int cond_slot, Tile16 tl, int mode,
                                                   const c64* __restrict__ mats, int minv, const T* Z, T* Out,
                                                   const T* __restrict__ Other, c64* part) {
    if (stopped(ctl)) return;
    if (cond_slot >= 0 && !ctl->qr_shift[cond_slot]) return;
    extern __shared__ c64 dyn[];
    const int s = tl.s;
    c64* M = dyn;                 // s*s
    c64* tile = dyn + s * s;      // 16*s
    lds_load_mat(M, mats + (size_t)minv * s * s, s);
    GramAcc<J, Tr<T>::cplx> g;
    g.clear();
    SKR_TILE_LOOP(tl) {
        const int i = base_ + grp;
        const bool valid = i < r1_;
        c64 z[J], o[J];
        load_row<T, J>(Z, i, valid, lane, s, z);
        __syncthreads();
        put_tile<J>(tile, grp, lane, s, z);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < J; ++j) o[j] = {0.0, 0.0};
        tile_times<J>(tile, M, grp, lane, s, o);
        if (!valid) {
#pragma unroll
            for (int j = 0; j < J; ++j) o[j] = {0.0, 0.0};
        }
        if (mode & TRI_WRITE) store_row<T, J>(Out, i, valid, lane, s, o);
        if (mode & TRI_G_OUT_OUT) g.add(o, o);
        if (mode & (TRI_G_OTHER_OUT | TRI_G_OUT_OTHER)) {
            c64 ot[J];
            load_row<T, J>(Other, i, valid, lane, s, ot);
            if (mode & TRI_G_OTHER_OUT) g.add(ot, o);
            else g.add(o, ot);
        }
    }
    if (mode & (TRI_G_OUT_OUT | TRI_G_OTHER_OUT | TRI_G_OUT_OTHER)) {
        __syncthreads();
        g.store(s, dyn, part + (size_t)blockIdx.x * s * s);
    }
}

// Out = A + (B + gamma C) M  [+ part = Out^H Out]; A or C may be null; Out may alias A or B.
template <class T, int J, bool GRAM>
__global__ __launch_bounds__(kBlock) void k_bl_axpm(const Ctl* ctl, Tile16 tl, const c64* __restrict__ mats, int mslot,
                                                    const c64* __restrict__ sc, int gslot, const T* A,
                                                    const T* B, const T* __restrict__ Cm, T* Out, c64* part) {
    if (stopped(ctl)) return;
    extern __shared__ c64 dyn[];
    const int s = tl.s;
    c64* M = dyn;
    c64* tile = dyn + s * s;
    lds_load_mat(M, mats + (size_t)mslot * s * s, s);
    const c64 gamma = Cm ? sc[gslot] : c64{0.0, 0.0};
    GramAcc<J, Tr<T>::cplx> g;
    g.clear();
    SKR_TILE_LOOP(tl) {
        const int i = base_ + grp;
        const bool valid = i < r1_;
        c64 b[J], o[J];
        load_row<T, J>(B, i, valid, lane, s, b);
        if (Cm) {
            c64 cc[J];
            load_row<T, J>(Cm, i, valid, lane, s, cc);
#pragma unroll
            for (int j = 0; j < J; ++j) b[j] = b[j] + gamma * cc[j];
        }
        if (A) load_row<T, J>(A, i, valid, lane, s, o);
        else {
#pragma unroll
            for (int j = 0; j < J; ++j) o[j] = {0.0, 0.0};
        }
        __syncthreads();
        put_tile<J>(tile, grp, lane, s, b);
        __syncthreads();
        tile_times<J>(tile, M, grp, lane, s, o);
        store_row<T, J>(Out, i, valid, lane, s, o);
        if (GRAM) {
            if (!valid) {
#pragma unroll
                for (int j = 0; j < J; ++j) o[j] = {0.0, 0.0};
            }
            g.add(o, o);
        }
    }
    if (GRAM) {
        __syncthreads();
        g.store(s, dyn, part + (size_t)blockIdx.x * s * s);
    }
}

// Bl-BiCG-rQ: X += V (alpha C); Z = Q - W alpha; part = Z^H Z
template <class T, int J>
__global__ __launch_bounds__(kBlock) void k_blrq_updz(const Ctl* ctl, Tile16 tl, const c64* __restrict__ mats,
                                                      T* __restrict__ X, const T* __restrict__ V,
                                                      const T* __restrict__ Q, const T* __restrict__ W,
                                                      T* __restrict__ Z, c64* part) {
    if (stopped(ctl)) return;
    extern __shared__ c64 dyn[];
    const int s = tl.s;
    c64* Ma = dyn;                  // alpha
    c64* Mac = dyn + s * s;         // alpha C
    c64* tv = dyn + 2 * s * s;      // V tile
    c64* tw = tv + 16 * s;          // W tile
    lds_load_mat(Ma, mats + (size_t)M_ALPHA * s * s, s);
    lds_load_mat(Mac, mats + (size_t)M_ALPHAC * s * s, s);
    GramAcc<J, Tr<T>::cplx> g;
    g.clear();
    SKR_TILE_LOOP(tl) {
        const int i = base_ + grp;
        const bool valid = i < r1_;
        c64 v[J], w[J], x[J], z[J];
        load_row<T, J>(V, i, valid, lane, s, v);
        load_row<T, J>(W, i, valid, lane, s, w);
        load_row<T, J>(X, i, valid, lane, s, x);
        load_row<T, J>(Q, i, valid, lane, s, z);
        __syncthreads();
        put_tile<J>(tv, grp, lane, s, v);
        put_tile<J>(tw, grp, lane, s, w);
        __syncthreads();
        tile_times<J>(tv, Mac, grp, lane, s, x);
        c64 wa[J];
#pragma unroll
        for (int j = 0; j < J; ++j) wa[j] = {0.0, 0.0};
        tile_times<J>(tw, Ma, grp, lane, s, wa);
#pragma unroll
        for (int j = 0; j < J; ++j) z[j] = valid ? z[j] + wa[j] : c64{0.0, 0.0};  // mats holds -alpha
        store_row<T, J>(X, i, valid, lane, s, x);
        store_row<T, J>(Z, i, valid, lane, s, z);
        g.add(z, z);
    }
    __syncthreads();
    g.store(s, dyn, part + (size_t)blockIdx.x * s * s);
}

// Bl-BiCGStab-rQ: X += U (a C) + S~ (omega C); Z = S~ - omega T~; part = Z^H Z
template <class T, int J>
__global__ __launch_bounds__(kBlock) void k_blst_upd(const Ctl* ctl, Tile16 tl, const c64* __restrict__ mats,
                                                     const c64* __restrict__ sc, T* __restrict__ X,
                                                     const T* __restrict__ U, const T* __restrict__ St,
                                                     const T* __restrict__ Tt, T* __restrict__ Z, c64* part) {
    if (stopped(ctl)) return;
    extern __shared__ c64 dyn[];
    const int s = tl.s;
    c64* Mac = dyn;                 // a C
    c64* Mwc = dyn + s * s;         // omega C
    c64* tu = dyn + 2 * s * s;
    c64* ts = tu + 16 * s;
    lds_load_mat(Mac, mats + (size_t)M_AC * s * s, s);
    lds_load_mat(Mwc, mats + (size_t)M_WC * s * s, s);
    const c64 w = sc[SC_OMEGA];
    GramAcc<J, Tr<T>::cplx> g;
    g.clear();
    SKR_TILE_LOOP(tl) {
        const int i = base_ + grp;
        const bool valid = i < r1_;
        c64 u[J], st[J], tt[J], x[J], z[J];
        load_row<T, J>(U, i, valid, lane, s, u);
        load_row<T, J>(St, i, valid, lane, s, st);
        load_row<T, J>(Tt, i, valid, lane, s, tt);
        load_row<T, J>(X, i, valid, lane, s, x);
        __syncthreads();
        put_tile<J>(tu, grp, lane, s, u);
        put_tile<J>(ts, grp, lane, s, st);
        __syncthreads();
        tile_times<J>(tu, Mac, grp, lane, s, x);
        tile_times<J>(ts, Mwc, grp, lane, s, x);
#pragma unroll
        for (int j = 0; j < J; ++j) z[j] = st[j] - w * tt[j];
        store_row<T, J>(X, i, valid, lane, s, x);
        store_row<T, J>(Z, i, valid, lane, s, z);
        g.add(z, z);
    }
    __syncthreads();
    g.store(s, dyn, part + (size_t)blockIdx.x * s * s);
}

// ---------------------------------------------------------------- coefficient kernels
// Dynamic LDS: 6 s x s matrices.
__device__ inline void set_bd(Ctl* c) { set_breakdown(c); }

// QR step 1 (or 3): G -> S1 (with shift fallback on the first pass), S1inv.
// pass 1: reads the reduced Gram of Z; stores S1, S1INV of the slot.
// pass 2: Gram of Q1 -> S2; S12 = S2 S1, S12inv = S1inv S2inv; if no shift was
//         used these are the final factors (S, SINV).
// pass 3 (only with shift): Gram of Q2 -> S3; S = S3 S12, SINV = S12inv S3inv.
__global__ void k_qr_chol(Ctl* c, int slot, int pass, int n, int s, const c64* __restrict__ part2, int p2,
                          c64* __restrict__ mats) {
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
    c64* mS12i = mats + (size_t)(base + 3) * ss;
    c64* mS = mats + (size_t)(base + 4) * ss;
    c64* mSi = mats + (size_t)(base + 5) * ss;
    gram_final(part2, p2, ss, G);
    if (pass == 1) {
        if (threadIdx.x == 0) c->qr_shift[slot] = 0;
        sm_copy(A, G, ss);
        int ok = sm_cholesky(A, s, 0.0, &flag);
        if (!ok) {
            double trg = 0.0;
            for (int i = 0; i < s; ++i) trg += G[i * s + i].x;
            double shift = 11.0 * ((double)n * s + (double)s * (s + 1)) * 0x1p-53 * trg;
            sm_copy(A, G, ss);
            ok = sm_cholesky(A, s, shift, &flag);
            if (threadIdx.x == 0) c->qr_shift[slot] = 1;
            __syncthreads();
        }
        if (!ok) {
            if (threadIdx.x == 0) set_bd(c);
            return;
        }
        sm_tri_inv_upper(A, B, s);
        for (int e = threadIdx.x; e < ss; e += kBlock) {
            mS1[e] = A[e];
            mS1i[e] = B[e];
        }
        return;
    }
    sm_copy(A, G, ss);
    int ok = sm_cholesky(A, s, 0.0, &flag);
    if (!ok) {
        if (threadIdx.x == 0) set_bd(c);
        return;
    }
    sm_tri_inv_upper(A, B, s);  // B = S_k^{-1}
    const c64* prevS = pass == 2 ? mS1 : mS12;
    const c64* prevSi = pass == 2 ? mS1i : mS12i;
    sm_copy(G, prevS, ss);
    sm_gemm(D, A, 0, G, 0, s);   // S_k * prev
    sm_copy(G, prevSi, ss);
    sm_gemm(A, G, 0, B, 0, s);   // prev^{-1} S_k^{-1}
    const bool final_ = (pass == 3) || !c->qr_shift[slot];
    c64* oS = final_ ? mS : mS12;
    c64* oSi = final_ ? mSi : mS12i;
    for (int e = threadIdx.x; e < ss; e += kBlock) {
        oS[e] = D[e];
        oSi[e] = A[e];
    }
}

// Bl-BiCG-rQ: G = V^^H W -> alpha = G^{-1} M, alpha^ = G^{-H} M^H, alpha C.
__global__ void k_blrq_alpha(Ctl* c, int s, const c64* __restrict__ part2, int p2, c64* __restrict__ mats,
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
    for (int e = threadIdx.x; e < ss; e += kBlock) {      // M^H
        int i = e / s, j = e - i * s;
        B[e] = conj_(Mm[j * s + i]);
    }
    __syncthreads();
    sm_lu_solve_h(G, piv, B, s, s);                       // alpha^
    sm_copy(D, mats + (size_t)M_C * ss, ss);
    sm_gemm(G, A, 0, D, 0, s);                            // alpha C (G reused)
    for (int e = threadIdx.x; e < ss; e += kBlock) {
        mats[(size_t)M_ALPHA * ss + e] = -A[e];           // stored negated: Z = Q + W (-alpha)
        mats[(size_t)M_ALPHAH * ss + e] = -B[e];
        mats[(size_t)M_ALPHAC * ss + e] = G[e];
    }
    (void)sc;
}

// Bl-BiCG-rQ: M' = Q^'^H Q' -> C = S C, C^ = S^ C^, stopping test on ||C||_F,
// beta = M^{-1} S^^H M', beta^ = M^{-H} S^H M'^H, M = M'.
__global__ void k_blrq_beta(Ctl* c, double* hist, int s, const c64* __restrict__ part2, int p2,
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
    c64* E = dyn + 4 * ss;
    gram_final(part2, p2, ss, Mn);
    // C = S C, C^ = S^ C^
    sm_copy(A, mats + (size_t)M_S * ss, ss);
    sm_copy(B, mats + (size_t)M_C * ss, ss);
    sm_gemm(D, A, 0, B, 0, s);
    sm_copy(A, mats + (size_t)M_T * ss, ss);
    sm_copy(B, mats + (size_t)M_CH * ss, ss);
    sm_gemm(E, A, 0, B, 0, s);
    for (int e = threadIdx.x; e < ss; e += kBlock) {
        mats[(size_t)M_C * ss + e] = D[e];
        mats[(size_t)M_CH * ss + e] = E[e];
    }
    double res2 = sm_frob2(D, ss, &red);
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
    sm_copy(B, mats + (size_t)M_S * ss, ss);   // S
    sm_gemm(E, B, 1, Mn, 1, s);                // S^H M'^H
    sm_lu_solve_h(A, piv, E, s, s);            // beta^
    for (int e = threadIdx.x; e < ss; e += kBlock) {
        mats[(size_t)M_BETA * ss + e] = D[e];
        mats[(size_t)M_BETAH * ss + e] = E[e];
        mats[(size_t)M_M * ss + e] = Mn[e];
    }
}

// Initialisation of an rQ method after the first QR (slot 0): C = S, ||C||_F
// -> control block.  copy_hat: C^ = C (shadow = R0).  Reduced Gram (if p2 > 0)
// -> mats slot `gslot` (M = Q^H Q or N = R~^H Q).
__global__ void k_bl_init(Ctl* c, double* hist, int s, int copy_hat, const c64* __restrict__ part2, int p2,
                          int gslot, c64* __restrict__ mats) {
    if (stopped(c)) return;
    extern __shared__ c64 dyn[];
    __shared__ double red;
    const int ss = s * s;
    c64* G = dyn;
    if (p2 > 0) {
        gram_final(part2, p2, ss, G);
        for (int e = threadIdx.x; e < ss; e += kBlock) mats[(size_t)gslot * ss + e] = G[e];
    }
    sm_copy(G, mats + (size_t)M_S * ss, ss);
    for (int e = threadIdx.x; e < ss; e += kBlock) {
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
__global__ void k_blst_a(Ctl* c, int s, const c64* __restrict__ part2, int p2, c64* __restrict__ mats,
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
    for (int e = threadIdx.x; e < ss; e += kBlock) {
        mats[(size_t)M_A * ss + e] = A[e];
        mats[(size_t)M_TMP * ss + e] = -A[e];
        mats[(size_t)M_G * ss + e] = G[e];
    }
    for (int k = threadIdx.x; k < s; k += kBlock) sc[SC_PIV + k] = {(double)piv[k], 0.0};
}

// Bl-BiCGStab-rQ: (T~^H S~, T~^H T~) -> omega = tr(T~^H S~ K) / tr(T~^H T~ K), K = C C^H;
// a C and omega C for the X update.
__global__ void k_blst_omega(Ctl* c, int s, const c64* __restrict__ part2, int p2, c64* __restrict__ mats,
                             c64* __restrict__ sc) {
    if (stopped(c)) return;
    extern __shared__ c64 dyn[];
    const int ss = s * s;
    c64* G1 = dyn;
    c64* G2 = dyn + ss;
    c64* K = dyn + 2 * ss;
    c64* A = dyn + 3 * ss;
    c64* D = dyn + 4 * ss;
    // the two Grams are stored back to back: entries [0, ss) and [ss, 2 ss)
    for (int e = threadIdx.x; e < 2 * ss; e += kBlock) {
        c64 acc = part2[e];
        for (int y = 1; y < p2; ++y) acc = acc + part2[(size_t)y * 2 * ss + e];
        if (e < ss) G1[e] = acc;
        else G2[e - ss] = acc;
    }
    __syncthreads();
    sm_copy(A, mats + (size_t)M_C * ss, ss);
    sm_gemm(K, A, 0, A, 1, s);                 // C C^H
    if (threadIdx.x == 0) {
        c64 num = {0.0, 0.0}, den = {0.0, 0.0};
        for (int a = 0; a < s; ++a)
            for (int b = 0; b < s; ++b) {
                num = num + G1[a * s + b] * K[b * s + a];
                den = den + G2[a * s + b] * K[b * s + a];
            }
        if (bad_den(den)) {
            set_bd(c);
        } else {
            sc[SC_OMEGA] = cdiv(num, den);
        }
    }
    __syncthreads();
    if (stopped(c)) return;
    const c64 w = sc[SC_OMEGA];
    sm_copy(D, mats + (size_t)M_A * ss, ss);
    sm_gemm(G1, D, 0, A, 0, s);                // a C
    for (int e = threadIdx.x; e < ss; e += kBlock) {
        mats[(size_t)M_AC * ss + e] = G1[e];
        mats[(size_t)M_WC * ss + e] = w * A[e];
    }
}

// Bl-BiCGStab-rQ: N' = R~^H Q' -> C = Sigma C, stopping test, b = (1/omega) G^{-1} N', N = N'.
__global__ void k_blst_b(Ctl* c, double* hist, int s, const c64* __restrict__ part2, int p2,
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
    for (int e = threadIdx.x; e < ss; e += kBlock) mats[(size_t)M_C * ss + e] = D[e];
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
    for (int k = threadIdx.x; k < s; k += kBlock) piv[k] = (int)sc[SC_PIV + k].x;
    sm_copy(B, Nn, ss);
    sm_lu_solve(A, piv, B, s, s);
    const c64 iw = cdiv(c64{1.0, 0.0}, w);
    for (int e = threadIdx.x; e < ss; e += kBlock) {
        mats[(size_t)M_B * ss + e] = iw * B[e];
        mats[(size_t)M_N * ss + e] = Nn[e];
    }
    if (threadIdx.x == 0) sc[SC_GAMMA] = -w;
}

}  // namespace skr
