// One-wavefront coefficient kernels of the methods without QR of the residual
// block: block BiCG (Algorithm 3), loop-interchanged BiCG (Algorithm 1, s
// independent BiCG recurrences, written as block BiCG with diagonal
// coefficient matrices) and block BiCGStab (El Guennouni et al.).  The s x s
// algebra is FP64 in LDS; the breakdown rule is the one of every method: a
// scalar denominator that is 0 or not finite, or an LU pivot failing the test
// of sm_lu.
#pragma once

#include "blk.hpp"

namespace skr {

// mats[slot] = the reduced s x s matrix in part2 (E = s * s entries)
__global__ __launch_bounds__(kScalar) void k_stash(const Ctl* c, const c64* __restrict__ part2, int p2, int s,
                                                   c64* __restrict__ mats, int slot) {
    if (stopped(c)) return;
    const int ss = s * s;
    for (int e = threadIdx.x; e < ss; e += blockDim.x) {
        c64 acc = part2[e];
        for (int y = 1; y < p2; ++y) acc = acc + part2[(size_t)y * ss + e];
        mats[(size_t)slot * ss + e] = acc;
    }
}

// alpha step.  G1 = P^^H A P (mats M_G1), RhR = R^^H R (mats M_RHR), and for the
// block method G2 = P^H A^H P^ (part2).
//   block:  alpha = G1^{-1} RhR,  alpha^ = G2^{-1} RhR^H
//   Li:     alpha_c = (RhR)_cc / (G1)_cc,  alpha^ = conj(alpha)
// Stores alpha (M_ALPHA), -alpha (M_TMP) and -alpha^ (M_ALPHAH).
__global__ __launch_bounds__(kScalar) void k_blb_alpha(Ctl* c, int s, int diag, const c64* __restrict__ part2,
                                                       int p2, c64* __restrict__ mats) {
    if (stopped(c)) return;
    extern __shared__ c64 dyn[];
    __shared__ int flag;
    __shared__ int piv[kMaxS];
    const int ss = s * s;
    c64* G = dyn;
    c64* A = dyn + ss;
    c64* B = dyn + 2 * ss;
    const c64* rhr = mats + (size_t)M_RHR * ss;
    if (diag) {
        int ok = 1;
        for (int e = threadIdx.x; e < ss; e += blockDim.x) {
            const int i = e / s, j = e - i * s;
            c64 a = {0.0, 0.0};
            if (i == j) {
                const c64 sig = mats[(size_t)M_G1 * ss + e];
                if (bad_den(sig)) ok = 0;
                else a = cdiv(rhr[e], sig);
            }
            A[e] = a;
        }
        if (!wave_all(ok)) {
            if (threadIdx.x == 0) set_breakdown(c);
            return;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < ss; e += blockDim.x) {
            mats[(size_t)M_ALPHA * ss + e] = A[e];
            mats[(size_t)M_TMP * ss + e] = -A[e];
            mats[(size_t)M_ALPHAH * ss + e] = -conj_(A[e]);
        }
        return;
    }
    sm_copy(G, mats + (size_t)M_G1 * ss, ss);
    if (!sm_lu(G, piv, s, &flag)) {
        if (threadIdx.x == 0) set_breakdown(c);
        return;
    }
    sm_copy(A, rhr, ss);
    sm_lu_solve(G, piv, A, s, s);                      // alpha
    gram_final(part2, p2, ss, G);                      // G2
    if (!sm_lu(G, piv, s, &flag)) {
        if (threadIdx.x == 0) set_breakdown(c);
        return;
    }
    for (int e = threadIdx.x; e < ss; e += blockDim.x) {
        const int i = e / s, j = e - i * s;
        B[e] = conj_(rhr[j * s + i]);                  // RhR^H
    }
    __syncthreads();
    sm_lu_solve(G, piv, B, s, s);                      // alpha^
    for (int e = threadIdx.x; e < ss; e += blockDim.x) {
        mats[(size_t)M_ALPHA * ss + e] = A[e];
        mats[(size_t)M_TMP * ss + e] = -A[e];
        mats[(size_t)M_ALPHAH * ss + e] = -B[e];
    }
}

// beta step after the updates.  ||R||_F^2 = tr(R^H R) (mats M_RR) drives the
// stopping rule; RhR' = R^^H R (part2), RhR (old, mats M_RHR).
//   block:  beta = RhR^{-1} RhR',  beta^ = RhR^{-H} RhR'^H
//   Li:     beta_c = (RhR')_cc / (RhR)_cc,  beta^ = conj(beta)
// Stores beta (M_BETA), beta^ (M_BETAH) and RhR' (M_RHR).
__global__ __launch_bounds__(kScalar) void k_blb_beta(Ctl* c, double* hist, int s, int diag,
                                                      const c64* __restrict__ part2, int p2,
                                                      c64* __restrict__ mats) {
    if (stopped(c)) return;
    extern __shared__ c64 dyn[];
    __shared__ int flag;
    __shared__ int piv[kMaxS];
    const int ss = s * s;
    c64* Rn = dyn;
    c64* A = dyn + ss;
    c64* B = dyn + 2 * ss;
    double t = 0.0;
    for (int i = threadIdx.x; i < s; i += blockDim.x) t += mats[(size_t)M_RR * ss + i * s + i].x;
    const double res2 = wave_sum(t);
    if (threadIdx.x == 0) flag = end_of_iteration(c, hist, res2) ? 1 : 0;
    __syncthreads();
    if (!flag) return;
    __syncthreads();
    gram_final(part2, p2, ss, Rn);
    const c64* rhr = mats + (size_t)M_RHR * ss;
    if (diag) {
        int ok = 1;
        for (int e = threadIdx.x; e < ss; e += blockDim.x) {
            const int i = e / s, j = e - i * s;
            c64 b = {0.0, 0.0};
            if (i == j) {
                if (bad_den(rhr[e])) ok = 0;
                else b = cdiv(Rn[e], rhr[e]);
            }
            A[e] = b;
        }
        if (!wave_all(ok)) {
            if (threadIdx.x == 0) set_breakdown(c);
            return;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < ss; e += blockDim.x) {
            mats[(size_t)M_BETA * ss + e] = A[e];
            mats[(size_t)M_BETAH * ss + e] = conj_(A[e]);
            mats[(size_t)M_RHR * ss + e] = Rn[e];
        }
        return;
    }
    sm_copy(B, rhr, ss);
    if (!sm_lu(B, piv, s, &flag)) {
        if (threadIdx.x == 0) set_breakdown(c);
        return;
    }
    sm_copy(A, Rn, ss);
    sm_lu_solve(B, piv, A, s, s);                      // beta
    for (int e = threadIdx.x; e < ss; e += blockDim.x) {
        mats[(size_t)M_BETA * ss + e] = A[e];
        const int i = e / s, j = e - i * s;
        A[e] = conj_(Rn[j * s + i]);                   // RhR'^H
    }
    __syncthreads();
    sm_lu_solve_h(B, piv, A, s, s);                    // beta^
    for (int e = threadIdx.x; e < ss; e += blockDim.x) {
        mats[(size_t)M_BETAH * ss + e] = A[e];
        mats[(size_t)M_RHR * ss + e] = Rn[e];
    }
}

// Block BiCGStab omega from the (tr(T^H S), tr(T^H T)) partials; stores omega,
// -omega (SC_GAMMA) and the scaled identities omega I (M_W), -omega I (M_MW).
__global__ __launch_bounds__(kScalar) void k_blbs_omega(Ctl* c, int s, const c64* __restrict__ part, int np,
                                                        c64* __restrict__ sc, c64* __restrict__ mats) {
    if (stopped(c)) return;
    __shared__ c64 r[2];
    sum_partials<2>(part, np, r);
    const c64 num = r[0], den = r[1];
    if (bad_den(den)) {
        if (threadIdx.x == 0) set_breakdown(c);
        return;
    }
    const c64 w = cdiv(num, den);
    const int ss = s * s;
    for (int e = threadIdx.x; e < ss; e += blockDim.x) {
        const int i = e / s, j = e - i * s;
        mats[(size_t)M_W * ss + e] = i == j ? w : c64{0.0, 0.0};
        mats[(size_t)M_MW * ss + e] = i == j ? -w : c64{0.0, 0.0};
    }
    if (threadIdx.x == 0) {
        sc[SC_OMEGA] = w;
        sc[SC_GAMMA] = -w;
    }
}

// Block BiCGStab beta after the updates: ||R||_F^2 = tr(R^H R) (mats M_RR)
// drives the stopping rule; beta = -G^{-1} (R~^H T) with G's LU (M_G, pivots in
// sc) and R~^H T (M_RT); N' = R~^H R (part2) replaces N (M_N).
__global__ __launch_bounds__(kScalar) void k_blbs_beta(Ctl* c, double* hist, int s, const c64* __restrict__ part2,
                                                       int p2, c64* __restrict__ mats,
                                                       const c64* __restrict__ sc) {
    if (stopped(c)) return;
    extern __shared__ c64 dyn[];
    __shared__ int flag;
    __shared__ int piv[kMaxS];
    const int ss = s * s;
    c64* G = dyn;
    c64* A = dyn + ss;
    double t = 0.0;
    for (int i = threadIdx.x; i < s; i += blockDim.x) t += mats[(size_t)M_RR * ss + i * s + i].x;
    const double res2 = wave_sum(t);
    if (threadIdx.x == 0) flag = end_of_iteration(c, hist, res2) ? 1 : 0;
    __syncthreads();
    if (!flag) return;
    __syncthreads();
    sm_copy(G, mats + (size_t)M_G * ss, ss);
    for (int k = threadIdx.x; k < s; k += blockDim.x) piv[k] = (int)sc[SC_PIV + k].x;
    sm_copy(A, mats + (size_t)M_RT * ss, ss);
    sm_lu_solve(G, piv, A, s, s);
    for (int e = threadIdx.x; e < ss; e += blockDim.x) mats[(size_t)M_B * ss + e] = -A[e];
    gram_final(part2, p2, ss, A);
    for (int e = threadIdx.x; e < ss; e += blockDim.x) mats[(size_t)M_N * ss + e] = A[e];
}

}  // namespace skr
