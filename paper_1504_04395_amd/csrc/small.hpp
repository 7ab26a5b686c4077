// One-workgroup FP64 linear algebra on s x s matrices (s <= 32) in LDS, used by
// the coefficient kernels of every iteration: LU with partial pivoting and the
// pivot breakdown test, solves with G and with G^H, upper Cholesky factors
// (G = S^H S), triangular inverses and small products.  Matrices are row-major
// complex doubles; real problems carry zero imaginary parts, which every routine
// here keeps exactly zero.  All routines are called by the whole workgroup: one
// wavefront, or kCoefThreads threads for the per-iteration coefficient kernels
// of the block methods, whose elimination steps then update one entry per
// thread instead of four.  The steps of a factorisation or substitution are
// parallel over the matrix entries they update, with a barrier between steps;
// reductions take a butterfly within each wave and the waves in order.
#pragma once

#include "common.hpp"

namespace skr {

__device__ inline double cabs1(c64 a) { return fabs(a.x) + fabs(a.y); }

__device__ inline void sm_copy(c64* dst, const c64* src, int count) {
    for (int e = threadIdx.x; e < count; e += blockDim.x) dst[e] = src[e];
    __syncthreads();
}

__device__ inline void sm_identity(c64* A, int s) {
    for (int e = threadIdx.x; e < s * s; e += blockDim.x) {
        int i = e / s, j = e - i * s;
        A[e] = {i == j ? 1.0 : 0.0, 0.0};
    }
    __syncthreads();
}

// C = op(A) * op(B); ta / tb: 0 = as is, 1 = conjugate transpose.
// C must not alias A or B.
__device__ inline void sm_gemm(c64* C, const c64* A, int ta, const c64* B, int tb, int s) {
    for (int e = threadIdx.x; e < s * s; e += blockDim.x) {
        int i = e / s, j = e - i * s;
        c64 acc = {0.0, 0.0};
        for (int k = 0; k < s; ++k) {
            c64 a = ta ? conj_(A[k * s + i]) : A[i * s + k];
            c64 b = tb ? conj_(B[j * s + k]) : B[k * s + j];
            acc = acc + a * b;
        }
        C[e] = acc;
    }
    __syncthreads();
}

constexpr int kCoefThreads = 256;   // workgroup of the block methods' coefficient kernels

__device__ inline double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ inline int wave_all(int ok) { return __all(ok); }

// Workgroup reductions for up to kCoefThreads threads (one wave: the wave's own
// result).  Every thread receives the result; the waves are combined in order.
__device__ inline double wg_sum(double v) {
    v = wave_sum(v);
    if (blockDim.x <= 64) return v;
    __shared__ double r[kCoefThreads / 64];
    __syncthreads();   // an earlier call's readers are done
    if ((threadIdx.x & 63) == 0) r[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = r[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) t += r[i];
    return t;
}
__device__ inline double wg_max(double v) {
    v = wave_max(v);
    if (blockDim.x <= 64) return v;
    __shared__ double r[kCoefThreads / 64];
    __syncthreads();
    if ((threadIdx.x & 63) == 0) r[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = r[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) t = fmax(t, r[i]);
    return t;
}
__device__ inline int wg_all(int ok) {
    ok = __all(ok);
    if (blockDim.x <= 64) return ok;
    __shared__ int r[kCoefThreads / 64];
    __syncthreads();
    if ((threadIdx.x & 63) == 0) r[threadIdx.x >> 6] = ok;
    __syncthreads();
    int t = 1;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t &= r[i];
    return t;
}

// ||A||_F^2 over `count` entries (fixed order: strided per thread, butterfly,
// waves in order).
__device__ inline double sm_frob2(const c64* A, int count, double* red /* unused */) {
    (void)red;
    double t = 0.0;
    for (int e = threadIdx.x; e < count; e += blockDim.x) t += abs2(A[e]);
    return wg_sum(t);
}

// Work split of an update over the rows of an s x m array: thread t owns
// column t % m and rows t / m, t / m + 64 / m, ... (m <= 64), computed once.
struct Split {
    int j, r0, rs;
    bool on;
};
__device__ inline Split split_cols(int m) {
    const int t = threadIdx.x, rs = blockDim.x / m;
    return {t % m, t / m, rs, t < rs * m};
}

// One step of an update X[i][j] -= L(i) * x for the rows i = i0, i0 + rs, ...
// below iend of column j (row stride ldx; L(i) = Lm[i * lds + lk] or the
// conjugate of Lm[lk * lds + i]).
template <bool CONJT>
__device__ inline void sm_axpy_rows(c64* X, int ldx, int j, const c64* Lm, int lds, int lk, c64 x, int i0, int rs,
                                    int iend) {
    for (int i = i0; i < iend; i += rs) {
        const c64 l = CONJT ? conj_(Lm[lk * lds + i]) : Lm[i * lds + lk];
        X[i * ldx + j] = X[i * ldx + j] - l * x;
    }
}

// In-place LU with partial pivoting, P G = L U (unit L below the diagonal, U on
// and above).  piv[k] = row swapped with k at step k: the first row of largest
// |re| + |im| in column k (LAPACK's choice).  Returns 1 if U passes the pivot
// test |u_kk| > s * 2^-52 * max |u_ij| with all entries finite, else 0.
__device__ inline int sm_lu(c64* __restrict__ A, int* __restrict__ piv, int s, int* flag) {
    (void)flag;
    const int t = threadIdx.x;
    const Split sp = split_cols(s);
    for (int k = 0; k < s; ++k) {
        if (t < 64) {   // the first wave searches the column (rows k..s-1, s <= 64)
            double v = -1.0;
            int idx = k;
            if (t >= k && t < s) {
                v = cabs1(A[t * s + k]);
                idx = t;
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const double v2 = __shfl_xor(v, off, 64);
                const int i2 = __shfl_xor(idx, off, 64);
                if (v2 > v || (v2 == v && i2 < idx)) {
                    v = v2;
                    idx = i2;
                }
            }
            if (t == 0) piv[k] = idx;
        }
        __syncthreads();
        const int p = piv[k];
        if (p != k) {
            for (int j = t; j < s; j += blockDim.x) {
                c64 x = A[k * s + j];
                A[k * s + j] = A[p * s + j];
                A[p * s + j] = x;
            }
            __syncthreads();
        }
        // multipliers l_ik = a_ik / a_kk (column k) and the trailing update, in
        // one step: each updater forms l_ik itself; column k is rewritten after
        const c64 d = A[k * s + k];
        if (sp.on && sp.j > k) {   // a_ij -= (a_ik / d) u_kj
            const c64 ukj = A[k * s + sp.j];
            for (int i = k + 1 + sp.r0; i < s; i += sp.rs) A[i * s + sp.j] = A[i * s + sp.j] - cdiv(A[i * s + k], d) * ukj;
        }
        __syncthreads();
        if (sp.on && sp.j == k)   // column k is read by the update above, so it is scaled after it
            for (int i = k + 1 + sp.r0; i < s; i += sp.rs) A[i * s + k] = cdiv(A[i * s + k], d);
        __syncthreads();
    }
    double umax = 0.0;
    int fin = 1;
    for (int e = t; e < s * s; e += blockDim.x) {
        const int i = e / s, j = e - i * s;
        const c64 u = A[e];
        if (!cfinite(u)) fin = 0;
        if (j >= i) umax = fmax(umax, cabs(u));
    }
    umax = wg_max(umax);
    int ok = fin && umax > 0.0;
    for (int k = t; k < s; k += blockDim.x)
        if (!(cabs(A[k * s + k]) > s * 0x1p-52 * umax)) ok = 0;
    return wg_all(ok);
}

// B := G^{-1} B for B s x m (row-major, leading dimension m), G = P^T L U.
// Row swaps column by column; forward substitution with L; back substitution
// with U where each step uses x_k = b_k / u_kk formed by every updater and row
// k itself is divided once at the end, so each step needs one barrier.
__device__ inline void sm_lu_solve(const c64* __restrict__ LU, const int* __restrict__ piv, c64* __restrict__ B,
                                   int s, int m) {
    const int t = threadIdx.x;
    for (int j = t; j < m; j += blockDim.x)
        for (int k = 0; k < s; ++k) {
            const int p = piv[k];
            if (p != k) {
                c64 x = B[k * m + j];
                B[k * m + j] = B[p * m + j];
                B[p * m + j] = x;
            }
        }
    __syncthreads();
    const Split sp = split_cols(m);
    for (int k = 0; k + 1 < s; ++k) {   // unit lower
        if (sp.on) sm_axpy_rows<false>(B, m, sp.j, LU, s, k, B[k * m + sp.j], k + 1 + sp.r0, sp.rs, s);
        __syncthreads();
    }
    for (int k = s - 1; k > 0; --k) {   // upper
        if (sp.on) sm_axpy_rows<false>(B, m, sp.j, LU, s, k, cdiv(B[k * m + sp.j], LU[k * s + k]), sp.r0, sp.rs, k);
        __syncthreads();
    }
    for (int e = t; e < s * m; e += blockDim.x) {
        const int i = e / m;
        B[e] = cdiv(B[e], LU[i * s + i]);
    }
    __syncthreads();
}

// B := G^{-H} B, with G = P^T L U, i.e. solve U^H L^H P X = B.
__device__ inline void sm_lu_solve_h(const c64* __restrict__ LU, const int* __restrict__ piv, c64* __restrict__ B,
                                     int s, int m) {
    const int t = threadIdx.x;
    const Split sp = split_cols(m);
    for (int k = 0; k + 1 < s; ++k) {   // U^H: lower, diagonal conj(u_kk)
        if (sp.on)
            sm_axpy_rows<true>(B, m, sp.j, LU, s, k, cdiv(B[k * m + sp.j], conj_(LU[k * s + k])), k + 1 + sp.r0,
                               sp.rs, s);
        __syncthreads();
    }
    for (int e = t; e < s * m; e += blockDim.x) {
        const int i = e / m;
        B[e] = cdiv(B[e], conj_(LU[i * s + i]));
    }
    __syncthreads();
    for (int k = s - 1; k > 0; --k) {   // L^H: unit upper
        if (sp.on) sm_axpy_rows<true>(B, m, sp.j, LU, s, k, B[k * m + sp.j], sp.r0, sp.rs, k);
        __syncthreads();
    }
    for (int j = t; j < m; j += blockDim.x)   // X = P^T W
        for (int k = s - 1; k >= 0; --k) {
            const int p = piv[k];
            if (p != k) {
                c64 x = B[k * m + j];
                B[k * m + j] = B[p * m + j];
                B[p * m + j] = x;
            }
        }
    __syncthreads();
}

// In-place upper Cholesky factor G = S^H S of a Hermitian matrix (upper
// triangle of G is used; the strict lower triangle is set to 0).  `shift` is
// added to the diagonal first.  Returns 1 on success, 0 if a pivot is not
// safely positive (d <= tau * largest original diagonal entry, or not finite).
// CholeskyQR callers pass tau = 1e4 u for the first pass (u = unit roundoff of
// the stored block: a condition number beyond (1e4 u)^{-1/2} would leave the
// first-pass Q too far from orthonormal for a second pass to repair).
// Step k updates the trailing part with the unscaled row k divided by the
// pivot d_k; the rows are scaled by 1 / sqrt(d_k) at the end.
__device__ inline int sm_cholesky(c64* G, int s, double shift, int* flag /* shared */, double tau) {
    __shared__ double diag0[kMaxS];
    __shared__ double piv[kMaxS];
    for (int i = threadIdx.x; i < s; i += blockDim.x) {
        G[i * s + i].x += shift;
        G[i * s + i].y = 0.0;
        diag0[i] = G[i * s + i].x;
    }
    __syncthreads();
    double dmax = 0.0;
    for (int i = 0; i < s; ++i) dmax = fmax(dmax, diag0[i]);
    const Split sp = split_cols(s);
    int ok = 1;
    for (int k = 0; k < s; ++k) {
        const double d = G[k * s + k].x;
        if (!(d > tau * dmax) || !isfinite(d) || !(diag0[k] > 0.0)) {
            ok = 0;
            break;   // uniform: every thread reads the same d
        }
        if (threadIdx.x == 0) piv[k] = d;
        if (sp.on && sp.j > k)
            sm_axpy_rows<true>(G, s, sp.j, G, s, k, (1.0 / d) * G[k * s + sp.j], k + 1 + sp.r0, sp.rs, sp.j + 1);
        __syncthreads();
    }
    if (ok) {
        for (int e = threadIdx.x; e < s * s; e += blockDim.x) {
            const int i = e / s, j = e - i * s;
            if (j < i) G[e] = {0.0, 0.0};
            else if (j == i) G[e] = {sqrt(piv[i]), 0.0};
            else G[e] = (1.0 / sqrt(piv[i])) * G[e];
        }
    } else {
        for (int e = threadIdx.x; e < s * s; e += blockDim.x) {
            const int i = e / s, j = e - i * s;
            if (j < i) G[e] = {0.0, 0.0};
        }
    }
    if (threadIdx.x == 0) *flag = ok;
    __syncthreads();
    return ok;
}

// Sinv = S^{-1} for upper triangular S (Sinv must not alias S): back
// substitution on the identity, one barrier per step, diagonal division last.
__device__ inline void sm_tri_inv_upper(const c64* __restrict__ S, c64* __restrict__ Sinv, int s) {
    for (int e = threadIdx.x; e < s * s; e += blockDim.x) {
        const int i = e / s, j = e - i * s;
        Sinv[e] = {i == j ? 1.0 : 0.0, 0.0};
    }
    __syncthreads();
    const Split sp = split_cols(s);
    for (int k = s - 1; k > 0; --k) {
        if (sp.on && sp.j >= k)
            sm_axpy_rows<false>(Sinv, s, sp.j, S, s, k, cdiv(Sinv[k * s + sp.j], S[k * s + k]), sp.r0, sp.rs, k);
        __syncthreads();
    }
    for (int e = threadIdx.x; e < s * s; e += blockDim.x) {
        const int i = e / s;
        Sinv[e] = cdiv(Sinv[e], S[i * s + i]);
    }
    __syncthreads();
}

}  // namespace skr
