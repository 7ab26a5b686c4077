// One-workgroup FP64 linear algebra on s x s matrices (s <= 32) in LDS, used by
// the coefficient kernels of every iteration: LU with partial pivoting and the
// pivot breakdown test, solves with G and with G^H, upper Cholesky factors
// (G = S^H S), triangular inverses and small products.  Matrices are row-major
// complex doubles; real problems carry zero imaginary parts, which every routine
// here keeps exactly zero.  All routines are called by the whole workgroup, which
// is one wavefront (64 threads): reductions across it use lane shuffles, and
// the steps of a factorisation or substitution are parallel over the matrix
// entries they update, with a barrier between steps.
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

__device__ inline double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ inline int wave_all(int ok) { return __all(ok); }

// ||A||_F^2 over `count` entries (fixed order: strided per lane, butterfly).
__device__ inline double sm_frob2(const c64* A, int count, double* red /* unused */) {
    (void)red;
    double t = 0.0;
    for (int e = threadIdx.x; e < count; e += blockDim.x) t += abs2(A[e]);
    return wave_sum(t);
}

// In-place LU with partial pivoting, P G = L U (unit L below the diagonal, U on
// and above).  piv[k] = row swapped with k at step k: the first row of largest
// |re| + |im| in column k (LAPACK's choice).  Returns 1 if U passes the pivot
// test |u_kk| > s * 2^-52 * max |u_ij| with all entries finite, else 0.
__device__ inline int sm_lu(c64* A, int* piv, int s, int* flag) {
    (void)flag;
    const int t = threadIdx.x;
    for (int k = 0; k < s; ++k) {
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
        const int p = idx;
        if (t == 0) piv[k] = p;
        if (p != k) {
            for (int j = t; j < s; j += blockDim.x) {
                c64 x = A[k * s + j];
                A[k * s + j] = A[p * s + j];
                A[p * s + j] = x;
            }
            __syncthreads();
        }
        const c64 d = A[k * s + k];
        for (int i = k + 1 + t; i < s; i += blockDim.x) A[i * s + k] = cdiv(A[i * s + k], d);
        __syncthreads();
        const int m = s - k - 1;
        for (int e = t; e < m * m; e += blockDim.x) {
            const int i = k + 1 + e / m, j = k + 1 + e % m;
            A[i * s + j] = A[i * s + j] - A[i * s + k] * A[k * s + j];
        }
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
    umax = wave_max(umax);
    int ok = fin && umax > 0.0;
    for (int k = t; k < s; k += blockDim.x)
        if (!(cabs(A[k * s + k]) > s * 0x1p-52 * umax)) ok = 0;
    return wave_all(ok);
}

// B := G^{-1} B for B s x m (row-major, leading dimension m), G = P^T L U.
// Row swaps column by column, then forward and back substitution, each step
// parallel over the entries it updates.
__device__ inline void sm_lu_solve(const c64* LU, const int* piv, c64* B, int s, int m) {
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
    for (int k = 0; k + 1 < s; ++k) {   // unit lower
        const int n1 = (s - k - 1) * m;
        for (int e = t; e < n1; e += blockDim.x) {
            const int i = k + 1 + e / m, j = e % m;
            B[i * m + j] = B[i * m + j] - LU[i * s + k] * B[k * m + j];
        }
        __syncthreads();
    }
    for (int k = s - 1; k >= 0; --k) {  // upper
        for (int j = t; j < m; j += blockDim.x) B[k * m + j] = cdiv(B[k * m + j], LU[k * s + k]);
        __syncthreads();
        const int n1 = k * m;
        for (int e = t; e < n1; e += blockDim.x) {
            const int i = e / m, j = e % m;
            B[i * m + j] = B[i * m + j] - LU[i * s + k] * B[k * m + j];
        }
        __syncthreads();
    }
}

// B := G^{-H} B, with G = P^T L U, i.e. solve U^H L^H P X = B.
__device__ inline void sm_lu_solve_h(const c64* LU, const int* piv, c64* B, int s, int m) {
    const int t = threadIdx.x;
    for (int k = 0; k < s; ++k) {       // U^H: lower, diagonal conj(u_kk)
        for (int j = t; j < m; j += blockDim.x) B[k * m + j] = cdiv(B[k * m + j], conj_(LU[k * s + k]));
        __syncthreads();
        const int n1 = (s - k - 1) * m;
        for (int e = t; e < n1; e += blockDim.x) {
            const int i = k + 1 + e / m, j = e % m;
            B[i * m + j] = B[i * m + j] - conj_(LU[k * s + i]) * B[k * m + j];
        }
        __syncthreads();
    }
    for (int k = s - 1; k > 0; --k) {   // L^H: unit upper
        const int n1 = k * m;
        for (int e = t; e < n1; e += blockDim.x) {
            const int i = e / m, j = e % m;
            B[i * m + j] = B[i * m + j] - conj_(LU[k * s + i]) * B[k * m + j];
        }
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
__device__ inline int sm_cholesky(c64* G, int s, double shift, int* flag /* shared */, double tau) {
    __shared__ double diag0[kMaxS];
    for (int i = threadIdx.x; i < s; i += blockDim.x) {
        G[i * s + i].x += shift;
        G[i * s + i].y = 0.0;
        diag0[i] = G[i * s + i].x;
    }
    if (threadIdx.x == 0) *flag = 1;
    __syncthreads();
    double dmax = 0.0;
    for (int i = 0; i < s; ++i) dmax = fmax(dmax, diag0[i]);
    for (int k = 0; k < s; ++k) {
        double d = G[k * s + k].x;
        bool bad = !(d > tau * dmax) || !isfinite(d) || !(diag0[k] > 0.0);
        if (bad) {
            if (threadIdx.x == 0) *flag = 0;
            __syncthreads();
            break;
        }
        double r = sqrt(d);
        __syncthreads();
        for (int j = k + threadIdx.x; j < s; j += blockDim.x) {
            if (j == k) G[k * s + k] = {r, 0.0};
            else G[k * s + j] = (1.0 / r) * G[k * s + j];
        }
        __syncthreads();
        const int m = s - k - 1;
        for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
            int i = k + 1 + e / m, j = k + 1 + e % m;
            if (j >= i) G[i * s + j] = G[i * s + j] - conj_(G[k * s + i]) * G[k * s + j];
        }
        __syncthreads();
    }
    int ok = *flag;
    for (int e = threadIdx.x; e < s * s; e += blockDim.x) {
        int i = e / s, j = e - i * s;
        if (j < i) G[e] = {0.0, 0.0};
    }
    __syncthreads();
    return ok;
}

// Sinv = S^{-1} for upper triangular S.  Sinv must not alias S.
__device__ inline void sm_tri_inv_upper(const c64* S, c64* Sinv, int s) {
    for (int e = threadIdx.x; e < s * s; e += blockDim.x) Sinv[e] = {0.0, 0.0};
    __syncthreads();
    for (int j = threadIdx.x; j < s; j += blockDim.x) {
        Sinv[j * s + j] = cdiv(c64{1.0, 0.0}, S[j * s + j]);
        for (int i = j - 1; i >= 0; --i) {
            c64 acc = {0.0, 0.0};
            for (int k = i + 1; k <= j; ++k) acc = acc + S[i * s + k] * Sinv[k * s + j];
            Sinv[i * s + j] = cdiv(-acc, S[i * s + i]);
        }
    }
    __syncthreads();
}

}  // namespace skr
