// Common device types and helpers for the gfx950 simultaneous Krylov solvers.
//
// Data layout: an n x s block is row-major with leading dimension s (the s
// right-hand sides of one row are contiguous), so one sparse row of A reads one
// contiguous row of the block for all s columns.  Complex values are (re, im)
// pairs.  Every reduction (traces tr(Y^H X), Gram matrices Y^H X, norms) is
// accumulated in FP64 in a fixed order (wave shuffles, then waves in order,
// then blocks in order), so results are bitwise reproducible run to run.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>

namespace skr {

constexpr int kBlock = 256;      // threads per workgroup for every streaming kernel
constexpr int kWaves = kBlock / 64;
constexpr int kScalar = 64;      // one wavefront: the one-workgroup coefficient kernels
constexpr int kMaxS = 32;        // largest block width the kernels support
constexpr int64_t kMaxRows = (1LL << 31) - (1LL << 20);   // largest n: row sweeps step int indices past n

struct c64 { double x, y; };
struct c32 { float x, y; };

// ---------------------------------------------------------------- arithmetic
__host__ __device__ inline c64 operator+(c64 a, c64 b) { return {a.x + b.x, a.y + b.y}; }
__host__ __device__ inline c64 operator-(c64 a, c64 b) { return {a.x - b.x, a.y - b.y}; }
__host__ __device__ inline c64 operator-(c64 a) { return {-a.x, -a.y}; }
__host__ __device__ inline c64 operator*(c64 a, c64 b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__host__ __device__ inline c64 operator*(double a, c64 b) { return {a * b.x, a * b.y}; }
__host__ __device__ inline c32 operator+(c32 a, c32 b) { return {a.x + b.x, a.y + b.y}; }
__host__ __device__ inline c32 operator-(c32 a, c32 b) { return {a.x - b.x, a.y - b.y}; }
__host__ __device__ inline c32 operator*(c32 a, c32 b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }

__host__ __device__ inline double conj_(double a) { return a; }
__host__ __device__ inline float conj_(float a) { return a; }
__host__ __device__ inline c64 conj_(c64 a) { return {a.x, -a.y}; }
__host__ __device__ inline c32 conj_(c32 a) { return {a.x, -a.y}; }

__host__ __device__ inline double abs2(c64 a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ inline double cabs(c64 a) { return hypot(a.x, a.y); }

// Complex division by Smith's method; for purely real operands it reduces to one
// real division, so real problems see exactly the real arithmetic.
__host__ __device__ inline c64 cdiv(c64 a, c64 b) {
    if (fabs(b.y) <= fabs(b.x)) {
        double r = b.y / b.x;
        double d = b.x + b.y * r;
        return {(a.x + a.y * r) / d, (a.y - a.x * r) / d};
    }
    double r = b.x / b.y;
    double d = b.y + b.x * r;
    return {(a.x * r + a.y) / d, (a.y * r - a.x) / d};
}
__host__ __device__ inline bool cfinite(c64 a) { return isfinite(a.x) && isfinite(a.y); }
__host__ __device__ inline bool czero(c64 a) { return a.x == 0.0 && a.y == 0.0; }

// Storage-type traits.  R is the real type, cplx tells complex storage.
template <class T> struct Tr;
template <> struct Tr<double> { using R = double; static constexpr bool cplx = false; };
template <> struct Tr<float> { using R = float; static constexpr bool cplx = false; };
template <> struct Tr<c64> { using R = double; static constexpr bool cplx = true; };
template <> struct Tr<c32> { using R = float; static constexpr bool cplx = true; };

// widen to the FP64 accumulation type
__host__ __device__ inline c64 up(double a) { return {a, 0.0}; }
__host__ __device__ inline c64 up(float a) { return {(double)a, 0.0}; }
__host__ __device__ inline c64 up(c64 a) { return a; }
__host__ __device__ inline c64 up(c32 a) { return {(double)a.x, (double)a.y}; }

// narrow an FP64 (complex) coefficient to storage type
template <class T> __host__ __device__ inline T down(c64 v);
template <> __host__ __device__ inline double down<double>(c64 v) { return v.x; }
template <> __host__ __device__ inline float down<float>(c64 v) { return (float)v.x; }
template <> __host__ __device__ inline c64 down<c64>(c64 v) { return v; }
template <> __host__ __device__ inline c32 down<c32>(c64 v) { return {(float)v.x, (float)v.y}; }

// Streaming load with the non-temporal hint: blocks read once per pass are not
// kept in the caches (measured 7-14% faster for the n x s block kernels).
template <class T> __device__ inline T ld_nt(const T* p) { return __builtin_nontemporal_load(p); }
template <> __device__ inline c64 ld_nt<c64>(const c64* p) {
    typedef double v2 __attribute__((ext_vector_type(2)));
    const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
    return {v.x, v.y};
}
template <> __device__ inline c32 ld_nt<c32>(const c32* p) {
    typedef float v2 __attribute__((ext_vector_type(2)));
    const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
    return {v.x, v.y};
}

template <class T> __host__ __device__ inline T zero();
template <> __host__ __device__ inline double zero<double>() { return 0.0; }
template <> __host__ __device__ inline float zero<float>() { return 0.0f; }
template <> __host__ __device__ inline c64 zero<c64>() { return {0.0, 0.0}; }
template <> __host__ __device__ inline c32 zero<c32>() { return {0.0f, 0.0f}; }

// a*b + c in storage precision
__device__ inline double fma_(double a, double b, double c) { return fma(a, b, c); }
__device__ inline float fma_(float a, float b, float c) { return fmaf(a, b, c); }
__device__ inline c64 fma_(c64 a, c64 b, c64 c) {
    return {fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y))};
}
__device__ inline c32 fma_(c32 a, c32 b, c32 c) {
    return {fmaf(a.x, b.x, fmaf(-a.y, b.y, c.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, c.y))};
}
__device__ inline double mul_(double a, double b) { return a * b; }
__device__ inline float mul_(float a, float b) { return a * b; }
__device__ inline c64 mul_(c64 a, c64 b) { return a * b; }
__device__ inline c32 mul_(c32 a, c32 b) { return a * b; }
__device__ inline double add_(double a, double b) { return a + b; }
__device__ inline float add_(float a, float b) { return a + b; }
__device__ inline c64 add_(c64 a, c64 b) { return a + b; }
__device__ inline c32 add_(c32 a, c32 b) { return a + b; }
__device__ inline double sub_(double a, double b) { return a - b; }
__device__ inline float sub_(float a, float b) { return a - b; }
__device__ inline c64 sub_(c64 a, c64 b) { return a - b; }
__device__ inline c32 sub_(c32 a, c32 b) { return a - b; }

// acc += conj(a) * b in FP64
template <class T> __device__ inline void dot_acc(c64& acc, T a, T b) {
    c64 A = up(a), B = up(b);
    acc.x = fma(A.x, B.x, fma(A.y, B.y, acc.x));
    acc.y = fma(A.x, B.y, fma(-A.y, B.x, acc.y));
}
template <class T> __device__ inline void nrm_acc(double& acc, T a) {
    c64 A = up(a);
    acc = fma(A.x, A.x, fma(A.y, A.y, acc));
}

// ---------------------------------------------------------------- control block
// Device-resident iteration state.  Every kernel of an iteration returns at
// entry once `done` is set, so the host may enqueue iterations ahead of the
// convergence test and the iteration count stays exact.
struct Ctl {
    int done;           // 1 once the iteration has stopped
    int status;         // 0 converged, 1 running / not converged, 2 breakdown
    int iter;           // completed iterations
    int bd_iter;        // iteration of a breakdown, else -1
    int maxit;
    int qr_shift[4];    // per QR slot: 1 when the shifted first CholeskyQR pass was used
    int pad;
    double tol;
    double nr0;         // ||R_0||_F
    double res;         // latest recursive ||R_k||_F
    double div_limit;   // > 0: stop as diverged once ||R_k|| > div_limit * ||R_0|| (inner solves)
};

enum { ST_OK = 0, ST_RUNNING = 1, ST_BREAKDOWN = 2 };

__device__ inline bool stopped(const Ctl* c) { return c != nullptr && c->done != 0; }

// ---------------------------------------------------------------- reductions
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum K complex values over the workgroup and store them at out[0..K).
// Order: butterfly within each wave, then waves 0..3 in order.
template <int K>
__device__ inline void block_reduce_store(c64 (&v)[K], c64* out) {
    __shared__ c64 sm[kWaves][K > 0 ? K : 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double a = wave_sum(v[k].x), b = wave_sum(v[k].y);
        if (lane == 0) sm[w][k] = {a, b};
    }
    __syncthreads();
    if (threadIdx.x < K) {
        c64 t = sm[0][threadIdx.x];
#pragma unroll
        for (int i = 1; i < kWaves; ++i) t = t + sm[i][threadIdx.x];
        out[threadIdx.x] = t;
    }
}

// In a single workgroup (any size that is a multiple of 64, at most 256): sum K
// values over `np` per-block partials laid out [block][K]; result in res[0..K)
// (shared memory), visible after return.  Fixed order: strided per thread over
// four accumulators, butterfly within each wave, waves in order.
template <int K>
__device__ inline void sum_partials(const c64* __restrict__ part, int np, c64* res) {
    __shared__ c64 sm[kWaves][K];
    c64 v[K], acc[4][K];   // four independent accumulators keep four loads in flight
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int k = 0; k < K; ++k) acc[u][k] = {0.0, 0.0};
    const int st = blockDim.x;
    int b = threadIdx.x;
    for (; b + 3 * st < np; b += 4 * st) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k = 0; k < K; ++k) acc[u][k] = acc[u][k] + part[(size_t)(b + u * st) * K + k];
    }
    for (; b < np; b += st) {
#pragma unroll
        for (int k = 0; k < K; ++k) acc[0][k] = acc[0][k] + part[(size_t)b * K + k];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = (acc[0][k] + acc[1][k]) + (acc[2][k] + acc[3][k]);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double a = wave_sum(v[k].x), b = wave_sum(v[k].y);
        if (lane == 0) sm[w][k] = {a, b};
    }
    __syncthreads();
    if (threadIdx.x < K) {
        c64 t = sm[0][threadIdx.x];
        for (int i = 1; i < nw; ++i) t = t + sm[i][threadIdx.x];
        res[threadIdx.x] = t;
    }
    __syncthreads();
}

// FP64 value type of the block kernels and accumulators: double for real storage, c64 for complex.
template <class T> struct VT { using type = c64; };
template <> struct VT<double> { using type = double; };
template <> struct VT<float> { using type = double; };
template <class T> using Val = typename VT<T>::type;

__device__ inline double vup(double a) { return a; }
__device__ inline double vup(float a) { return (double)a; }
__device__ inline c64 vup(c64 a) { return a; }
__device__ inline c64 vup(c32 a) { return up(a); }
template <class T> __device__ inline T vdown(double v);
template <> __device__ inline double vdown<double>(double v) { return v; }
template <> __device__ inline float vdown<float>(double v) { return (float)v; }
template <class T> __device__ inline T vdown(c64 v) { return down<T>(v); }
template <class Vt> __device__ inline Vt vzero();
template <> __device__ inline double vzero<double>() { return 0.0; }
template <> __device__ inline c64 vzero<c64>() { return {0.0, 0.0}; }
__device__ inline double vfma(double a, double b, double c) { return fma(a, b, c); }
__device__ inline c64 vfma(c64 a, c64 b, c64 c) {
    return {fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y))};
}

// ---------------------------------------------------------------- MFMA Gram
// Gram accumulation G += conj(Y)^T X over rows with v_mfma_f64_16x16x4f64.
// Lane layout ("tile-16"): a wave covers 4 rows; lane l holds row l/16 of them,
// columns (l%16) + 16 j, j < J.  That is exactly the MFMA A operand layout
// (A[i][k] in lane i + 16k, i = column of Y, k = row) and B operand layout
// (B[k][j] in lane j + 16k), so no data movement is needed.  The 16x16 result
// D[i][j] sits in lane j + 16 (i % 4), register i / 4 (checked on gfx950).
typedef double d4 __attribute__((ext_vector_type(4)));

template <int J, bool CPLX>
struct GramAcc {
    d4 re[J][J];
    d4 im[J][J];
    __device__ inline void clear() {
#pragma unroll
        for (int a = 0; a < J; ++a)
#pragma unroll
            for (int b = 0; b < J; ++b) {
                re[a][b] = d4{0.0, 0.0, 0.0, 0.0};
                im[a][b] = d4{0.0, 0.0, 0.0, 0.0};
            }
    }
    // y, x: this lane's elements (already zero for padding / rows past n)
    __device__ inline void add(const c64 (&y)[J], const c64 (&x)[J]) {
#pragma unroll
        for (int a = 0; a < J; ++a)
#pragma unroll
            for (int b = 0; b < J; ++b) {
                re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(y[a].x, x[b].x, re[a][b], 0, 0, 0);
                if (CPLX) {
                    re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(y[a].y, x[b].y, re[a][b], 0, 0, 0);
                    im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(y[a].x, x[b].y, im[a][b], 0, 0, 0);
                    im[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-y[a].y, x[b].x, im[a][b], 0, 0, 0);
                }
            }
    }
    // real operands
    __device__ inline void add(const double (&y)[J], const double (&x)[J]) {
#pragma unroll
        for (int a = 0; a < J; ++a)
#pragma unroll
            for (int b = 0; b < J; ++b) re[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(y[a], x[b], re[a][b], 0, 0, 0);
    }
    // Sum the 4 waves' partial Grams and write the s x s result (row-major,
    // G[a][b] at out[a*s+b]) for this workgroup.  `lds` must hold
    // (16J)^2 c64.  Must be called by the whole workgroup.
    __device__ inline void store(int s, c64* lds, c64* out) {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        const int S = 16 * J;
        for (int ww = 0; ww < kWaves; ++ww) {
            if (w == ww) {
#pragma unroll
                for (int a = 0; a < J; ++a)
#pragma unroll
                    for (int b = 0; b < J; ++b)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            int i = 16 * a + 4 * v + (lane >> 4);
                            int j = 16 * b + (lane & 15);
                            c64 val = {re[a][b][v], CPLX ? im[a][b][v] : 0.0};
                            if (ww == 0) lds[i * S + j] = val;
                            else lds[i * S + j] = lds[i * S + j] + val;
                        }
            }
            __syncthreads();
        }
        for (int e = threadIdx.x; e < s * s; e += kBlock) {
            int a = e / s, b = e - a * s;
            out[e] = lds[a * S + b];
        }
        __syncthreads();
    }
};

// Workgroup -> work-chunk mapping that keeps consecutive chunks on the same XCD
// (workgroups are dispatched round-robin over the 8 XCDs, each with its own L2):
// workgroup b runs logical chunk (b % 8) * (nb / 8) + b / 8.  nb % 8 == 0.
__device__ inline int xcd_chunk(int b, int nb) { return (b & 7) * (nb >> 3) + (b >> 3); }

}  // namespace skr
