// Gl-BiCG (Algorithm 2), eGl-BiCG (Algorithm 4) and Gl-BiCGStab (Section 4)
// for small systems, every iteration in one kernel launch on one workgroup.
//
// With n <= 1024 rows, one workgroup of 1024 threads holds the whole block
// system: thread i keeps row i of X, R, P and of the shadow R^, P^ (or the
// shadow vector entries r^_i, p^_i of eGl-BiCG) in registers.  The two blocks
// the products gather from, P and P^ (p^), are written to LDS at the start of
// each iteration; row i of A P and of A^H P^ is then formed from the row's
// stored entries and the LDS rows they name.  Traces and norms are summed in
// FP64 in a fixed order (within each wave, then over the 16 wave sums), so
// every thread holds the same bits and takes the same branch.  The stopping test, breakdown rules and history are those of the
// general schedule (end_of_iteration, bad_den), so the loop ends at
// convergence, breakdown or maxit in every wave at once.  Three barriers per
// iteration (after the LDS writes, and in the two workgroup sums: sigma, then
// ||R||^2 with rho') replace the six dependent launches per iteration that
// dominate small systems on the general schedule.
#pragma once

#include "blk.hpp"
#include "common.hpp"
#include "glk.hpp"
#include "small.hpp"
#include "spmm.hpp"

namespace skr {

constexpr int kSmallThreads = 1024;
constexpr int kSmallMaxRows = kSmallThreads;
// widest block the register budget of 1024 threads (128 VGPRs each) holds
// without spilling: seven rows of s values (X, R, P, R^, P^, A P, A^H P^)
template <class T> struct SmallMaxS { static constexpr int value = Tr<T>::cplx ? 2 : 4; };

// conj(a) * b + acc and |a|^2 + acc in the FP64 value type (real arithmetic
// for real data)
__device__ inline double sdot(double a, double b, double acc) { return fma(a, b, acc); }
__device__ inline c64 sdot(c64 a, c64 b, c64 acc) {
    return {fma(a.x, b.x, fma(a.y, b.y, acc.x)), fma(a.x, b.y, fma(-a.y, b.x, acc.y))};
}
__device__ inline double snrm(double a, double acc) { return fma(a, a, acc); }
__device__ inline double snrm(c64 a, double acc) { return fma(a.x, a.x, fma(a.y, a.y, acc)); }
// Sums over a wave without LDS traffic: DPP exchanges inside each 16-lane row
// (quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror; each
// step adds a lane's value and its partner's, which gives both lanes the same
// bits), then the four row sums read as scalars and added in a fixed order.
template <int CTRL>
__device__ inline double dpp64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline double row16_sum(double v) {
    v += dpp64<0xB1>(v);
    v += dpp64<0x4E>(v);
    v += dpp64<0x141>(v);
    v += dpp64<0x140>(v);
    return v;
}
__device__ inline double lane64(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline double swave(double v) {
    v = row16_sum(v);
    return (lane64(v, 0) + lane64(v, 16)) + (lane64(v, 32) + lane64(v, 48));
}
__device__ inline c64 swave(c64 v) { return {swave(v.x), swave(v.y)}; }
// the sum of the 16 values in lanes 0..15 (every row holds the same 16)
__device__ inline double srow(double v) { return lane64(row16_sum(v), 0); }
__device__ inline c64 srow(c64 v) { return {srow(v.x), srow(v.y)}; }
__device__ inline c64 sc64(double v) { return {v, 0.0}; }
__device__ inline c64 sc64(c64 v) { return v; }

// Workgroup sums with one barrier each.  Every thread receives the totals.
// Order: the wave sums above, then the same sum over the 16 wave sums, which
// every wave forms from the same inputs in the same order, so all threads hold
// the same bits.  The slots
// are read after the barrier and not written again until the caller has passed
// another barrier (each call site owns its slots, and consecutive uses of one
// site are separated by the barriers of the others).
template <class V>
__device__ inline V small_allreduce(V v, V* red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v = swave(v);
    if (lane == 0) red[w] = v;
    __syncthreads();
    return srow(red[lane & 15]);
}

template <class V>
__device__ inline void small_allreduce2(double& a, V& b, double* ra, V* rb) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    a = swave(a);
    b = swave(b);
    if (lane == 0) {
        ra[w] = a;
        rb[w] = b;
    }
    __syncthreads();
    a = srow(ra[lane & 15]);
    b = srow(rb[lane & 15]);
}

// entries a row's product loads per round (together, the first round before
// the barrier): 2 real / 1 complex measured fastest, wider rounds cost more
// registers than their overlapped latency saves
template <class T> struct SmallBatch { static constexpr int value = Tr<T>::cplx ? 1 : 2; };

// Column indices and values of entries k0 .. min(k0 + KB, k1) - 1 of a CSR
// operand (the rest left unset: the consumer tests k < k1).
template <class T, int KB>
__device__ inline void small_fetch(const CsrOp<T>& M, int k0, int k1, int (&cc)[KB], T (&vv)[KB]) {
#pragma unroll
    for (int u = 0; u < KB; ++u) {
        if (k0 + u < k1) {
            cc[u] = M.ci[k0 + u];
            vv[u] = M.va[k0 + u];
        }
    }
}

// R0 (preprocessed) in rhs, the correction D written to x.  Dynamic LDS: P
// (n x s) then P^ (n x s, or n for the economic variant).  The host has
// written tol and maxit to ctl; thread 0 keeps ctl and the history, and every
// thread takes the same stopping decisions from the same sums.
template <class T, bool ECON, int S>
__global__ __launch_bounds__(kSmallThreads) void k_small_bicg(Ctl* ctl, double* hist, CsrOp<T> A, CsrOp<T> AH,
                                                              const T* __restrict__ rhs, T* __restrict__ x) {
    constexpr int s = S;
    constexpr int SM = S;
    constexpr int NW = kSmallThreads / 64;
    constexpr int KB = SmallBatch<T>::value;
    static_assert(NW == 16, "the workgroup sums take one 16-lane row of wave sums");
    using V = Val<T>;   // double for real data, c64 for complex
    extern __shared__ c64 dyn[];
    T* Pl = reinterpret_cast<T*>(dyn);
    T* Phl = Pl + (size_t)A.n * s;
    __shared__ V red_sig[NW], red_rho[NW];
    __shared__ double red_nrm[NW];
    const int n = A.n;
    const int i = threadIdx.x;
    const bool row = i < n;
    const double tol = ctl->tol;
    const int maxit = ctl->maxit;
    // the row's entry ranges in A and A^H (fixed for the whole solve)
    const int a0 = row ? A.rp[i] : 0, a1 = row ? A.rp[i + 1] : 0;
    const int h0 = row ? AH.rp[i] : 0, h1 = row ? AH.rp[i + 1] : 0;
    T X[SM], R[SM], P[SM], Rh[ECON ? 1 : SM], Ph[ECON ? 1 : SM];
    T rh = zero<T>(), ph = zero<T>();
#pragma unroll
    for (int c = 0; c < SM; ++c) {
        X[c] = zero<T>();
        R[c] = row ? rhs[(size_t)i * s + c] : zero<T>();
        P[c] = R[c];
        if constexpr (!ECON) {
            Rh[c] = R[c];
            Ph[c] = R[c];
        }
    }
    if constexpr (ECON) {   // shadow: the arithmetic mean of the initial residual columns
        V sum = vzero<V>();
#pragma unroll
        for (int c = 0; c < SM; ++c)
            sum = sum + vup(R[c]);
        rh = row ? vdown<T>((1.0 / s) * sum) : zero<T>();
        ph = rh;
    }
    // ||R0||^2 and rho = tr(R^^H R) (or sum(r^^H R))
    double nr = 0.0;
    V rho = vzero<V>();
#pragma unroll
    for (int c = 0; c < SM; ++c) {
        nr = snrm(R[c], nr);
        rho = sdot(ECON ? rh : Rh[ECON ? 0 : c], R[c], rho);
    }
    small_allreduce2(nr, rho, red_nrm, red_rho);
    const double nr0 = sqrt(nr);
    bool go = nr0 > 0.0 && isfinite(nr0) && maxit > 0;
    if (threadIdx.x == 0) {
        ctl->nr0 = nr0;
        ctl->res = nr0;
        ctl->iter = 0;
        ctl->bd_iter = -1;
        hist[0] = 1.0;
        ctl->status = !(nr0 > 0.0) ? ST_OK : (!isfinite(nr0) ? ST_BREAKDOWN : ST_RUNNING);
        ctl->done = go ? 0 : 1;
    }
    int it = 0;
    while (go) {
        // this row's first KB entries of A and A^H: loaded before the barrier,
        // so their latency overlaps the LDS writes and the wait
        int ca[KB], ch[KB];
        T va[KB], vh[KB];
        small_fetch(A, a0, a1, ca, va);
        small_fetch(AH, h0, h1, ch, vh);
        // the blocks the products gather from
        if (row) {
#pragma unroll
            for (int c = 0; c < SM; ++c) {
                Pl[(size_t)i * s + c] = P[c];
                if constexpr (!ECON) Phl[(size_t)i * s + c] = Ph[c];
            }
            if constexpr (ECON) Phl[i] = ph;
        }
        __syncthreads();
        // Q = A P, Z^ = A^H P^ (z^ = A^H p^), sigma = tr(P^^H Q) (sum(p^^H Q));
        // entries in ascending order, KB at a time
        T Q[SM], Zh[ECON ? 1 : SM];
        T zh = zero<T>();
#pragma unroll
        for (int c = 0; c < SM; ++c) {
            Q[c] = zero<T>();
            if constexpr (!ECON) Zh[c] = zero<T>();
        }
        for (int k = a0;;) {
#pragma unroll
            for (int u = 0; u < KB; ++u) {
                if (k + u < a1) {
                    const T* pr = Pl + (size_t)ca[u] * s;
#pragma unroll
                    for (int c = 0; c < SM; ++c)
                        Q[c] = fma_(va[u], pr[c], Q[c]);
                }
            }
            k += KB;
            if (k >= a1) break;
            small_fetch(A, k, a1, ca, va);
        }
        for (int k = h0;;) {
#pragma unroll
            for (int u = 0; u < KB; ++u) {
                if (k + u < h1) {
                    if constexpr (ECON) {
                        zh = fma_(vh[u], Phl[ch[u]], zh);
                    } else {
                        const T* pr = Phl + (size_t)ch[u] * s;
#pragma unroll
                        for (int c = 0; c < SM; ++c)
                            Zh[c] = fma_(vh[u], pr[c], Zh[c]);
                    }
                }
            }
            k += KB;
            if (k >= h1) break;
            small_fetch(AH, k, h1, ch, vh);
        }
        V sg = vzero<V>();
#pragma unroll
        for (int c = 0; c < SM; ++c)
            sg = sdot(ECON ? ph : Ph[ECON ? 0 : c], Q[c], sg);
        const c64 sigma = sc64(small_allreduce(sg, red_sig));
        if (bad_den(sigma)) {
            if (threadIdx.x == 0) set_breakdown(ctl);
            break;
        }
        const c64 alpha = cdiv(sc64(rho), sigma);
        const T a = down<T>(alpha), ma = down<T>(-alpha), mac = down<T>(-conj_(alpha));
        if constexpr (ECON) rh = fma_(mac, zh, rh);
        nr = 0.0;
        V rhon = vzero<V>();
#pragma unroll
        for (int c = 0; c < SM; ++c) {
            X[c] = fma_(a, P[c], X[c]);
            R[c] = fma_(ma, Q[c], R[c]);
            if constexpr (!ECON) Rh[c] = fma_(mac, Zh[c], Rh[c]);
            nr = snrm(R[c], nr);
            rhon = sdot(ECON ? rh : Rh[ECON ? 0 : c], R[c], rhon);
        }
        small_allreduce2(nr, rhon, red_nrm, red_rho);
        // the stopping rule of end_of_iteration, taken by every thread
        ++it;
        const double res = sqrt(nr);
        go = !(res <= tol * nr0) && isfinite(res) && it < maxit;
        if (threadIdx.x == 0) (void)end_of_iteration(ctl, hist, nr);
        if (go && bad_den(sc64(rho))) {
            if (threadIdx.x == 0) set_breakdown(ctl);
            go = false;
        }
        if (!go) break;
        const c64 beta = cdiv(sc64(rhon), sc64(rho));
        rho = rhon;
        const T b = down<T>(beta), bc = down<T>(conj_(beta));
#pragma unroll
        for (int c = 0; c < SM; ++c) {
            P[c] = fma_(b, P[c], R[c]);
            if constexpr (!ECON) Ph[c] = fma_(bc, Ph[c], Rh[c]);
        }
        if constexpr (ECON) ph = fma_(bc, ph, rh);
    }
    if (row) {
#pragma unroll
        for (int c = 0; c < SM; ++c)
            x[(size_t)i * s + c] = X[c];
    }
}

// Gl-BiCGStab (the global BiCGStab of Section 4) on the same single-workgroup
// layout: thread i keeps row i of X, R, R~ (the shadow R0), P, V = A P, S and
// T = A S.  The two products gather from one LDS block, P first and then S.
// Five barriers per iteration: after each LDS write, and in the three workgroup
// sums (sigma = tr(R~^H V); tr(T^H S) with tr(T^H T); ||R||^2 with rho').
template <class T, int S>
__global__ __launch_bounds__(kSmallThreads) void k_small_bicgstab(Ctl* ctl, double* hist, CsrOp<T> A,
                                                                  const T* __restrict__ rhs, T* __restrict__ x) {
    constexpr int s = S;
    constexpr int NW = kSmallThreads / 64;
    constexpr int KB = SmallBatch<T>::value;
    static_assert(NW == 16, "the workgroup sums take one 16-lane row of wave sums");
    using V = Val<T>;
    extern __shared__ c64 dyn[];
    T* Bl = reinterpret_cast<T*>(dyn);   // P, then S, of every row
    __shared__ V red_sig[NW], red_num[NW], red_rho[NW];
    __shared__ double red_den[NW], red_nrm[NW];
    const int n = A.n;
    const int i = threadIdx.x;
    const bool row = i < n;
    const double tol = ctl->tol;
    const int maxit = ctl->maxit;
    const int a0 = row ? A.rp[i] : 0, a1 = row ? A.rp[i + 1] : 0;
    // row i of A times the LDS block (entries in ascending order, KB at a time)
    auto product = [&](T (&Y)[S]) {
        int ca[KB];
        T va[KB];
#pragma unroll
        for (int c = 0; c < S; ++c) Y[c] = zero<T>();
        small_fetch(A, a0, a1, ca, va);
        for (int k = a0;;) {
#pragma unroll
            for (int u = 0; u < KB; ++u) {
                if (k + u < a1) {
                    const T* pr = Bl + (size_t)ca[u] * s;
#pragma unroll
                    for (int c = 0; c < S; ++c) Y[c] = fma_(va[u], pr[c], Y[c]);
                }
            }
            k += KB;
            if (k >= a1) break;
            small_fetch(A, k, a1, ca, va);
        }
    };
    T X[S], R[S], Rt[S], P[S];
#pragma unroll
    for (int c = 0; c < S; ++c) {
        X[c] = zero<T>();
        R[c] = row ? rhs[(size_t)i * s + c] : zero<T>();
        Rt[c] = R[c];
        P[c] = R[c];
    }
    double nr = 0.0;
    V rho = vzero<V>();
#pragma unroll
    for (int c = 0; c < S; ++c) {
        nr = snrm(R[c], nr);
        rho = sdot(Rt[c], R[c], rho);
    }
    small_allreduce2(nr, rho, red_nrm, red_rho);
    const double nr0 = sqrt(nr);
    bool go = nr0 > 0.0 && isfinite(nr0) && maxit > 0;
    if (threadIdx.x == 0) {
        ctl->nr0 = nr0;
        ctl->res = nr0;
        ctl->iter = 0;
        ctl->bd_iter = -1;
        hist[0] = 1.0;
        ctl->status = !(nr0 > 0.0) ? ST_OK : (!isfinite(nr0) ? ST_BREAKDOWN : ST_RUNNING);
        ctl->done = go ? 0 : 1;
    }
    int it = 0;
    while (go) {
        if (row) {
#pragma unroll
            for (int c = 0; c < S; ++c) Bl[(size_t)i * s + c] = P[c];
        }
        __syncthreads();
        T Vr[S];
        product(Vr);   // V = A P
        V sg = vzero<V>();
#pragma unroll
        for (int c = 0; c < S; ++c) sg = sdot(Rt[c], Vr[c], sg);
        const c64 sigma = sc64(small_allreduce(sg, red_sig));   // also orders the reads of P before the writes of S
        if (bad_den(sigma)) {
            if (threadIdx.x == 0) set_breakdown(ctl);
            break;
        }
        const c64 alpha = cdiv(sc64(rho), sigma);
        const T a = down<T>(alpha), ma = down<T>(-alpha);
        T Sr[S];
#pragma unroll
        for (int c = 0; c < S; ++c) Sr[c] = fma_(ma, Vr[c], R[c]);
        if (row) {
#pragma unroll
            for (int c = 0; c < S; ++c) Bl[(size_t)i * s + c] = Sr[c];
        }
        __syncthreads();
        T Tr[S];
        product(Tr);   // T = A S
        V num = vzero<V>();
        double den = 0.0;
#pragma unroll
        for (int c = 0; c < S; ++c) {
            num = sdot(Tr[c], Sr[c], num);
            den = snrm(Tr[c], den);
        }
        small_allreduce2(den, num, red_den, red_num);   // orders the reads of S before the next writes
        if (bad_den(c64{den, 0.0})) {
            if (threadIdx.x == 0) set_breakdown(ctl);
            break;
        }
        const c64 omega = cdiv(sc64(num), c64{den, 0.0});
        const T w = down<T>(omega), mw = down<T>(-omega);
        nr = 0.0;
        V rhon = vzero<V>();
#pragma unroll
        for (int c = 0; c < S; ++c) {
            X[c] = fma_(w, Sr[c], fma_(a, P[c], X[c]));
            R[c] = fma_(mw, Tr[c], Sr[c]);
            nr = snrm(R[c], nr);
            rhon = sdot(Rt[c], R[c], rhon);
        }
        small_allreduce2(nr, rhon, red_nrm, red_rho);
        ++it;
        const double res = sqrt(nr);
        go = !(res <= tol * nr0) && isfinite(res) && it < maxit;
        if (threadIdx.x == 0) (void)end_of_iteration(ctl, hist, nr);
        if (go && (bad_den(sc64(rho)) || bad_den(omega))) {
            if (threadIdx.x == 0) set_breakdown(ctl);
            go = false;
        }
        if (!go) break;
        const c64 beta = cdiv(sc64(rhon), sc64(rho)) * cdiv(alpha, omega);
        rho = rhon;
        const T b = down<T>(beta);
#pragma unroll
        for (int c = 0; c < S; ++c) P[c] = fma_(b, fma_(mw, Vr[c], P[c]), R[c]);
    }
    if (row) {
#pragma unroll
        for (int c = 0; c < S; ++c) x[(size_t)i * s + c] = X[c];
    }
}

// acc + z m for one entry of a row times an s x s matrix (the matrix is held as
// complex FP64; its imaginary parts are zero for real data)
__device__ inline double smac(double z, c64 m, double acc) { return fma(z, m.x, acc); }
__device__ inline c64 smac(c64 z, c64 m, c64 acc) {
    return {fma(z.x, m.x, fma(-z.y, m.y, acc.x)), fma(z.x, m.y, fma(z.y, m.x, acc.y))};
}

// The QR preprocessing of the block of initial residuals (Section 5) for the
// single-workgroup path, in one launch: thread i keeps row i of Z.  The same
// shifted CholeskyQR2 as the general schedule's k_qr_chol passes (the same
// factorisations, shift and breakdown tests, through the same device
// functions), on Grams summed in the fixed order of the small kernels: pass 1
// factors Z^H Z (shifted if the plain factorisation fails), pass 2 the Gram of
// Q1 = Z S1^{-1}, pass 3 (shifted case only) that of Q2 = Q1 S2^{-1}.  Z is
// overwritten by Q and the R factor S_k ... S_1 is written to M_S and M_RB; a
// failed factorisation records a breakdown in ctl and leaves Z unchanged.
template <class T, int S>
__global__ __launch_bounds__(kSmallThreads) void k_small_qr(Ctl* ctl, int n, T* __restrict__ Z, c64* __restrict__ mats,
                                                            double u) {
    constexpr int s = S, ss = S * S, NW = kSmallThreads / 64;
    using V = Val<T>;
    __shared__ V red[NW][ss];
    __shared__ c64 G[ss], Am[ss], Bm[ss], Rm[ss], Dm[ss];
    __shared__ int flag;
    const int i = threadIdx.x, lane = i & 63, w = i >> 6;
    T q[S];
#pragma unroll
    for (int b = 0; b < S; ++b) q[b] = T{};
    if (i < n) {
#pragma unroll
        for (int b = 0; b < S; ++b) q[b] = Z[(size_t)i * s + b];
    }
    // G = q^H q over all rows: each wave's sums, then the 16 wave sums in order
    auto gram = [&]() {
#pragma unroll
        for (int a = 0; a < S; ++a) {
#pragma unroll
            for (int b = 0; b < S; ++b) {
                const V g = swave(sdot(q[a], q[b], V{}));
                if (lane == 0) red[w][a * S + b] = g;
            }
        }
        __syncthreads();
        if (i < ss) {
            V t = red[0][i];
            for (int k = 1; k < NW; ++k) t = t + red[k][i];
            G[i] = sc64(t);
        }
        __syncthreads();
    };
    // q = q M (M upper triangular, in LDS)
    auto apply = [&](const c64* M) {
        T r[S];
#pragma unroll
        for (int b = 0; b < S; ++b) {
            T acc{};
#pragma unroll
            for (int a = 0; a < S; ++a) acc = smac(q[a], M[a * S + b], acc);
            r[b] = acc;
        }
#pragma unroll
        for (int b = 0; b < S; ++b) q[b] = r[b];
    };
    gram();
    sm_copy(Am, G, ss);
    int ok = sm_cholesky(Am, s, 0.0, &flag, 1e4 * u);
    int shifted = 0;
    if (!ok) {
        double trg = 0.0;
        for (int k = 0; k < s; ++k) trg += G[k * s + k].x;
        const double shift = fmax(11.0 * ((double)n * s + (double)s * (s + 1)) * 0x1p-53, 1e3 * u) * trg;
        sm_copy(Am, G, ss);
        ok = sm_cholesky(Am, s, shift, &flag, fmax(1e2 * u, 1e-12));
        shifted = 1;
    }
    if (!ok) {   // uniform: every thread holds the same flag
        if (i == 0) set_breakdown(ctl);
        return;
    }
    sm_tri_inv_upper(Am, Bm, s);   // S1^{-1}
    sm_copy(Rm, Am, ss);
    apply(Bm);
    const int passes = shifted ? 3 : 2;
    for (int p = 2; p <= passes; ++p) {
        gram();
        sm_copy(Am, G, ss);
        ok = sm_cholesky(Am, s, 0.0, &flag, fmax(1e2 * u, 1e-12));
        if (!ok) {
            if (i == 0) set_breakdown(ctl);
            return;
        }
        sm_tri_inv_upper(Am, Bm, s);   // S_p^{-1}
        sm_gemm(Dm, Am, 0, Rm, 0, s);  // S_p (S_{p-1} ... S_1)
        sm_copy(Rm, Dm, ss);
        apply(Bm);
    }
    if (i < n) {
#pragma unroll
        for (int b = 0; b < S; ++b) Z[(size_t)i * s + b] = q[b];
    }
    if (i < ss) {
        mats[(size_t)M_S * ss + i] = Rm[i];
        mats[(size_t)M_RB * ss + i] = Rm[i];
    }
    if (i == 0) ctl->qr_shift[0] = shifted;
}

}  // namespace skr
