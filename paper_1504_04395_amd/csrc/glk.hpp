// Kernels of the global family: Gl-BiCG (Algorithm 2), eGl-BiCG (Algorithm 4),
// Gl-QMR / eGl-QMR (Sections 2 and 4) and Gl-BiCGStab (Sections 2-3).
//
// The global methods are the single-RHS methods applied to (I (x) A) x = b
// (eq. (global)); after matricisation every vector operation is an elementwise
// operation on the n x s blocks with one scalar coefficient, and every inner
// product is tr(Y^H X).  Those updates are "flat" kernels over the n*s
// elements; the economic variants carry one n-vector shadow, so their updates
// run row-wise (a group of L lanes per row) and the shadow entry of row i is
// combined with all s entries of the block row.
//
// Scalars (alpha, beta, omega, QMR's theta/gamma/eta, ...) live in a small
// device array `sc` (complex FP64) written by one-workgroup coefficient kernels
// and read by the update kernels, so no value crosses to the host inside the
// iteration.
#pragma once

#include "common.hpp"
#include "spmm.hpp"

namespace skr {

// indices into the scalar array sc[] (complex FP64)
enum {
    S_RHO = 0, S_ALPHA, S_BETA, S_OMEGA, S_SIGMA,
    // QMR
    Q_RHO, Q_XI, Q_DELTA, Q_EPS, Q_BETA, Q_GAMMA, Q_ETA, Q_THETA, Q_F, Q_CP, Q_CQ, Q_IRHO, Q_IXI,
    Q_RHON, Q_XIN, Q_DELTAN, Q_FIRST,
    S_COUNT
};

// Flat mapping: workgroup b owns elements [chunk*per, (chunk+1)*per).
struct Flat {
    size_t total;
    size_t per;
};

#define SKR_FLAT_LOOP(fl)                                                              \
    const size_t e0_ = (size_t)xcd_chunk(blockIdx.x, gridDim.x) * (fl).per;            \
    const size_t e1_ = (e0_ + (fl).per < (fl).total) ? e0_ + (fl).per : (fl).total;      \
    for (size_t e = e0_ + threadIdx.x; e < e1_; e += kBlock)

#define SKR_ROW_LOOP(ly, n, rpc)                                                       \
    const int lane = threadIdx.x & ((ly).L - 1);                                       \
    const int grp = threadIdx.x >> (ly).lgL;                                           \
    const int rpb_ = kBlock >> (ly).lgL;                                               \
    const int r0_ = xcd_chunk(blockIdx.x, gridDim.x) * (rpc);                          \
    const int r1_ = min((n), r0_ + (rpc));                                             \
    for (int base_ = r0_; base_ < r1_; base_ += rpb_)

__device__ inline void set_breakdown(Ctl* c) {
    c->status = ST_BREAKDOWN;
    c->bd_iter = c->iter;
    c->done = 1;
}
__device__ inline bool bad_den(c64 d) { return czero(d) || !cfinite(d); }

// Record ||R_k||, count the iteration and apply the stopping rule.  Returns
// true if the iteration continues.
__device__ inline bool end_of_iteration(Ctl* c, double* hist, double res2) {
    double res = sqrt(res2);
    c->iter += 1;
    c->res = res;
    hist[c->iter] = res / c->nr0;
    if (res <= c->tol * c->nr0) {
        c->status = ST_OK;
        c->done = 1;
        return false;
    }
    if (!isfinite(res)) {  // a non-finite residual only arises from a vanished denominator
        set_breakdown(c);
        return false;
    }
    if (c->div_limit > 0.0 && res > c->div_limit * c->nr0) {   // inner solves only
        set_breakdown(c);
        return false;
    }
    if (c->iter >= c->maxit) {
        c->status = ST_RUNNING;
        c->done = 1;
        return false;
    }
    return true;
}

// ------------------------------------------------------------------ init
// Initial residual norm from 2-wide partials (component 0 = ||R0||^2); stops
// immediately when R0 = 0.
__global__ __launch_bounds__(kScalar) void k_init_ctl2(Ctl* c, double* hist, const c64* part, int np) {
    __shared__ c64 r[2];
    sum_partials<2>(part, np, r);
    if (threadIdx.x == 0) {
        double nr0 = sqrt(r[0].x);
        c->nr0 = nr0;
        c->res = nr0;
        c->iter = 0;
        c->bd_iter = -1;
        hist[0] = 1.0;
        if (!(nr0 > 0.0)) {
            c->status = ST_OK;
            c->done = 1;
        } else if (!isfinite(nr0)) {
            c->status = ST_BREAKDOWN;
            c->done = 1;
        } else {
            c->status = ST_RUNNING;
            c->done = c->maxit <= 0 ? 1 : 0;
        }
    }
}

// part = ||Y||^2 and tr(Z^H Y) (flat)
template <class T>
__global__ __launch_bounds__(kBlock) void k_flat_nrm_dot(Flat fl, const T* __restrict__ Y, const T* __restrict__ Z,
                                                          c64* part) {
    c64 acc[2] = {{0.0, 0.0}, {0.0, 0.0}};
    SKR_FLAT_LOOP(fl) {
        T y = Y[e];
        nrm_acc(acc[0].x, y);
        if (Z) dot_acc(acc[1], Z[e], y);
    }
    block_reduce_store<2>(acc, part + (size_t)blockIdx.x * 2);
}

// Gram-free copy kernels
template <class T>
__global__ __launch_bounds__(kBlock) void k_copy(Flat fl, const T* __restrict__ src, T* __restrict__ d0,
                                                 T* __restrict__ d1, T* __restrict__ d2) {
    SKR_FLAT_LOOP(fl) {
        T v = src[e];
        if (d0) d0[e] = v;
        if (d1) d1[e] = v;
        if (d2) d2[e] = v;
    }
}
template <class T>
__global__ __launch_bounds__(kBlock) void k_fill0(Flat fl, T* __restrict__ d0, T* __restrict__ d1, T* __restrict__ d2,
                                                  T* __restrict__ d3) {
    SKR_FLAT_LOOP(fl) {
        if (d0) d0[e] = zero<T>();
        if (d1) d1[e] = zero<T>();
        if (d2) d2[e] = zero<T>();
        if (d3) d3[e] = zero<T>();
    }
}

// mean of each row's s entries: rh[i] = (1/s) sum_c R[i, c]
template <class T>
__global__ __launch_bounds__(kBlock) void k_row_mean(int n, int s, const T* __restrict__ R, T* __restrict__ rh) {
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    c64 acc = {0.0, 0.0};
    for (int c = 0; c < s; ++c) acc = acc + up(R[(size_t)i * s + c]);
    rh[i] = down<T>((1.0 / s) * acc);
}

// ---------------------------------------------------------- coefficient kernels
// sigma -> alpha = rho / sigma (Gl-BiCG, eGl-BiCG, Gl-BiCGStab)
__global__ __launch_bounds__(kScalar) void k_s_alpha(Ctl* c, const c64* part, int np, c64* sc) {
    if (stopped(c)) return;
    __shared__ c64 r[1];
    sum_partials<1>(part, np, r);
    if (threadIdx.x == 0) {
        c64 sig = r[0];
        if (bad_den(sig)) { set_breakdown(c); return; }
        sc[S_SIGMA] = sig;
        sc[S_ALPHA] = cdiv(sc[S_RHO], sig);
    }
}

// (||R||^2, rho') -> stopping test, beta = rho'/rho   (Gl-BiCG, eGl-BiCG)
__global__ __launch_bounds__(kScalar) void k_s_beta(Ctl* c, double* hist, const c64* part, int np, c64* sc) {
    if (stopped(c)) return;
    __shared__ c64 r[2];
    sum_partials<2>(part, np, r);
    if (threadIdx.x == 0) {
        if (!end_of_iteration(c, hist, r[0].x)) return;
        c64 rho = sc[S_RHO];
        if (bad_den(rho)) { set_breakdown(c); return; }
        sc[S_BETA] = cdiv(r[1], rho);
        sc[S_RHO] = r[1];
    }
}

// initial rho = tr(R^H R) (or sum(r^H R)) from partials, component 1
__global__ __launch_bounds__(kScalar) void k_s_rho0(const c64* part, int np, int comp, int ncomp, c64* sc) {
    __shared__ c64 r[2];
    sum_partials<2>(part, np, r);
    if (threadIdx.x == 0) sc[S_RHO] = r[comp];
    (void)ncomp;
}

// ---------------------------------------------------------- Gl-BiCG updates
// X += a P; R -= a Q; Rh -= conj(a) Zh; part = (||R||^2, tr(Rh^H R))
template <class T>
__global__ __launch_bounds__(kBlock) void k_glbicg_upd(const Ctl* ctl, Flat fl, const c64* sc, T* __restrict__ X,
                                                       T* __restrict__ R, T* __restrict__ Rh, const T* __restrict__ P,
                                                       const T* __restrict__ Q, const T* __restrict__ Zh, c64* part) {
    if (stopped(ctl)) return;
    const T a = down<T>(sc[S_ALPHA]);
    const T ma = down<T>(-sc[S_ALPHA]);
    const T mac = down<T>(-conj_(sc[S_ALPHA]));
    c64 acc[2] = {{0.0, 0.0}, {0.0, 0.0}};
    SKR_FLAT_LOOP(fl) {
        X[e] = fma_(a, P[e], X[e]);
        T r = fma_(ma, Q[e], R[e]);
        T rh = fma_(mac, Zh[e], Rh[e]);
        R[e] = r;
        Rh[e] = rh;
        nrm_acc(acc[0].x, r);
        dot_acc(acc[1], rh, r);
    }
    block_reduce_store<2>(acc, part + (size_t)blockIdx.x * 2);
}

// P = R + b P; Ph = Rh + conj(b) Ph
template <class T>
__global__ __launch_bounds__(kBlock) void k_glbicg_dir(const Ctl* ctl, Flat fl, const c64* sc, const T* __restrict__ R,
                                                       const T* __restrict__ Rh, T* __restrict__ P, T* __restrict__ Ph) {
    if (stopped(ctl)) return;
    const T b = down<T>(sc[S_BETA]);
    const T bc = down<T>(conj_(sc[S_BETA]));
    SKR_FLAT_LOOP(fl) {
        P[e] = fma_(b, P[e], R[e]);
        Ph[e] = fma_(bc, Ph[e], Rh[e]);
    }
}

// ---------------------------------------------------------- eGl-BiCG updates
// X += a P; R -= a Q; rh -= conj(a) zh; part = (||R||^2, sum(rh^H R))
template <class T>
__global__ __launch_bounds__(kBlock) void k_eglbicg_upd(const Ctl* ctl, Layout ly, int n, int rpc, const c64* sc,
                                                        T* __restrict__ X, T* __restrict__ R, T* __restrict__ rh,
                                                        const T* __restrict__ P, const T* __restrict__ Q,
                                                        const T* __restrict__ zh, c64* part) {
    if (stopped(ctl)) return;
    const T a = down<T>(sc[S_ALPHA]);
    const T ma = down<T>(-sc[S_ALPHA]);
    const T mac = down<T>(-conj_(sc[S_ALPHA]));
    const int s = ly.s;
    c64 acc[2] = {{0.0, 0.0}, {0.0, 0.0}};
    SKR_ROW_LOOP(ly, n, rpc) {
        const int i = base_ + grp;
        if (i < r1_) {
            const T rhi = fma_(mac, zh[i], rh[i]);
            for (int c = lane; c < s; c += ly.L) {
                size_t e = (size_t)i * s + c;
                X[e] = fma_(a, P[e], X[e]);
                T r = fma_(ma, Q[e], R[e]);
                R[e] = r;
                nrm_acc(acc[0].x, r);
                dot_acc(acc[1], rhi, r);
            }
            if (lane == 0) rh[i] = rhi;
        }
    }
    block_reduce_store<2>(acc, part + (size_t)blockIdx.x * 2);
}

// P = R + b P; ph = rh + conj(b) ph
template <class T>
__global__ __launch_bounds__(kBlock) void k_eglbicg_dir(const Ctl* ctl, Layout ly, int n, int rpc, const c64* sc,
                                                        const T* __restrict__ R, const T* __restrict__ rh,
                                                        T* __restrict__ P, T* __restrict__ ph) {
    if (stopped(ctl)) return;
    const T b = down<T>(sc[S_BETA]);
    const T bc = down<T>(conj_(sc[S_BETA]));
    const int s = ly.s;
    SKR_ROW_LOOP(ly, n, rpc) {
        const int i = base_ + grp;
        if (i < r1_) {
            for (int c = lane; c < s; c += ly.L) {
                size_t e = (size_t)i * s + c;
                P[e] = fma_(b, P[e], R[e]);
            }
            if (lane == 0) ph[i] = fma_(bc, ph[i], rh[i]);
        }
    }
}

// ---------------------------------------------------------- Gl-BiCGStab
// S = R - a V
template <class T>
__global__ __launch_bounds__(kBlock) void k_stab_s(const Ctl* ctl, Flat fl, const c64* sc, const T* __restrict__ R,
                                                   const T* __restrict__ V, T* __restrict__ S) {
    if (stopped(ctl)) return;
    const T ma = down<T>(-sc[S_ALPHA]);
    SKR_FLAT_LOOP(fl) { S[e] = fma_(ma, V[e], R[e]); }
}

// (tr(T^H S), tr(T^H T)) -> omega
__global__ __launch_bounds__(kScalar) void k_s_omega(Ctl* c, const c64* part, int np, c64* sc) {
    if (stopped(c)) return;
    __shared__ c64 r[2];
    sum_partials<2>(part, np, r);
    if (threadIdx.x == 0) {
        if (bad_den(r[1])) { set_breakdown(c); return; }
        sc[S_OMEGA] = cdiv(r[0], r[1]);
    }
}

// X += a P + w S; R = S - w T; part = (||R||^2, tr(Rt^H R))
template <class T>
__global__ __launch_bounds__(kBlock) void k_stab_upd(const Ctl* ctl, Flat fl, const c64* sc, T* __restrict__ X,
                                                     T* __restrict__ R, const T* __restrict__ Rt,
                                                     const T* __restrict__ P, const T* __restrict__ S,
                                                     const T* __restrict__ Tm, c64* part) {
    if (stopped(ctl)) return;
    const T a = down<T>(sc[S_ALPHA]);
    const T w = down<T>(sc[S_OMEGA]);
    const T mw = down<T>(-sc[S_OMEGA]);
    c64 acc[2] = {{0.0, 0.0}, {0.0, 0.0}};
    SKR_FLAT_LOOP(fl) {
        T sv = S[e];
        X[e] = fma_(w, sv, fma_(a, P[e], X[e]));
        T r = fma_(mw, Tm[e], sv);
        R[e] = r;
        nrm_acc(acc[0].x, r);
        dot_acc(acc[1], Rt[e], r);
    }
    block_reduce_store<2>(acc, part + (size_t)blockIdx.x * 2);
}

// stopping test, beta = (rho'/rho)(alpha/omega)
__global__ __launch_bounds__(kScalar) void k_s_stab_beta(Ctl* c, double* hist, const c64* part, int np, c64* sc) {
    if (stopped(c)) return;
    __shared__ c64 r[2];
    sum_partials<2>(part, np, r);
    if (threadIdx.x == 0) {
        if (!end_of_iteration(c, hist, r[0].x)) return;
        c64 rho = sc[S_RHO], w = sc[S_OMEGA];
        if (bad_den(rho) || bad_den(w)) { set_breakdown(c); return; }
        sc[S_BETA] = cdiv(r[1], rho) * cdiv(sc[S_ALPHA], w);
        sc[S_RHO] = r[1];
    }
}

// P = R + b (P - w V)
template <class T>
__global__ __launch_bounds__(kBlock) void k_stab_dir(const Ctl* ctl, Flat fl, const c64* sc, const T* __restrict__ R,
                                                     const T* __restrict__ V, T* __restrict__ P) {
    if (stopped(ctl)) return;
    const T b = down<T>(sc[S_BETA]);
    const T mw = down<T>(-sc[S_OMEGA]);
    SKR_FLAT_LOOP(fl) { P[e] = fma_(b, fma_(mw, V[e], P[e]), R[e]); }
}

// ---------------------------------------------------------- Gl-QMR / eGl-QMR
// Initial scalars: rho = ||Vt||, xi = ||Wt|| (economic: sqrt(s) ||wt||),
// delta_raw = tr(Wt^H Vt); part = (||Vt||^2, ||Wt||^2, tr(Wt^H Vt)).
__global__ __launch_bounds__(kScalar) void k_qmr_s0(Ctl* c, const c64* part, int np, c64* sc, double xscale) {
    if (stopped(c)) return;
    __shared__ c64 r[3];
    sum_partials<3>(part, np, r);
    if (threadIdx.x == 0) {
        double rho = sqrt(r[0].x), xi = sqrt(xscale * r[1].x);
        c64 delta = cdiv(r[2], c64{rho * xi, 0.0});
        if (!(rho > 0.0) || !(xi > 0.0) || !isfinite(rho) || !isfinite(xi) || bad_den(delta)) {
            set_breakdown(c);
            return;
        }
        sc[Q_RHO] = {rho, 0.0};
        sc[Q_XI] = {xi, 0.0};
        sc[Q_DELTA] = delta;
        sc[Q_IRHO] = {1.0 / rho, 0.0};
        sc[Q_IXI] = {1.0 / xi, 0.0};
        sc[Q_CP] = {0.0, 0.0};
        sc[Q_CQ] = {0.0, 0.0};
        sc[Q_GAMMA] = {1.0, 0.0};
        sc[Q_ETA] = {-1.0, 0.0};
        sc[Q_THETA] = {0.0, 0.0};
        sc[Q_F] = {0.0, 0.0};
    }
}

// epsilon -> beta = eps / delta
__global__ __launch_bounds__(kScalar) void k_qmr_s1(Ctl* c, const c64* part, int np, c64* sc) {
    if (stopped(c)) return;
    __shared__ c64 r[1];
    sum_partials<1>(part, np, r);
    if (threadIdx.x == 0) {
        c64 eps = r[0];
        if (bad_den(eps)) { set_breakdown(c); return; }
        sc[Q_EPS] = eps;
        sc[Q_BETA] = cdiv(eps, sc[Q_DELTA]);
    }
}

// (||Vt||^2, ||Wt||^2, tr(Wt^H Vt)) -> theta, gamma, eta, the D/S weight and
// the next iteration's direction coefficients.
__global__ __launch_bounds__(kScalar) void k_qmr_s2(Ctl* c, const c64* part, int np, c64* sc, double xscale) {
    if (stopped(c)) return;
    __shared__ c64 r[3];
    sum_partials<3>(part, np, r);
    if (threadIdx.x == 0) {
        c64 beta = sc[Q_BETA];
        double gp = sc[Q_GAMMA].x;
        if (bad_den(beta) || !(gp != 0.0) || !isfinite(gp)) { set_breakdown(c); return; }
        double rhon = sqrt(r[0].x), xin = sqrt(xscale * r[1].x);
        double theta = rhon / (gp * cabs(beta));
        double gamma = 1.0 / sqrt(1.0 + theta * theta);
        if (!(gamma != 0.0) || !isfinite(gamma)) { set_breakdown(c); return; }
        double rho = sc[Q_RHO].x;
        c64 etap = sc[Q_ETA];
        c64 eta = cdiv(-(rho * gamma * gamma) * etap, (gp * gp) * beta);
        double thp = sc[Q_THETA].x;
        double f = (thp * gamma) * (thp * gamma);
        sc[Q_ETA] = eta;
        sc[Q_F] = {f, 0.0};
        sc[Q_GAMMA] = {gamma, 0.0};
        sc[Q_THETA] = {theta, 0.0};
        // next iteration: V = Vt/rhon, W = Wt/xin, delta = tr(W^H V)
        c64 deltan = cdiv(r[2], c64{rhon * xin, 0.0});
        c64 eps = sc[Q_EPS];
        sc[Q_CP] = cdiv(xin * deltan, eps);
        sc[Q_CQ] = conj_(cdiv(rhon * deltan, eps));
        sc[Q_IRHO] = {1.0 / rhon, 0.0};
        sc[Q_IXI] = {1.0 / xin, 0.0};
        sc[Q_RHON] = {rhon, 0.0};
        sc[Q_XIN] = {xin, 0.0};
        sc[Q_DELTAN] = deltan;
    }
}

// ||R||^2 -> stopping test, then the next iteration's breakdown tests.
__global__ __launch_bounds__(kScalar) void k_qmr_s3(Ctl* c, double* hist, const c64* part, int np, c64* sc) {
    if (stopped(c)) return;
    __shared__ c64 r[1];
    sum_partials<1>(part, np, r);
    if (threadIdx.x == 0) {
        if (!end_of_iteration(c, hist, r[0].x)) return;
        double rhon = sc[Q_RHON].x, xin = sc[Q_XIN].x;
        c64 deltan = sc[Q_DELTAN];
        if (!(rhon != 0.0) || !isfinite(rhon) || !(xin != 0.0) || !isfinite(xin) || bad_den(deltan) ||
            bad_den(sc[Q_EPS])) {
            set_breakdown(c);
            return;
        }
        sc[Q_RHO] = {rhon, 0.0};
        sc[Q_XI] = {xin, 0.0};
        sc[Q_DELTA] = deltan;
    }
}

// Gl-QMR: Vt = Pt - b V (in place over V); Wt = Zh - conj(b) W (in place over W);
// part = (||Vt||^2, ||Wt||^2, tr(Wt^H Vt))
template <class T>
__global__ __launch_bounds__(kBlock) void k_glqmr_lanczos(const Ctl* ctl, Flat fl, const c64* sc, T* __restrict__ V,
                                                          T* __restrict__ W, const T* __restrict__ Pt,
                                                          const T* __restrict__ Zh, c64* part) {
    if (stopped(ctl)) return;
    const T mb = down<T>(-sc[Q_BETA]);
    const T mbc = down<T>(-conj_(sc[Q_BETA]));
    c64 acc[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    SKR_FLAT_LOOP(fl) {
        T v = fma_(mb, V[e], Pt[e]);
        T w = fma_(mbc, W[e], Zh[e]);
        V[e] = v;
        W[e] = w;
        nrm_acc(acc[0].x, v);
        nrm_acc(acc[1].x, w);
        dot_acc(acc[2], w, v);
    }
    block_reduce_store<3>(acc, part + (size_t)blockIdx.x * 3);
}

// Gl-QMR fused step: D = eta P + f D; S = eta Pt + f S; X += D; R -= S;
// then the next directions V = Vt/rho, W = Wt/xi, P = V - cP P, Qd = W - cQ Qd.
// With upd = 0 only the direction part runs (initialisation, P = Qd = 0 then).
// part = ||R||^2.
template <class T>
__global__ __launch_bounds__(kBlock) void k_glqmr_step(const Ctl* ctl, Flat fl, const c64* sc, int upd,
                                                       T* __restrict__ X, T* __restrict__ R, T* __restrict__ D,
                                                       T* __restrict__ S, T* __restrict__ P, const T* __restrict__ Pt,
                                                       T* __restrict__ V, T* __restrict__ W, T* __restrict__ Qd,
                                                       c64* part) {
    if (stopped(ctl)) return;
    const T eta = down<T>(sc[Q_ETA]);
    const T f = down<T>(sc[Q_F]);
    const T irho = down<T>(sc[Q_IRHO]);
    const T ixi = down<T>(sc[Q_IXI]);
    const T mcp = down<T>(-sc[Q_CP]);
    const T mcq = down<T>(-sc[Q_CQ]);
    c64 acc[1] = {{0.0, 0.0}};
    SKR_FLAT_LOOP(fl) {
        T p = P[e];
        if (upd) {
            T d = fma_(f, D[e], mul_(eta, p));
            T sv = fma_(f, S[e], mul_(eta, Pt[e]));
            D[e] = d;
            S[e] = sv;
            X[e] = add_(X[e], d);
            T r = sub_(R[e], sv);
            R[e] = r;
            nrm_acc(acc[0].x, r);
        }
        T v = mul_(V[e], irho);
        T w = mul_(W[e], ixi);
        V[e] = v;
        W[e] = w;
        P[e] = fma_(mcp, p, v);
        Qd[e] = fma_(mcq, Qd[e], w);
    }
    if (upd) block_reduce_store<1>(acc, part + (size_t)blockIdx.x);
}

// eGl-QMR: Vt = Pt - b V (block, in place); wt = zh - conj(b) w (vector, in place);
// part = (||Vt||^2, ||wt||^2, sum(wt^H Vt))
template <class T>
__global__ __launch_bounds__(kBlock) void k_eglqmr_lanczos(const Ctl* ctl, Layout ly, int n, int rpc, const c64* sc,
                                                           T* __restrict__ V, T* __restrict__ w,
                                                           const T* __restrict__ Pt, const T* __restrict__ zh,
                                                           c64* part) {
    if (stopped(ctl)) return;
    const T mb = down<T>(-sc[Q_BETA]);
    const T mbc = down<T>(-conj_(sc[Q_BETA]));
    const int s = ly.s;
    c64 acc[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    SKR_ROW_LOOP(ly, n, rpc) {
        const int i = base_ + grp;
        if (i < r1_) {
            const T wi = fma_(mbc, w[i], zh[i]);
            for (int c = lane; c < s; c += ly.L) {
                size_t e = (size_t)i * s + c;
                T v = fma_(mb, V[e], Pt[e]);
                V[e] = v;
                nrm_acc(acc[0].x, v);
                dot_acc(acc[2], wi, v);
            }
            if (lane == 0) {
                w[i] = wi;
                nrm_acc(acc[1].x, wi);
            }
        }
    }
    block_reduce_store<3>(acc, part + (size_t)blockIdx.x * 3);
}

// eGl-QMR fused step (block part as Gl-QMR, shadow vectors w, qd)
template <class T>
__global__ __launch_bounds__(kBlock) void k_eglqmr_step(const Ctl* ctl, Layout ly, int n, int rpc, const c64* sc,
                                                        int upd, T* __restrict__ X, T* __restrict__ R,
                                                        T* __restrict__ D, T* __restrict__ S, T* __restrict__ P,
                                                        const T* __restrict__ Pt, T* __restrict__ V,
                                                        T* __restrict__ w, T* __restrict__ qd, c64* part) {
    if (stopped(ctl)) return;
    const T eta = down<T>(sc[Q_ETA]);
    const T f = down<T>(sc[Q_F]);
    const T irho = down<T>(sc[Q_IRHO]);
    const T ixi = down<T>(sc[Q_IXI]);
    const T mcp = down<T>(-sc[Q_CP]);
    const T mcq = down<T>(-sc[Q_CQ]);
    const int s = ly.s;
    c64 acc[1] = {{0.0, 0.0}};
    SKR_ROW_LOOP(ly, n, rpc) {
        const int i = base_ + grp;
        if (i < r1_) {
            for (int c = lane; c < s; c += ly.L) {
                size_t e = (size_t)i * s + c;
                T p = P[e];
                if (upd) {
                    T d = fma_(f, D[e], mul_(eta, p));
                    T sv = fma_(f, S[e], mul_(eta, Pt[e]));
                    D[e] = d;
                    S[e] = sv;
                    X[e] = add_(X[e], d);
                    T r = sub_(R[e], sv);
                    R[e] = r;
                    nrm_acc(acc[0].x, r);
                }
                T v = mul_(V[e], irho);
                V[e] = v;
                P[e] = fma_(mcp, p, v);
            }
            if (lane == 0) {
                T wi = mul_(w[i], ixi);
                w[i] = wi;
                qd[i] = fma_(mcq, qd[i], wi);
            }
        }
    }
    if (upd) block_reduce_store<1>(acc, part + (size_t)blockIdx.x);
}

// economic init: part = (||Vt||^2, ||wt||^2, sum(wt^H Vt)) with wt a vector
template <class T>
__global__ __launch_bounds__(kBlock) void k_egl_init_red(Layout ly, int n, int rpc, const T* __restrict__ V,
                                                         const T* __restrict__ w, c64* part) {
    const int s = ly.s;
    c64 acc[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    SKR_ROW_LOOP(ly, n, rpc) {
        const int i = base_ + grp;
        if (i < r1_) {
            const T wi = w[i];
            for (int c = lane; c < s; c += ly.L) {
                T v = V[(size_t)i * s + c];
                nrm_acc(acc[0].x, v);
                dot_acc(acc[2], wi, v);
            }
            if (lane == 0) nrm_acc(acc[1].x, wi);
        }
    }
    block_reduce_store<3>(acc, part + (size_t)blockIdx.x * 3);
}

// flat init for Gl-QMR: part = (||V||^2, ||W||^2, tr(W^H V))
template <class T>
__global__ __launch_bounds__(kBlock) void k_gl_init_red3(Flat fl, const T* __restrict__ V, const T* __restrict__ W,
                                                         c64* part) {
    c64 acc[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    SKR_FLAT_LOOP(fl) {
        T v = V[e], w = W[e];
        nrm_acc(acc[0].x, v);
        nrm_acc(acc[1].x, w);
        dot_acc(acc[2], w, v);
    }
    block_reduce_store<3>(acc, part + (size_t)blockIdx.x * 3);
}

// economic init: part = (||R||^2, sum(rh^H R))
template <class T>
__global__ __launch_bounds__(kBlock) void k_egl_init_red2(Layout ly, int n, int rpc, const T* __restrict__ R,
                                                          const T* __restrict__ rh, c64* part) {
    const int s = ly.s;
    c64 acc[2] = {{0.0, 0.0}, {0.0, 0.0}};
    SKR_ROW_LOOP(ly, n, rpc) {
        const int i = base_ + grp;
        if (i < r1_) {
            const T ri = rh[i];
            for (int c = lane; c < s; c += ly.L) {
                T v = R[(size_t)i * s + c];
                nrm_acc(acc[0].x, v);
                dot_acc(acc[1], ri, v);
            }
        }
    }
    block_reduce_store<2>(acc, part + (size_t)blockIdx.x * 2);
}

}  // namespace skr
