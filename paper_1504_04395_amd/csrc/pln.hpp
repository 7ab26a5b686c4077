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

// ------------------------------------------- loop-interchanged BiCGStab
// s independent BiCGStab recurrences (van der Vorst), written as block
// BiCGStab with diagonal coefficient matrices: every per-column scalar sits on
// the diagonal of an s x s slot, so the block update kernels apply it.

// sum over the p2 partial copies (stride `stride`) of entry e of part2
__device__ inline c64 part_entry(const c64* __restrict__ part2, int p2, int stride, int e) {
    c64 acc = part2[e];
    for (int y = 1; y < p2; ++y) acc = acc + part2[(size_t)y * stride + e];
    return acc;
}

// alpha_c = rho_c / sigma_c with rho = diag(R~^H R) (mats M_N) and
// sigma = diag(R~^H V) (part2).  Stores diag(alpha) (M_A) and -diag(alpha) (M_TMP).
__global__ __launch_bounds__(kScalar) void k_lbs_alpha(Ctl* c, int s, const c64* __restrict__ part2, int p2,
                                                       c64* __restrict__ mats) {
    if (stopped(c)) return;
    const int ss = s * s;
    int ok = 1;
    for (int j = threadIdx.x; j < s; j += blockDim.x)
        if (bad_den(part_entry(part2, p2, ss, j * s + j))) ok = 0;
    if (!wave_all(ok)) {
        if (threadIdx.x == 0) set_breakdown(c);
        return;
    }
    for (int e = threadIdx.x; e < ss; e += blockDim.x) {
        const int i = e / s, j = e - i * s;
        const c64 a = i == j ? cdiv(mats[(size_t)M_N * ss + e], part_entry(part2, p2, ss, e)) : c64{0.0, 0.0};
        mats[(size_t)M_A * ss + e] = a;
        mats[(size_t)M_TMP * ss + e] = -a;
    }
}

// omega_c = (t_c^H s_c) / (t_c^H t_c) from the back-to-back Grams (T^H S,
// T^H T) in part2.  Stores diag(omega) (M_W) and -diag(omega) (M_MW).
__global__ __launch_bounds__(kScalar) void k_lbs_omega(Ctl* c, int s, const c64* __restrict__ part2, int p2,
                                                       c64* __restrict__ mats) {
    if (stopped(c)) return;
    const int ss = s * s;
    int ok = 1;
    for (int j = threadIdx.x; j < s; j += blockDim.x)
        if (bad_den(part_entry(part2, p2, 2 * ss, ss + j * s + j))) ok = 0;
    if (!wave_all(ok)) {
        if (threadIdx.x == 0) set_breakdown(c);
        return;
    }
    for (int e = threadIdx.x; e < ss; e += blockDim.x) {
        const int i = e / s, j = e - i * s;
        const c64 w = i == j ? cdiv(part_entry(part2, p2, 2 * ss, e), part_entry(part2, p2, 2 * ss, ss + e))
                             : c64{0.0, 0.0};
        mats[(size_t)M_W * ss + e] = w;
        mats[(size_t)M_MW * ss + e] = -w;
    }
}

// After the updates: ||R||_F^2 = tr(R^H R) (mats M_RR) drives the stopping
// rule; then beta_c = (rho'_c / rho_c)(alpha_c / omega_c) with rho' =
// diag(R~^H R) (part2).  Stores diag(beta) (M_B) and rho' (M_N).
__global__ __launch_bounds__(kScalar) void k_lbs_beta(Ctl* c, double* hist, int s, const c64* __restrict__ part2,
                                                      int p2, c64* __restrict__ mats) {
    if (stopped(c)) return;
    __shared__ int flag;
    const int ss = s * s;
    double t = 0.0;
    for (int i = threadIdx.x; i < s; i += blockDim.x) t += mats[(size_t)M_RR * ss + i * s + i].x;
    const double res2 = wave_sum(t);
    if (threadIdx.x == 0) flag = end_of_iteration(c, hist, res2) ? 1 : 0;
    __syncthreads();
    if (!flag) return;
    int ok = 1;
    for (int j = threadIdx.x; j < s; j += blockDim.x) {
        const int d = j * s + j;
        if (bad_den(mats[(size_t)M_N * ss + d]) || bad_den(mats[(size_t)M_W * ss + d])) ok = 0;
    }
    if (!wave_all(ok)) {
        if (threadIdx.x == 0) set_breakdown(c);
        return;
    }
    for (int e = threadIdx.x; e < ss; e += blockDim.x) {
        const int i = e / s, j = e - i * s;
        const c64 rn = part_entry(part2, p2, ss, e);
        c64 b = {0.0, 0.0};
        if (i == j)
            b = cdiv(rn, mats[(size_t)M_N * ss + e]) * cdiv(mats[(size_t)M_A * ss + e], mats[(size_t)M_W * ss + e]);
        mats[(size_t)M_B * ss + e] = b;
        mats[(size_t)M_N * ss + e] = rn;
    }
}

// ------------------------------------------------- loop-interchanged QMR
// s independent QMR recurrences (the coupled two-term QMR of the global
// variant, one set of scalars per column).  Per-column scalar x_c lives at
// the diagonal entry (c, c) of its slot; slots applied to blocks are written
// whole, zero off the diagonal.

__device__ inline c64 dg(const c64* __restrict__ mats, int slot, int s, int c) {
    return mats[(size_t)slot * s * s + (size_t)c * s + c];
}
// writes diag(v(c)) into slot for the whole s x s matrix
template <class F>
__device__ inline void put_diag(c64* __restrict__ mats, int slot, int s, F v) {
    const int ss = s * s;
    for (int e = threadIdx.x; e < ss; e += blockDim.x) {
        const int i = e / s, j = e - i * s;
        mats[(size_t)slot * ss + e] = i == j ? v(j) : c64{0.0, 0.0};
    }
}
__device__ inline bool bad_pos(double v) { return !(v != 0.0) || !isfinite(v); }

// Start: rho_c = ||vt_c||, xi_c = ||wt_c||, delta_c = wt_c^H vt_c / (rho_c xi_c)
// from the Grams in M_QVV, M_QWW, M_QWV; gamma = 1, eta = -1, theta = 0;
// the direction coefficients are zero (P = Qd = 0 before the first step);
// also the identity slots.
__global__ __launch_bounds__(kScalar) void k_lqmr_s0(Ctl* c, int s, c64* __restrict__ mats) {
    if (stopped(c)) return;
    int ok = 1;
    for (int j = threadIdx.x; j < s; j += blockDim.x) {
        const double rho = sqrt(dg(mats, M_QVV, s, j).x), xi = sqrt(dg(mats, M_QWW, s, j).x);
        if (bad_pos(rho) || bad_pos(xi) || bad_den(cdiv(dg(mats, M_QWV, s, j), c64{rho * xi, 0.0}))) ok = 0;
    }
    if (!wave_all(ok)) {
        if (threadIdx.x == 0) set_breakdown(c);
        return;
    }
    const c64 one = {1.0, 0.0}, zero = {0.0, 0.0};
    put_diag(mats, M_QRHO, s, [&](int j) { return c64{sqrt(dg(mats, M_QVV, s, j).x), 0.0}; });
    put_diag(mats, M_QXI, s, [&](int j) { return c64{sqrt(dg(mats, M_QWW, s, j).x), 0.0}; });
    __syncthreads();
    put_diag(mats, M_QDELTA, s, [&](int j) {
        return cdiv(dg(mats, M_QWV, s, j), c64{dg(mats, M_QRHO, s, j).x * dg(mats, M_QXI, s, j).x, 0.0});
    });
    put_diag(mats, M_QIRHO, s, [&](int j) { return c64{1.0 / dg(mats, M_QRHO, s, j).x, 0.0}; });
    put_diag(mats, M_QIXI, s, [&](int j) { return c64{1.0 / dg(mats, M_QXI, s, j).x, 0.0}; });
    put_diag(mats, M_QGAMMA, s, [&](int) { return one; });
    put_diag(mats, M_QETA, s, [&](int) { return c64{-1.0, 0.0}; });
    put_diag(mats, M_QTHETA, s, [&](int) { return zero; });
    put_diag(mats, M_QMCP, s, [&](int) { return zero; });
    put_diag(mats, M_QMCQ, s, [&](int) { return zero; });
    put_diag(mats, M_ID, s, [&](int) { return one; });
    put_diag(mats, M_MID, s, [&](int) { return c64{-1.0, 0.0}; });
}

// eps_c = qd_c^H pt_c (part2) -> beta_c = eps_c / delta_c; stores eps, beta,
// diag(-beta) (M_QMB) and diag(-conj beta) (M_QMBC).
__global__ __launch_bounds__(kScalar) void k_lqmr_s1(Ctl* c, int s, const c64* __restrict__ part2, int p2,
                                                     c64* __restrict__ mats) {
    if (stopped(c)) return;
    const int ss = s * s;
    int ok = 1;
    for (int j = threadIdx.x; j < s; j += blockDim.x)
        if (bad_den(part_entry(part2, p2, ss, j * s + j))) ok = 0;
    if (!wave_all(ok)) {
        if (threadIdx.x == 0) set_breakdown(c);
        return;
    }
    put_diag(mats, M_QEPS, s, [&](int j) { return part_entry(part2, p2, ss, j * s + j); });
    put_diag(mats, M_QBETA, s, [&](int j) { return cdiv(part_entry(part2, p2, ss, j * s + j), dg(mats, M_QDELTA, s, j)); });
    __syncthreads();
    put_diag(mats, M_QMB, s, [&](int j) { return -dg(mats, M_QBETA, s, j); });
    put_diag(mats, M_QMBC, s, [&](int j) { return -conj_(dg(mats, M_QBETA, s, j)); });
}

// From ||vt_c||^2, ||wt_c||^2, wt_c^H vt_c (M_QVV, M_QWW, M_QWV): theta, gamma,
// eta and the D/S weight f (diag slots M_QETA, M_QF), then the next step's
// normalisations and direction coefficients c_P = xi' delta' / eps,
// c_Q = conj(rho' delta' / eps) as diag(-c_P), diag(-c_Q).
__global__ __launch_bounds__(kScalar) void k_lqmr_s2(Ctl* c, int s, c64* __restrict__ mats) {
    if (stopped(c)) return;
    int ok = 1;
    for (int j = threadIdx.x; j < s; j += blockDim.x) {
        const double gp = dg(mats, M_QGAMMA, s, j).x;
        const c64 beta = dg(mats, M_QBETA, s, j);
        if (bad_den(beta) || bad_pos(gp)) ok = 0;
        else {
            const double theta = sqrt(dg(mats, M_QVV, s, j).x) / (gp * cabs(beta));
            const double gamma = 1.0 / sqrt(1.0 + theta * theta);
            if (bad_pos(gamma)) ok = 0;
        }
    }
    if (!wave_all(ok)) {
        if (threadIdx.x == 0) set_breakdown(c);
        return;
    }
    // eta and f need the previous gamma, eta and theta: computed before those are replaced
    put_diag(mats, M_QRHON, s, [&](int j) { return c64{sqrt(dg(mats, M_QVV, s, j).x), 0.0}; });
    put_diag(mats, M_QXIN, s, [&](int j) { return c64{sqrt(dg(mats, M_QWW, s, j).x), 0.0}; });
    __syncthreads();
    put_diag(mats, M_QF, s, [&](int j) {   // f = (theta_prev gamma)^2; scratch use of the slot below
        const double gp = dg(mats, M_QGAMMA, s, j).x;
        const double theta = dg(mats, M_QRHON, s, j).x / (gp * cabs(dg(mats, M_QBETA, s, j)));
        const double gamma = 1.0 / sqrt(1.0 + theta * theta);
        const double tg = dg(mats, M_QTHETA, s, j).x * gamma;
        return c64{tg * tg, 0.0};
    });
    put_diag(mats, M_QDELTAN, s, [&](int j) {
        return cdiv(dg(mats, M_QWV, s, j), c64{dg(mats, M_QRHON, s, j).x * dg(mats, M_QXIN, s, j).x, 0.0});
    });
    __syncthreads();
    // eta = -eta_prev rho gamma^2 / (beta gamma_prev^2), written over eta_prev
    // column by column by the thread that read it
    for (int e = threadIdx.x; e < s * s; e += blockDim.x) {
        const int i = e / s, j = e - i * s;
        if (i != j) continue;
        const double gp = dg(mats, M_QGAMMA, s, j).x;
        const c64 beta = dg(mats, M_QBETA, s, j);
        const double theta = dg(mats, M_QRHON, s, j).x / (gp * cabs(beta));
        const double gamma = 1.0 / sqrt(1.0 + theta * theta);
        const double rho = dg(mats, M_QRHO, s, j).x;
        const c64 eta = cdiv(-(rho * gamma * gamma) * dg(mats, M_QETA, s, j), (gp * gp) * beta);
        mats[(size_t)M_QETA * s * s + e] = eta;
        mats[(size_t)M_QGAMMA * s * s + e] = c64{gamma, 0.0};
        mats[(size_t)M_QTHETA * s * s + e] = c64{theta, 0.0};
    }
    put_diag(mats, M_QIRHO, s, [&](int j) { return c64{1.0 / dg(mats, M_QRHON, s, j).x, 0.0}; });
    put_diag(mats, M_QIXI, s, [&](int j) { return c64{1.0 / dg(mats, M_QXIN, s, j).x, 0.0}; });
    put_diag(mats, M_QMCP, s, [&](int j) {
        return -cdiv(dg(mats, M_QXIN, s, j).x * dg(mats, M_QDELTAN, s, j), dg(mats, M_QEPS, s, j));
    });
    put_diag(mats, M_QMCQ, s, [&](int j) {
        return -conj_(cdiv(dg(mats, M_QRHON, s, j).x * dg(mats, M_QDELTAN, s, j), dg(mats, M_QEPS, s, j)));
    });
}

// ||R||_F^2 = tr(R^H R) (M_RR) -> stopping test; then the next step's
// breakdown tests (rho', xi' nonzero and finite, delta' and eps usable) and
// rho, xi, delta <- rho', xi', delta'.
__global__ __launch_bounds__(kScalar) void k_lqmr_s3(Ctl* c, double* hist, int s, c64* __restrict__ mats) {
    if (stopped(c)) return;
    __shared__ int flag;
    double t = 0.0;
    for (int i = threadIdx.x; i < s; i += blockDim.x) t += dg(mats, M_RR, s, i).x;
    const double res2 = wave_sum(t);
    if (threadIdx.x == 0) flag = end_of_iteration(c, hist, res2) ? 1 : 0;
    __syncthreads();
    if (!flag) return;
    int ok = 1;
    for (int j = threadIdx.x; j < s; j += blockDim.x)
        if (bad_pos(dg(mats, M_QRHON, s, j).x) || bad_pos(dg(mats, M_QXIN, s, j).x) ||
            bad_den(dg(mats, M_QDELTAN, s, j)) || bad_den(dg(mats, M_QEPS, s, j)))
            ok = 0;
    if (!wave_all(ok)) {
        if (threadIdx.x == 0) set_breakdown(c);
        return;
    }
    for (int e = threadIdx.x; e < s * s; e += blockDim.x) {
        const size_t ss = (size_t)s * s;
        mats[M_QRHO * ss + e] = mats[M_QRHON * ss + e];
        mats[M_QXI * ss + e] = mats[M_QXIN * ss + e];
        mats[M_QDELTA * ss + e] = mats[M_QDELTAN * ss + e];
    }
}

}  // namespace skr
