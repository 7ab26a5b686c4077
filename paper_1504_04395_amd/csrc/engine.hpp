// Host-side schedules of the simultaneous Krylov methods.
//
// One iteration of every method is a fixed sequence of kernel launches on one
// stream: sparse products (with fused reductions), stage-2 reductions, one
// one-workgroup coefficient kernel per global reduction, and block updates.
// The host enqueues `m` iterations at a time (optionally as one captured
// hipGraph replayed each time) and then reads the 64-byte control block; that
// read is the only device-to-host transfer inside the iteration.  Kernels
// return at entry once the control block says the iteration stopped, so the
// reported iteration count is exact.
#pragma once

#include <functional>
#include <string>
#include <vector>

#include "blk.hpp"
#include "cblk.hpp"
#include "common.hpp"
#include "glk.hpp"
#include "ilu.hpp"
#include "pln.hpp"
#include "spmm.hpp"

namespace skr {



struct HipError {
    hipError_t e;
    const char* what;
};
#define SKR_HIP(x)                                   \
    do {                                             \
        hipError_t e_ = (x);                         \
        if (e_ != hipSuccess) throw HipError{e_, #x}; \
    } while (0)
#define SKR_LAUNCHED() SKR_HIP(hipGetLastError())

struct Unsupported {
    std::string what;
};

// Arena of device memory carved per solve (grow-only, owned by the context).
struct Arena {
    char* base = nullptr;
    size_t cap = 0;
    size_t off = 0;
    void* take(size_t bytes) {
        size_t a = (off + 255) & ~size_t(255);
        off = a + ((bytes + 255) & ~size_t(255));
        return base ? base + a : nullptr;
    }
};

// A sparse operand (A or A^H) in one storage precision and format.
template <class T>
struct Operand {
    bool sell = false;
    CsrOp<T> csr{};
    SellOp<T> sl{};
};

template <class T>
struct Env {
    hipStream_t st{};
    int n = 0, s = 0;
    int nb = 0;              // workgroups per streaming kernel (multiple of 8)
    int rpc = 0;             // rows per workgroup chunk
    int p2 = 1;              // partials left after the second reduction stage
    Flat fl{};               // n*s elements
    Layout ly{};             // row layout of the global family (L = min(2^ceil(log2 s), 16))
    Layout lyv{};            // vector layout (s = 1, L = 1)
    Tile16 tl{};             // tile-16 layout of the block family
    Ctl* ctl = nullptr;
    double* hist = nullptr;
    c64* part = nullptr;
    c64* part2 = nullptr;
    c64* sc = nullptr;
    c64* mats = nullptr;
    Operand<T> A, AH;
    int J = 1;               // ceil(s/16)
    // right preconditioning M = L U: while pc_on, products with A become
    // A M^-1 and products with A^H become M^-H A^H (pc_tmp: one n x s block)
    const Ilu* pc = nullptr;
    bool pc_on = false;
    T* pc_tmp = nullptr;
    size_t blk_bytes() const { return (size_t)n * s * sizeof(T); }
};

template <class T>
constexpr bool kFp64 = std::is_same<T, double>::value || std::is_same<T, c64>::value;

// Y = M^-1 Z (adj: M^-H Z) with M = L U; Y may equal Z.
template <class T>
void prec_apply(Env<T>& e, int s, const T* Z, T* Y, bool adj, const Ctl* ctl) {
    if constexpr (kFp64<T>) {
        const Ilu& p = *e.pc;
        if (!adj) {
            tri_solve<T>(e.st, p.L, s, Z, Y, ctl);
            tri_solve<T>(e.st, p.U, s, Y, Y, ctl);
        } else {
            tri_solve<T>(e.st, p.UH, s, Z, Y, ctl);
            tri_solve<T>(e.st, p.LH, s, Y, Y, ctl);
        }
        SKR_LAUNCHED();
    } else {
        throw Unsupported{"preconditioning needs FP64 data"};
    }
}

inline int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

template <class T>
void env_layout(Env<T>& e, int n, int s) {
    e.n = n;
    e.s = s;
    int L = 1 << ilog2(s);
    if (L > 16) L = 16;
    e.ly = Layout{s, L, ilog2(L)};
    e.lyv = Layout{1, 1, 0};
    int nb = (n + 63) / 64;
    nb = ((nb + 7) / 8) * 8;
    if (nb > 2048) nb = 2048;
    if (nb < 8) nb = 8;
    e.nb = nb;
    e.rpc = (n + nb - 1) / nb;
    e.rpc = ((e.rpc + 15) / 16) * 16;
    e.fl.total = (size_t)n * s;
    size_t per = (e.fl.total + nb - 1) / nb;
    e.fl.per = ((per + kBlock - 1) / kBlock) * kBlock;
    e.tl = Tile16{n, s, e.rpc};
    e.J = (s + 15) / 16;
}

// ------------------------------------------------------------------ launch helpers
template <class T, int J, class Epi, int J16 = (J == 1 ? 1 : 2)>
void spmm_j(Env<T>& e, const Operand<T>& op, const Layout& ly, const T* X, T* Y, Epi epi, const Ctl* ctl) {
    if (e.pc_on) {
        e.pc_on = false;
        if (&op == &e.A) {                                   // Y = A (M^-1 X), epilogue on Y
            prec_apply(e, ly.s, X, e.pc_tmp, false, ctl);
            spmm_j<T, J, Epi, J16>(e, op, ly, e.pc_tmp, Y, epi, ctl);
        } else {                                             // Y = M^-H (A^H X), epilogue after
            spmm_j<T, J, EpiNone, J16>(e, op, ly, X, e.pc_tmp, EpiNone{}, ctl);
            prec_apply(e, ly.s, e.pc_tmp, Y, true, ctl);
            if constexpr (std::is_same<Epi, EpiGram<T, J>>::value) {
                k_bl_gram<T, J><<<e.nb, kBlock, 0, e.st>>>(ctl, e.tl, epi.Z, Y, epi.part);   // Z^H Y
                SKR_LAUNCHED();
            } else if constexpr (!std::is_same<Epi, EpiNone>::value) {
                throw Unsupported{"epilogue not available on the preconditioned adjoint product"};
            }
        }
        e.pc_on = true;
        return;
    }
    // s > 16 Gram epilogues as separate streaming passes over Y and Z: fused,
    // the s x s accumulators would cut the gather loop's occupancy to 1-2 waves
    // per SIMD
    auto gram_after = [&](auto& ep) {
        const int ss = ly.s * ly.s;
        if constexpr (std::is_same<std::decay_t<decltype(ep)>, EpiGram<T, 2>>::value) {
            k_bl_gram<T, 2><<<e.nb, kBlock, 0, e.st>>>(ctl, e.tl, ep.Z, Y, ep.part);   // Z^H Y
        } else {
            k_bl_gram<T, 2><<<e.nb, kBlock, 0, e.st>>>(ctl, e.tl, Y, ep.Z, ep.part, 2 * ss, 0);   // Y^H Z
            SKR_LAUNCHED();
            k_bl_gram<T, 2><<<e.nb, kBlock, 0, e.st>>>(ctl, e.tl, Y, Y, ep.part, 2 * ss, ss);      // Y^H Y
        }
    };
    if (op.sell) {
        // 16 lanes per row, J16 = ceil(s / 16) columns per lane, one pass of 16
        // sorted positions of a chunk per workgroup step
        const int nchunks = (e.n + op.sl.C - 1) / op.sl.C;
        const int cpb = (nchunks + e.nb - 1) / e.nb;
        const Layout l16{ly.s, 16, 4};
        if constexpr (J16 == 2 && EpiIsGram<Epi>::value && J == 2) {
            k_spmm_sell16<T, 2, EpiNone><<<e.nb, kBlock, 0, e.st>>>(ctl, op.sl, l16, cpb, X, Y, EpiNone{});
            SKR_LAUNCHED();
            gram_after(epi);
        } else if constexpr (!EpiIsGram<Epi>::value || J == J16) {
            k_spmm_sell16<T, J16, Epi><<<e.nb, kBlock, 0, e.st>>>(ctl, op.sl, l16, cpb, X, Y, epi);
        } else {
            throw Unsupported{"Gram epilogue with a layout other than 16 lanes per row"};
        }
    } else if (!Tr<T>::cplx && J16 == 1 && ly.s % 2 == 0) {
        if constexpr (!Tr<T>::cplx && J16 == 1) {
            // real, even s <= 16: 8 lanes per row, two columns per lane
            const int per_xcd = ((e.n + 7) / 8 + 63) / 64 * 64;
            k_spmm_csr8<T, Epi><<<e.nb, kBlock, 0, e.st>>>(ctl, op.csr, ly, per_xcd, X, Y, epi);
        }
    } else {
        // CSR kernel: 16 lanes per row whatever s is (its lane layout is the DPP row)
        const Layout l16{ly.s, 16, 4};
        const int step = 32;                           // RP * 16 rows per workgroup pass (upper bound)
        const int per_xcd = ((e.n + 7) / 8 + step - 1) / step * step;
        if constexpr (J16 == 2 && EpiIsGram<Epi>::value && J == 2) {
            k_spmm_csr<T, 2, EpiNone><<<e.nb, kBlock, 0, e.st>>>(ctl, op.csr, l16, per_xcd, X, Y, EpiNone{});
            SKR_LAUNCHED();
            gram_after(epi);
        } else {
            k_spmm_csr<T, J16, Epi><<<e.nb, kBlock, 0, e.st>>>(ctl, op.csr, l16, per_xcd, X, Y, epi);
        }
    }
    SKR_LAUNCHED();
}
template <class T, class Epi>
void spmm(Env<T>& e, const Operand<T>& op, const Layout& ly, const T* X, T* Y, Epi epi, const Ctl* ctl) {
    if (e.pc_on) {
        e.pc_on = false;
        if (&op == &e.A) {                                   // Y = A (M^-1 X), epilogue on Y
            prec_apply(e, ly.s, X, e.pc_tmp, false, ctl);
            spmm(e, op, ly, e.pc_tmp, Y, epi, ctl);
        } else {                                             // Y = M^-H (A^H X)
            if constexpr (!std::is_same<Epi, EpiNone>::value)
                throw Unsupported{"epilogue not available on the preconditioned adjoint product"};
            spmm(e, op, ly, X, e.pc_tmp, EpiNone{}, ctl);
            prec_apply(e, ly.s, e.pc_tmp, Y, true, ctl);
        }
        e.pc_on = true;
        return;
    }
    if constexpr (std::is_same<Epi, EpiNone>::value) {
        if (ly.s == 1 && !op.sell) {   // single vector: 8 lanes per row
            const int per_xcd = ((e.n + 7) / 8 + 31) / 32 * 32;
            k_spmv_csr<T><<<e.nb, kBlock, 0, e.st>>>(ctl, op.csr, per_xcd, X, Y);
            SKR_LAUNCHED();
            return;
        }
    }
    // J of the SELL kernel follows ly; the CSR kernel always uses 16 lanes, J16 = ceil(s/16)
    const int J = (ly.s + ly.L - 1) / ly.L;
    const bool j16 = ly.s > 16;
    if (J == 1 && !j16) spmm_j<T, 1, Epi, 1>(e, op, ly, X, Y, epi, ctl);
    else if (J == 1) spmm_j<T, 1, Epi, 2>(e, op, ly, X, Y, epi, ctl);
    else if (!j16) spmm_j<T, 2, Epi, 1>(e, op, ly, X, Y, epi, ctl);
    else spmm_j<T, 2, Epi, 2>(e, op, ly, X, Y, epi, ctl);
}
template <class T>
Layout tile_layout(const Env<T>& e) { return Layout{e.s, 16, 4}; }

template <class T>
void reduce2(Env<T>& e, int E, int cond_slot = -1) {
    k_reduce_parts<<<(E + kWaves - 1) / kWaves, kBlock, 0, e.st>>>(e.ctl, cond_slot, e.part, e.nb, E, e.part2);
    SKR_LAUNCHED();
}

// Dynamic LDS of a tile kernel: nmat s x s matrices and ntile row tiles of
// RowPasses * 16 rows, in complex FP64 slots (real kernels use half), and at
// least the Gram reduction buffer.
inline size_t mat_lds(int s, int nmat, int ntile) {
    size_t J = (s + 15) / 16;
    size_t rp = s <= 16 ? 2 : 1;   // RowPasses tiles measured in complex FP64 slots
    size_t need = (size_t)nmat * s * s + (size_t)ntile * rp * 16 * s;
    size_t gram = (16 * J) * (16 * J);
    return (need > gram ? need : gram) * sizeof(c64);
}

// One CholeskyQR triangular pass (k_bl_tri arguments); real s <= 16 blocks use
// the MFMA tile kernel.
template <class T, int J>
void tri_pass(Env<T>& e, int slot, int cond, int nchain, int add_shift, int mode, const T* Z, T* Out,
              const T* Other) {
    if constexpr (!Tr<T>::cplx && J == 1) {
        const bool oth = (mode & (TRI_G_OTHER_OUT | TRI_G_OUT_OTHER)) != 0;
        if (nchain + add_shift <= 1 && !oth)
            k_bl_tri16<T, 1, false><<<e.nb, kBlock, 0, e.st>>>(e.ctl, slot, cond, nchain, add_shift, e.tl, mode,
                                                              e.mats, Z, Out, Other, e.part);
        else if (!oth)
            k_bl_tri16<T, 3, false><<<e.nb, kBlock, 0, e.st>>>(e.ctl, slot, cond, nchain, add_shift, e.tl, mode,
                                                              e.mats, Z, Out, Other, e.part);
        else
            k_bl_tri16<T, 3, true><<<e.nb, kBlock, 0, e.st>>>(e.ctl, slot, cond, nchain, add_shift, e.tl, mode,
                                                             e.mats, Z, Out, Other, e.part);
    } else {   // complex, or real with s > 16
        const bool oth = (mode & (TRI_G_OTHER_OUT | TRI_G_OUT_OTHER)) != 0;
        if (nchain + add_shift <= 1 && !oth)
            k_bl_tric<T, J, 1, false><<<e.nb, kBlock, 0, e.st>>>(e.ctl, slot, cond, nchain, add_shift, e.tl, mode,
                                                                 e.mats, Z, Out, Other, e.part);
        else if (!oth)
            k_bl_tric<T, J, 3, false><<<e.nb, kBlock, 0, e.st>>>(e.ctl, slot, cond, nchain, add_shift, e.tl, mode,
                                                                 e.mats, Z, Out, Other, e.part);
        else
            k_bl_tric<T, J, 3, true><<<e.nb, kBlock, 0, e.st>>>(e.ctl, slot, cond, nchain, add_shift, e.tl, mode,
                                                                e.mats, Z, Out, Other, e.part);
    }
    SKR_LAUNCHED();
}

// CholeskyQR2 (+ shifted first pass) of Z into Q; the Gram Z^H Z partials must
// already be in e.part.  R factor in mats (slot 0: M_S, slot 1: M_T).
// mode/Other: Gram fused into the final pass (TRI_* flags).
template <class T, int J>
void cholqr(Env<T>& e, int slot, const T* Z, T* Q, int mode, const T* Other) {
    const int s = e.s, ss = s * s;
    const double u = sizeof(typename Tr<T>::R) == 4 ? 0x1p-24 : 0x1p-53;   // stored precision
    size_t lds4 = 4 * (size_t)ss * sizeof(c64);
    reduce2(e, ss);
    k_qr_chol<<<1, kCoefThreads, lds4, e.st>>>(e.ctl, slot, 1, e.n, s, e.part2, e.p2, e.mats, u);
    SKR_LAUNCHED();
    // Gram of Q1 = Z S1^{-1}
    tri_pass<T, J>(e, slot, 0, 1, 0, TRI_G_OUT_OUT, Z, nullptr, nullptr);
    reduce2(e, ss);
    k_qr_chol<<<1, kCoefThreads, lds4, e.st>>>(e.ctl, slot, 2, e.n, s, e.part2, e.p2, e.mats, u);
    SKR_LAUNCHED();
    // shifted case only: Gram of Q2 = Z S1^{-1} S2^{-1}
    tri_pass<T, J>(e, slot, 1, 2, 0, TRI_G_OUT_OUT, Z, nullptr, nullptr);
    reduce2(e, ss, slot);
    k_qr_chol<<<1, kCoefThreads, lds4, e.st>>>(e.ctl, slot, 3, e.n, s, e.part2, e.p2, e.mats, u);
    SKR_LAUNCHED();
    // Q = Z S1^{-1} S2^{-1} [S3^{-1}]
    tri_pass<T, J>(e, slot, 0, 2, 1, mode | TRI_WRITE, Z, Q, Other);
}

// Block update launchers: real s <= 16 blocks use the MFMA tile kernels.
template <class T, int J, bool GRAM>
void axpm(Env<T>& e, int mslot, int gslot, const T* A, const T* B, const T* C, T* Out) {
    if constexpr (!Tr<T>::cplx && J == 1) {
        k_bl_axpm16<T, GRAM><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.tl, e.mats, mslot, e.sc, gslot, A, B, C, Out,
                                                        e.part);
    } else {   // complex, or real with s > 16
        k_bl_axpmc<T, J, GRAM><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.tl, e.mats, mslot, e.sc, gslot, A, B, C, Out,
                                                          e.part);
    }
    SKR_LAUNCHED();
}
template <class T, int J>
void blrq_updz(Env<T>& e, T* X, const T* V, const T* Q, const T* W, T* Z) {
    if constexpr (!Tr<T>::cplx && J == 1) {
        k_blrq_updz16<T><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.tl, e.mats, X, V, Q, W, Z, e.part);
    } else {   // complex, or real with s > 16
        k_blrq_updzc<T, J><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.tl, e.mats, X, V, Q, W, Z, e.part);
    }
    SKR_LAUNCHED();
}
template <class T, int J>
void blst_upd(Env<T>& e, T* X, const T* U, const T* St, const T* Tt, T* Z) {
    if constexpr (!Tr<T>::cplx && J == 1) {
        k_blst_upd16<T><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.tl, e.mats, e.sc, X, U, St, Tt, Z, e.part);
    } else {   // complex, or real with s > 16
        k_blst_updc<T, J><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.tl, e.mats, e.sc, X, U, St, Tt, Z, e.part);
    }
    SKR_LAUNCHED();
}

// ------------------------------------------------------------------ methods
// Each method: `init` enqueues the set-up for the system A D = R0 (R0 in `rhs`,
// result D in `x`), `iter` enqueues one iteration.  Matrix-vector products per
// iteration are reported by `mv_per_iter`.
template <class T>
struct Method {
    std::function<void()> init;
    std::function<void()> iter;
    long long mv_per_iter = 0;
};

template <class T>
Method<T> make_gl_bicg(Env<T>& e, Arena& ar, T* rhs, T* x) {
    Method<T> m;
    T* R = (T*)ar.take(e.blk_bytes());
    T* Rh = (T*)ar.take(e.blk_bytes());
    T* P = (T*)ar.take(e.blk_bytes());
    T* Ph = (T*)ar.take(e.blk_bytes());
    T* Q = (T*)ar.take(e.blk_bytes());
    T* Zh = (T*)ar.take(e.blk_bytes());
    m.mv_per_iter = 2LL * e.s;
    m.init = [=, &e]() {
        k_copy<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, rhs, R, Rh, P);
        k_copy<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, rhs, Ph, nullptr, nullptr);
        k_fill0<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, x, nullptr, nullptr, nullptr);
        k_flat_nrm_dot<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, R, Rh, e.part);
        k_s_rho0<<<1, kScalar, 0, e.st>>>(e.part, e.nb, 1, 2, e.sc);
        k_init_ctl2<<<1, kScalar, 0, e.st>>>(e.ctl, e.hist, e.part, e.nb);
        SKR_LAUNCHED();
    };
    m.iter = [=, &e]() {
        spmm(e, e.A, e.ly, P, Q, EpiTrace<T>{Ph, e.part}, e.ctl);
        spmm(e, e.AH, e.ly, Ph, Zh, EpiNone{}, e.ctl);
        k_s_alpha<<<1, kScalar, 0, e.st>>>(e.ctl, e.part, e.nb, e.sc);
        k_glbicg_upd<T><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.fl, e.sc, x, R, Rh, P, Q, Zh, e.part);
        k_s_beta<<<1, kScalar, 0, e.st>>>(e.ctl, e.hist, e.part, e.nb, e.sc);
        k_glbicg_dir<T><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.fl, e.sc, R, Rh, P, Ph);
        SKR_LAUNCHED();
    };
    return m;
}

template <class T>
Method<T> make_egl_bicg(Env<T>& e, Arena& ar, T* rhs, T* x) {
    Method<T> m;
    T* R = (T*)ar.take(e.blk_bytes());
    T* P = (T*)ar.take(e.blk_bytes());
    T* Q = (T*)ar.take(e.blk_bytes());
    T* rh = (T*)ar.take((size_t)e.n * sizeof(T));
    T* ph = (T*)ar.take((size_t)e.n * sizeof(T));
    T* zh = (T*)ar.take((size_t)e.n * sizeof(T));
    m.mv_per_iter = e.s + 1;
    m.init = [=, &e]() {
        k_copy<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, rhs, R, P, nullptr);
        k_fill0<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, x, nullptr, nullptr, nullptr);
        k_row_mean<T><<<(e.n + kBlock - 1) / kBlock, kBlock, 0, e.st>>>(e.n, e.s, rhs, rh);
        Flat fv{(size_t)e.n, (((size_t)e.n + e.nb - 1) / e.nb + kBlock - 1) / kBlock * kBlock};
        k_copy<T><<<e.nb, kBlock, 0, e.st>>>(fv, rh, ph, nullptr, nullptr);
        k_egl_init_red2<T><<<e.nb, kBlock, 0, e.st>>>(e.ly, e.n, e.rpc, R, rh, e.part);
        k_s_rho0<<<1, kScalar, 0, e.st>>>(e.part, e.nb, 1, 2, e.sc);
        k_init_ctl2<<<1, kScalar, 0, e.st>>>(e.ctl, e.hist, e.part, e.nb);
        SKR_LAUNCHED();
    };
    m.iter = [=, &e]() {
        spmm(e, e.A, e.ly, P, Q, EpiVecSum<T>{ph, e.part}, e.ctl);
        spmm(e, e.AH, e.lyv, ph, zh, EpiNone{}, e.ctl);
        k_s_alpha<<<1, kScalar, 0, e.st>>>(e.ctl, e.part, e.nb, e.sc);
        k_eglbicg_upd<T><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.ly, e.n, e.rpc, e.sc, x, R, rh, P, Q, zh, e.part);
        k_s_beta<<<1, kScalar, 0, e.st>>>(e.ctl, e.hist, e.part, e.nb, e.sc);
        k_eglbicg_dir<T><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.ly, e.n, e.rpc, e.sc, R, rh, P, ph);
        SKR_LAUNCHED();
    };
    return m;
}

template <class T>
Method<T> make_gl_qmr(Env<T>& e, Arena& ar, T* rhs, T* x) {
    Method<T> m;
    T* R = (T*)ar.take(e.blk_bytes());
    T* V = (T*)ar.take(e.blk_bytes());
    T* W = (T*)ar.take(e.blk_bytes());
    T* P = (T*)ar.take(e.blk_bytes());
    T* Qd = (T*)ar.take(e.blk_bytes());
    T* Pt = (T*)ar.take(e.blk_bytes());
    T* Zh = (T*)ar.take(e.blk_bytes());
    T* D = (T*)ar.take(e.blk_bytes());
    T* S = (T*)ar.take(e.blk_bytes());
    m.mv_per_iter = 2LL * e.s;
    m.init = [=, &e]() {
        k_copy<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, rhs, R, V, W);
        k_fill0<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, x, D, S, P);
        k_fill0<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, Qd, nullptr, nullptr, nullptr);
        k_flat_nrm_dot<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, R, nullptr, e.part);
        k_init_ctl2<<<1, kScalar, 0, e.st>>>(e.ctl, e.hist, e.part, e.nb);
        k_gl_init_red3<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, V, W, e.part);
        k_qmr_s0<<<1, kScalar, 0, e.st>>>(e.ctl, e.part, e.nb, e.sc, 1.0);
        k_glqmr_step<T><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.fl, e.sc, 0, x, R, D, S, P, Pt, V, W, Qd, e.part);
        SKR_LAUNCHED();
    };
    m.iter = [=, &e]() {
        spmm(e, e.A, e.ly, P, Pt, EpiTrace<T>{Qd, e.part}, e.ctl);
        spmm(e, e.AH, e.ly, Qd, Zh, EpiNone{}, e.ctl);
        k_qmr_s1<<<1, kScalar, 0, e.st>>>(e.ctl, e.part, e.nb, e.sc);
        k_glqmr_lanczos<T><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.fl, e.sc, V, W, Pt, Zh, e.part);
        k_qmr_s2<<<1, kScalar, 0, e.st>>>(e.ctl, e.part, e.nb, e.sc, 1.0);
        k_glqmr_step<T><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.fl, e.sc, 1, x, R, D, S, P, Pt, V, W, Qd, e.part);
        k_qmr_s3<<<1, kScalar, 0, e.st>>>(e.ctl, e.hist, e.part, e.nb, e.sc);
        SKR_LAUNCHED();
    };
    return m;
}

template <class T>
Method<T> make_egl_qmr(Env<T>& e, Arena& ar, T* rhs, T* x) {
    Method<T> m;
    T* R = (T*)ar.take(e.blk_bytes());
    T* V = (T*)ar.take(e.blk_bytes());
    T* P = (T*)ar.take(e.blk_bytes());
    T* Pt = (T*)ar.take(e.blk_bytes());
    T* D = (T*)ar.take(e.blk_bytes());
    T* S = (T*)ar.take(e.blk_bytes());
    T* w = (T*)ar.take((size_t)e.n * sizeof(T));
    T* qd = (T*)ar.take((size_t)e.n * sizeof(T));
    T* zh = (T*)ar.take((size_t)e.n * sizeof(T));
    m.mv_per_iter = e.s + 1;
    const double xs = (double)e.s;
    m.init = [=, &e]() {
        k_copy<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, rhs, R, V, nullptr);
        k_fill0<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, x, D, S, P);
        k_row_mean<T><<<(e.n + kBlock - 1) / kBlock, kBlock, 0, e.st>>>(e.n, e.s, rhs, w);
        Flat fv{(size_t)e.n, (((size_t)e.n + e.nb - 1) / e.nb + kBlock - 1) / kBlock * kBlock};
        k_fill0<T><<<e.nb, kBlock, 0, e.st>>>(fv, qd, nullptr, nullptr, nullptr);
        k_flat_nrm_dot<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, R, nullptr, e.part);
        k_init_ctl2<<<1, kScalar, 0, e.st>>>(e.ctl, e.hist, e.part, e.nb);
        k_egl_init_red<T><<<e.nb, kBlock, 0, e.st>>>(e.ly, e.n, e.rpc, V, w, e.part);
        k_qmr_s0<<<1, kScalar, 0, e.st>>>(e.ctl, e.part, e.nb, e.sc, xs);
        k_eglqmr_step<T><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.ly, e.n, e.rpc, e.sc, 0, x, R, D, S, P, Pt, V, w, qd,
                                                     e.part);
        SKR_LAUNCHED();
    };
    m.iter = [=, &e]() {
        spmm(e, e.A, e.ly, P, Pt, EpiVecSum<T>{qd, e.part}, e.ctl);
        spmm(e, e.AH, e.lyv, qd, zh, EpiNone{}, e.ctl);
        k_qmr_s1<<<1, kScalar, 0, e.st>>>(e.ctl, e.part, e.nb, e.sc);
        k_eglqmr_lanczos<T><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.ly, e.n, e.rpc, e.sc, V, w, Pt, zh, e.part);
        k_qmr_s2<<<1, kScalar, 0, e.st>>>(e.ctl, e.part, e.nb, e.sc, xs);
        k_eglqmr_step<T><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.ly, e.n, e.rpc, e.sc, 1, x, R, D, S, P, Pt, V, w, qd,
                                                     e.part);
        k_qmr_s3<<<1, kScalar, 0, e.st>>>(e.ctl, e.hist, e.part, e.nb, e.sc);
        SKR_LAUNCHED();
    };
    return m;
}

template <class T>
Method<T> make_gl_bicgstab(Env<T>& e, Arena& ar, T* rhs, T* x) {
    Method<T> m;
    T* R = (T*)ar.take(e.blk_bytes());
    T* Rt = (T*)ar.take(e.blk_bytes());
    T* P = (T*)ar.take(e.blk_bytes());
    T* V = (T*)ar.take(e.blk_bytes());
    T* S = (T*)ar.take(e.blk_bytes());
    T* Tm = (T*)ar.take(e.blk_bytes());
    m.mv_per_iter = 2LL * e.s;
    m.init = [=, &e]() {
        k_copy<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, rhs, R, Rt, P);
        k_fill0<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, x, nullptr, nullptr, nullptr);
        k_flat_nrm_dot<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, R, Rt, e.part);
        k_s_rho0<<<1, kScalar, 0, e.st>>>(e.part, e.nb, 1, 2, e.sc);
        k_init_ctl2<<<1, kScalar, 0, e.st>>>(e.ctl, e.hist, e.part, e.nb);
        SKR_LAUNCHED();
    };
    m.iter = [=, &e]() {
        spmm(e, e.A, e.ly, P, V, EpiTrace<T>{Rt, e.part}, e.ctl);
        k_s_alpha<<<1, kScalar, 0, e.st>>>(e.ctl, e.part, e.nb, e.sc);
        k_stab_s<T><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.fl, e.sc, R, V, S);
        spmm(e, e.A, e.ly, S, Tm, EpiTraceOmega<T>{S, e.part}, e.ctl);
        k_s_omega<<<1, kScalar, 0, e.st>>>(e.ctl, e.part, e.nb, e.sc);
        k_stab_upd<T><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.fl, e.sc, x, R, Rt, P, S, Tm, e.part);
        k_s_stab_beta<<<1, kScalar, 0, e.st>>>(e.ctl, e.hist, e.part, e.nb, e.sc);
        k_stab_dir<T><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.fl, e.sc, R, V, P);
        SKR_LAUNCHED();
    };
    return m;
}

template <class T, int J>
Method<T> make_bl_bicg_rq(Env<T>& e, Arena& ar, T* rhs, T* x) {
    Method<T> m;
    T* Q = (T*)ar.take(e.blk_bytes());
    T* Qh = (T*)ar.take(e.blk_bytes());
    T* V = (T*)ar.take(e.blk_bytes());
    T* Vh = (T*)ar.take(e.blk_bytes());
    T* W = (T*)ar.take(e.blk_bytes());
    T* Wh = (T*)ar.take(e.blk_bytes());
    T* Z = (T*)ar.take(e.blk_bytes());
    T* Zh = (T*)ar.take(e.blk_bytes());
    m.mv_per_iter = 2LL * e.s;
    const int s = e.s, ss = s * s;
    const Layout lt = tile_layout(e);
    m.init = [=, &e]() {
        k_fill0<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, x, nullptr, nullptr, nullptr);
        k_bl_gram<T, J><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.tl, rhs, rhs, e.part);
        SKR_LAUNCHED();
        cholqr<T, J>(e, 0, rhs, Q, TRI_G_OUT_OUT, nullptr);   // Q0, C0 = S, M = Q0^H Q0
        reduce2(e, ss);
        k_bl_init<<<1, kScalar, 4 * (size_t)ss * sizeof(c64), e.st>>>(e.ctl, e.hist, s, 1, e.part2, e.p2, M_M,
                                                                      e.mats);
        k_copy<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, Q, Qh, V, Vh);
        SKR_LAUNCHED();
    };
    m.iter = [=, &e]() {
        spmm_j<T, J>(e, e.A, lt, V, W, EpiGram<T, J>{Vh, e.part}, e.ctl);           // W = A V, G = V^^H W
        spmm_j<T, J>(e, e.AH, lt, Vh, Wh, EpiNone{}, e.ctl);                      // W^ = A^H V^
        reduce2(e, ss);
        k_blrq_alpha<<<1, kCoefThreads, 4 * (size_t)ss * sizeof(c64), e.st>>>(e.ctl, s, e.part2, e.p2, e.mats, e.sc);
        blrq_updz<T, J>(e, x, V, Q, W, Z);
        cholqr<T, J>(e, 0, Z, Q, 0, nullptr);                                     // Q' S = Q - W alpha
        axpm<T, J, true>(e, M_ALPHAH, 0, Qh, Wh, nullptr, Zh);
        cholqr<T, J>(e, 1, Zh, Qh, TRI_G_OUT_OTHER, Q);                           // Q^' S^, M' = Q^'^H Q'
        reduce2(e, ss);
        k_blrq_beta<<<1, kCoefThreads, 4 * (size_t)ss * sizeof(c64), e.st>>>(e.ctl, e.hist, s, e.part2, e.p2, e.mats);
        axpm<T, J, false>(e, M_BETA, 0, Q, V, nullptr, V);
        axpm<T, J, false>(e, M_BETAH, 0, Qh, Vh, nullptr, Vh);
    };
    return m;
}

template <class T, int J>
Method<T> make_bl_bicgstab_rq(Env<T>& e, Arena& ar, T* rhs, T* x) {
    Method<T> m;
    T* Q = (T*)ar.take(e.blk_bytes());
    T* U = (T*)ar.take(e.blk_bytes());
    T* W = (T*)ar.take(e.blk_bytes());
    T* St = (T*)ar.take(e.blk_bytes());
    T* Tt = (T*)ar.take(e.blk_bytes());
    T* Z = (T*)ar.take(e.blk_bytes());
    T* Rt = (T*)ar.take(e.blk_bytes());
    m.mv_per_iter = 2LL * e.s;
    const int s = e.s, ss = s * s;
    const Layout lt = tile_layout(e);
    m.init = [=, &e]() {
        k_copy<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, rhs, Rt, nullptr, nullptr);
        k_fill0<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, x, nullptr, nullptr, nullptr);
        k_bl_gram<T, J><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.tl, rhs, rhs, e.part);
        SKR_LAUNCHED();
        cholqr<T, J>(e, 0, rhs, Q, TRI_G_OTHER_OUT, Rt);                         // Q0, N = R~^H Q0
        reduce2(e, ss);
        k_bl_init<<<1, kScalar, 4 * (size_t)ss * sizeof(c64), e.st>>>(e.ctl, e.hist, s, 0, e.part2, e.p2, M_N,
                                                                      e.mats);
        k_copy<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, Q, U, nullptr, nullptr);
        SKR_LAUNCHED();
    };
    m.iter = [=, &e]() {
        spmm_j<T, J>(e, e.A, lt, U, W, EpiGram<T, J>{Rt, e.part}, e.ctl);           // W = A U, G = R~^H W
        reduce2(e, ss);
        k_blst_a<<<1, kCoefThreads, 4 * (size_t)ss * sizeof(c64), e.st>>>(e.ctl, s, e.part2, e.p2, e.mats, e.sc);
        axpm<T, J, false>(e, M_TMP, 0, Q, W, nullptr, St);                         // S~ = Q - W a
        spmm_j<T, J>(e, e.A, lt, St, Tt, EpiGramOmega<T, J>{St, e.part}, e.ctl);    // T~ = A S~
        reduce2(e, 2 * ss);
        k_blst_omega<<<1, kCoefThreads, 4 * (size_t)ss * sizeof(c64), e.st>>>(e.ctl, s, e.part2, e.p2, e.mats, e.sc);
        blst_upd<T, J>(e, x, U, St, Tt, Z);
        cholqr<T, J>(e, 0, Z, Q, TRI_G_OTHER_OUT, Rt);                            // Q' Sigma = Z, N' = R~^H Q'
        reduce2(e, ss);
        k_blst_b<<<1, kCoefThreads, 4 * (size_t)ss * sizeof(c64), e.st>>>(e.ctl, e.hist, s, e.part2, e.p2, e.mats, e.sc);
        axpm<T, J, false>(e, M_B, SC_GAMMA, Q, U, W, U);                           // U = Q + (U - omega W) b
    };
    return m;
}

// Block BiCG (Algorithm 3, all four s x s coefficient matrices from their own
// Gram matrices) and, with diag = 1, loop-interchanged BiCG (Algorithm 1): the
// same schedule with the diagonals of the Gram matrices, i.e. s independent
// BiCG recurrences (alpha^ = conj(alpha), beta^ = conj(beta)).
template <class T, int J>
Method<T> make_bl_bicg(Env<T>& e, Arena& ar, T* rhs, T* x, int diag) {
    Method<T> m;
    T* R = (T*)ar.take(e.blk_bytes());
    T* Rh = (T*)ar.take(e.blk_bytes());
    T* P = (T*)ar.take(e.blk_bytes());
    T* Ph = (T*)ar.take(e.blk_bytes());
    T* Q = (T*)ar.take(e.blk_bytes());
    T* Qh = (T*)ar.take(e.blk_bytes());
    m.mv_per_iter = 2LL * e.s;
    const int s = e.s, ss = s * s;
    const Layout lt = tile_layout(e);
    const size_t lds3 = 3 * (size_t)ss * sizeof(c64);
    m.init = [=, &e]() {
        k_copy<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, rhs, R, Rh, P);
        k_copy<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, rhs, Ph, nullptr, nullptr);
        k_fill0<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, x, nullptr, nullptr, nullptr);
        k_flat_nrm_dot<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, R, nullptr, e.part);
        k_init_ctl2<<<1, kScalar, 0, e.st>>>(e.ctl, e.hist, e.part, e.nb);
        k_bl_gram<T, J><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.tl, Rh, R, e.part);   // R^^H R
        SKR_LAUNCHED();
        reduce2(e, ss);
        k_stash<<<1, kScalar, 0, e.st>>>(e.ctl, e.part2, e.p2, s, e.mats, M_RHR);
        SKR_LAUNCHED();
    };
    m.iter = [=, &e]() {
        spmm_j<T, J>(e, e.A, lt, P, Q, EpiGram<T, J>{Ph, e.part}, e.ctl);           // Q = A P, G1 = P^^H Q
        reduce2(e, ss);
        k_stash<<<1, kScalar, 0, e.st>>>(e.ctl, e.part2, e.p2, s, e.mats, M_G1);
        SKR_LAUNCHED();
        if (diag) {
            spmm_j<T, J>(e, e.AH, lt, Ph, Qh, EpiNone{}, e.ctl);                    // Q^ = A^H P^
        } else {
            spmm_j<T, J>(e, e.AH, lt, Ph, Qh, EpiGram<T, J>{P, e.part}, e.ctl);     // Q^ = A^H P^, G2 = P^H Q^
            reduce2(e, ss);
        }
        k_blb_alpha<<<1, kScalar, lds3, e.st>>>(e.ctl, s, diag, e.part2, e.p2, e.mats);
        SKR_LAUNCHED();
        axpm<T, J, false>(e, M_ALPHA, 0, x, P, nullptr, x);                         // X += P alpha
        axpm<T, J, true>(e, M_TMP, 0, R, Q, nullptr, R);                            // R -= Q alpha, R^H R
        reduce2(e, ss);
        k_stash<<<1, kScalar, 0, e.st>>>(e.ctl, e.part2, e.p2, s, e.mats, M_RR);
        SKR_LAUNCHED();
        axpm<T, J, false>(e, M_ALPHAH, 0, Rh, Qh, nullptr, Rh);                     // R^ -= Q^ alpha^
        k_bl_gram<T, J><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.tl, Rh, R, e.part);     // R^^H R
        SKR_LAUNCHED();
        reduce2(e, ss);
        k_blb_beta<<<1, kScalar, lds3, e.st>>>(e.ctl, e.hist, s, diag, e.part2, e.p2, e.mats);
        SKR_LAUNCHED();
        axpm<T, J, false>(e, M_BETA, 0, R, P, nullptr, P);                          // P = R + P beta
        axpm<T, J, false>(e, M_BETAH, 0, Rh, Ph, nullptr, Ph);                      // P^ = R^ + P^ beta^
    };
    return m;
}

// Block BiCGStab (El Guennouni et al.): s x s alpha and beta, scalar omega.
template <class T, int J>
Method<T> make_bl_bicgstab(Env<T>& e, Arena& ar, T* rhs, T* x) {
    Method<T> m;
    T* R = (T*)ar.take(e.blk_bytes());
    T* Rt = (T*)ar.take(e.blk_bytes());
    T* P = (T*)ar.take(e.blk_bytes());
    T* V = (T*)ar.take(e.blk_bytes());
    T* S = (T*)ar.take(e.blk_bytes());
    T* Tm = (T*)ar.take(e.blk_bytes());
    m.mv_per_iter = 2LL * e.s;
    const int s = e.s, ss = s * s;
    const Layout lt = tile_layout(e);
    const size_t lds4 = 4 * (size_t)ss * sizeof(c64);
    m.init = [=, &e]() {
        k_copy<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, rhs, R, Rt, P);
        k_fill0<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, x, nullptr, nullptr, nullptr);
        k_flat_nrm_dot<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, R, nullptr, e.part);
        k_init_ctl2<<<1, kScalar, 0, e.st>>>(e.ctl, e.hist, e.part, e.nb);
        k_bl_gram<T, J><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.tl, Rt, R, e.part);    // N = R~^H R
        SKR_LAUNCHED();
        reduce2(e, ss);
        k_stash<<<1, kScalar, 0, e.st>>>(e.ctl, e.part2, e.p2, s, e.mats, M_N);
        SKR_LAUNCHED();
    };
    m.iter = [=, &e]() {
        spmm_j<T, J>(e, e.A, lt, P, V, EpiGram<T, J>{Rt, e.part}, e.ctl);           // V = A P, G = R~^H V
        reduce2(e, ss);
        k_blst_a<<<1, kCoefThreads, lds4, e.st>>>(e.ctl, s, e.part2, e.p2, e.mats, e.sc); // alpha = G^{-1} N
        SKR_LAUNCHED();
        axpm<T, J, false>(e, M_TMP, 0, R, V, nullptr, S);                           // S = R - V alpha
        spmm(e, e.A, e.ly, S, Tm, EpiTraceOmega<T>{S, e.part}, e.ctl);              // T = A S
        k_blbs_omega<<<1, kScalar, 0, e.st>>>(e.ctl, s, e.part, e.nb, e.sc, e.mats);
        SKR_LAUNCHED();
        axpm<T, J, false>(e, M_A, 0, x, P, nullptr, x);                             // X += P alpha
        axpm<T, J, false>(e, M_W, 0, x, S, nullptr, x);                             // X += omega S
        axpm<T, J, true>(e, M_MW, 0, S, Tm, nullptr, R);                            // R = S - omega T, R^H R
        reduce2(e, ss);
        k_stash<<<1, kScalar, 0, e.st>>>(e.ctl, e.part2, e.p2, s, e.mats, M_RR);
        k_bl_gram<T, J><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.tl, Rt, Tm, e.part);    // R~^H T
        SKR_LAUNCHED();
        reduce2(e, ss);
        k_stash<<<1, kScalar, 0, e.st>>>(e.ctl, e.part2, e.p2, s, e.mats, M_RT);
        k_bl_gram<T, J><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.tl, Rt, R, e.part);     // N' = R~^H R
        SKR_LAUNCHED();
        reduce2(e, ss);
        k_blbs_beta<<<1, kScalar, 2 * (size_t)ss * sizeof(c64), e.st>>>(e.ctl, e.hist, s, e.part2, e.p2, e.mats,
                                                                          e.sc);
        SKR_LAUNCHED();
        axpm<T, J, false>(e, M_B, SC_GAMMA, R, P, V, P);                            // P = R + (P - omega V) beta
    };
    return m;
}

// Loop-interchanged BiCGStab: s independent BiCGStab recurrences (shadow
// r~_c = r0_c), their products with A gathered into block products.  The
// per-column alpha, omega and beta are diagonal s x s slots applied by the block
// update kernels; the reductions are Gram diagonals.
template <class T, int J>
Method<T> make_li_bicgstab(Env<T>& e, Arena& ar, T* rhs, T* x) {
    Method<T> m;
    T* R = (T*)ar.take(e.blk_bytes());
    T* Rt = (T*)ar.take(e.blk_bytes());
    T* P = (T*)ar.take(e.blk_bytes());
    T* V = (T*)ar.take(e.blk_bytes());
    T* S = (T*)ar.take(e.blk_bytes());
    T* Tm = (T*)ar.take(e.blk_bytes());
    m.mv_per_iter = 2LL * e.s;
    const int s = e.s, ss = s * s;
    const Layout lt = tile_layout(e);
    m.init = [=, &e]() {
        k_copy<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, rhs, R, Rt, P);
        k_fill0<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, x, nullptr, nullptr, nullptr);
        k_flat_nrm_dot<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, R, nullptr, e.part);
        k_init_ctl2<<<1, kScalar, 0, e.st>>>(e.ctl, e.hist, e.part, e.nb);
        k_bl_gram<T, J><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.tl, Rt, R, e.part);    // rho = diag(R~^H R)
        SKR_LAUNCHED();
        reduce2(e, ss);
        k_stash<<<1, kScalar, 0, e.st>>>(e.ctl, e.part2, e.p2, s, e.mats, M_N);
        SKR_LAUNCHED();
    };
    m.iter = [=, &e]() {
        spmm_j<T, J>(e, e.A, lt, P, V, EpiGram<T, J>{Rt, e.part}, e.ctl);           // V = A P, R~^H V
        reduce2(e, ss);
        k_lbs_alpha<<<1, kScalar, 0, e.st>>>(e.ctl, s, e.part2, e.p2, e.mats);
        SKR_LAUNCHED();
        axpm<T, J, false>(e, M_TMP, 0, R, V, nullptr, S);                           // S = R - V diag(alpha)
        spmm_j<T, J>(e, e.A, lt, S, Tm, EpiGramOmega<T, J>{S, e.part}, e.ctl);      // T = A S, T^H S, T^H T
        reduce2(e, 2 * ss);
        k_lbs_omega<<<1, kScalar, 0, e.st>>>(e.ctl, s, e.part2, e.p2, e.mats);
        SKR_LAUNCHED();
        axpm<T, J, false>(e, M_A, 0, x, P, nullptr, x);                             // X += P diag(alpha)
        axpm<T, J, false>(e, M_W, 0, x, S, nullptr, x);                             // X += S diag(omega)
        axpm<T, J, true>(e, M_MW, 0, S, Tm, nullptr, R);                            // R = S - T diag(omega)
        reduce2(e, ss);
        k_stash<<<1, kScalar, 0, e.st>>>(e.ctl, e.part2, e.p2, s, e.mats, M_RR);
        k_bl_gram<T, J><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.tl, Rt, R, e.part);     // rho' = diag(R~^H R)
        SKR_LAUNCHED();
        reduce2(e, ss);
        k_lbs_beta<<<1, kScalar, 0, e.st>>>(e.ctl, e.hist, s, e.part2, e.p2, e.mats);
        SKR_LAUNCHED();
        axpm<T, J, false>(e, M_MW, 0, P, V, nullptr, P);                            // P -= V diag(omega)
        axpm<T, J, false>(e, M_B, 0, R, P, nullptr, P);                             // P = R + P diag(beta)
    };
    return m;
}

// Loop-interchanged QMR: s independent QMR recurrences (the coupled two-term
// form of the global variant, with per-column rho, xi, delta, eps, beta,
// theta, gamma, eta), their products with A and A^H gathered into block
// products.  Every per-column scaling is a diagonal slot applied by the block
// update kernels, every per-column reduction a Gram diagonal.
template <class T, int J>
Method<T> make_li_qmr(Env<T>& e, Arena& ar, T* rhs, T* x) {
    Method<T> m;
    T* R = (T*)ar.take(e.blk_bytes());
    T* V = (T*)ar.take(e.blk_bytes());
    T* W = (T*)ar.take(e.blk_bytes());
    T* P = (T*)ar.take(e.blk_bytes());
    T* Qd = (T*)ar.take(e.blk_bytes());
    T* Pt = (T*)ar.take(e.blk_bytes());
    T* Zh = (T*)ar.take(e.blk_bytes());
    T* D = (T*)ar.take(e.blk_bytes());
    T* S = (T*)ar.take(e.blk_bytes());
    m.mv_per_iter = 2LL * e.s;
    const int s = e.s, ss = s * s;
    const Layout lt = tile_layout(e);
    auto gram = [=, &e](const T* Z, const T* Y, int slot) {   // mats[slot] = Z^H Y
        k_bl_gram<T, J><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.tl, Z, Y, e.part);
        SKR_LAUNCHED();
        reduce2(e, ss);
        k_stash<<<1, kScalar, 0, e.st>>>(e.ctl, e.part2, e.p2, s, e.mats, slot);
        SKR_LAUNCHED();
    };
    auto stash = [=, &e](int slot) {
        reduce2(e, ss);
        k_stash<<<1, kScalar, 0, e.st>>>(e.ctl, e.part2, e.p2, s, e.mats, slot);
        SKR_LAUNCHED();
    };
    // V = V diag(1/rho), W = W diag(1/xi), P = V - P diag(c_P), Qd = W - Qd diag(c_Q)
    auto directions = [=, &e]() {
        axpm<T, J, false>(e, M_QIRHO, 0, nullptr, V, nullptr, V);
        axpm<T, J, false>(e, M_QIXI, 0, nullptr, W, nullptr, W);
        axpm<T, J, false>(e, M_QMCP, 0, V, P, nullptr, P);
        axpm<T, J, false>(e, M_QMCQ, 0, W, Qd, nullptr, Qd);
    };
    m.init = [=, &e]() {
        k_copy<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, rhs, R, V, W);
        k_fill0<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, x, D, S, P);
        k_fill0<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, Qd, nullptr, nullptr, nullptr);
        k_flat_nrm_dot<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, R, nullptr, e.part);
        k_init_ctl2<<<1, kScalar, 0, e.st>>>(e.ctl, e.hist, e.part, e.nb);
        SKR_LAUNCHED();
        gram(V, V, M_QVV);
        gram(W, W, M_QWW);
        gram(W, V, M_QWV);
        k_lqmr_s0<<<1, kScalar, 0, e.st>>>(e.ctl, s, e.mats);
        SKR_LAUNCHED();
        directions();
    };
    m.iter = [=, &e]() {
        spmm_j<T, J>(e, e.A, lt, P, Pt, EpiGram<T, J>{Qd, e.part}, e.ctl);         // Pt = A P, Qd^H Pt
        reduce2(e, ss);
        k_lqmr_s1<<<1, kScalar, 0, e.st>>>(e.ctl, s, e.part2, e.p2, e.mats);
        SKR_LAUNCHED();
        spmm_j<T, J>(e, e.AH, lt, Qd, Zh, EpiNone{}, e.ctl);                      // Zh = A^H Qd
        axpm<T, J, true>(e, M_QMB, 0, Pt, V, nullptr, V);                          // Vt = Pt - V diag(beta)
        stash(M_QVV);
        axpm<T, J, true>(e, M_QMBC, 0, Zh, W, nullptr, W);                         // Wt = Zh - W diag(conj beta)
        stash(M_QWW);
        gram(W, V, M_QWV);
        k_lqmr_s2<<<1, kScalar, 0, e.st>>>(e.ctl, s, e.mats);
        SKR_LAUNCHED();
        axpm<T, J, false>(e, M_QF, 0, nullptr, D, nullptr, D);                     // D = P diag(eta) + D diag(f)
        axpm<T, J, false>(e, M_QETA, 0, D, P, nullptr, D);
        axpm<T, J, false>(e, M_QF, 0, nullptr, S, nullptr, S);                     // S = Pt diag(eta) + S diag(f)
        axpm<T, J, false>(e, M_QETA, 0, S, Pt, nullptr, S);
        axpm<T, J, false>(e, M_ID, 0, x, D, nullptr, x);                           // X += D
        axpm<T, J, true>(e, M_MID, 0, R, S, nullptr, R);                           // R -= S
        stash(M_RR);
        k_lqmr_s3<<<1, kScalar, 0, e.st>>>(e.ctl, e.hist, s, e.mats);
        SKR_LAUNCHED();
        directions();
    };
    return m;
}

}  // namespace skr
