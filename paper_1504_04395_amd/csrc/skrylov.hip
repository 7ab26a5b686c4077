// C ABI of the simultaneous short-recurrence Krylov solvers (see include/skrylov.h).
//
// Matrix set-up: the index structure of A^H is built once per pattern on the
// host by a stable counting sort (column-major traversal of A's CSR), together
// with the permutation perm with A^H[p] = conj(A[perm[p]]); values are gathered
// through perm on the device, so a value refresh (skr_matrix_update_values)
// never touches the host.  SELL-C-sigma index structures are built on the host
// in the same way (plus a slot -> CSR-entry map for the device-side value
// gather).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/skrylov.h"
#include "engine.hpp"
#include "csr_host.hpp"
#include "sell.hpp"
#include "smallsys.hpp"

using namespace skr;

// ============================================================== device helpers
template <class T>
__global__ void k_gather_conj(int nnz, const int* __restrict__ perm, const T* __restrict__ va, T* __restrict__ out) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz) out[p] = conj_(va[perm[p]]);
}
template <class T>
__global__ void k_gather_sell(size_t slots, const int* __restrict__ idx, const T* __restrict__ va, T* __restrict__ out) {
    size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < slots) {
        int k = idx[p];
        out[p] = k >= 0 ? va[k] : zero<T>();
    }
}
template <class Tin, class Tout>
__global__ void k_convert(size_t count, const Tin* __restrict__ in, Tout* __restrict__ out) {
    size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < count) out[p] = down<Tout>(up(in[p]));
}
// dense strided <-> contiguous copies of an n x s block (ld in elements)
template <class T>
__global__ void k_pack(int n, int s, const T* __restrict__ src, int64_t lds_, T* __restrict__ dst, int64_t ldd) {
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)n * s) return;
    size_t i = e / s, c = e - i * s;
    dst[i * ldd + c] = src[i * lds_ + c];
}
// R = B - Y (T64), optional R32 = (T32) R; part = (||R||^2, ||B||^2)
template <class T, class T32>
__global__ __launch_bounds__(kBlock) void k_resid(Flat fl, const T* __restrict__ B, const T* __restrict__ Y,
                                                  T* __restrict__ R, T32* __restrict__ R32, c64* part) {
    c64 acc[2] = {{0.0, 0.0}, {0.0, 0.0}};
    SKR_FLAT_LOOP(fl) {
        T b = B[e];
        T r = sub_(b, Y[e]);
        if (R) R[e] = r;
        if (R32) R32[e] = down<T32>(up(r));
        nrm_acc(acc[0].x, r);
        nrm_acc(acc[1].x, b);
    }
    block_reduce_store<2>(acc, part + (size_t)blockIdx.x * 2);
}
// X += D (same type) or X += D * M (mats slot, FP64 arithmetic), D of type Td
template <class T, class Td, int J>
__global__ __launch_bounds__(kBlock) void k_xupd(Tile16 tl, const c64* __restrict__ mats, int mslot,
                                                 T* __restrict__ X, const Td* __restrict__ D, int zero_x) {
    extern __shared__ c64 dyn[];
    using VV = Val<T>;
    const int s = tl.s;
    VV* M = reinterpret_cast<VV*>(dyn);
    if (mslot >= 0) lds_load_mat(M, mats + (size_t)mslot * s * s, s);
    __syncthreads();
    Coef<T, J> cf;
    if (mslot >= 0) cf.load(M, s, threadIdx.x & 15);
    SKR_TILE_LOOP(tl) {
        const int i = base_ + grp;
        const bool valid = i < r1_;
        VV d[J], x[J];
        load_row<Td, J>(D, i, valid, lane, s, d);
        if (zero_x) {
#pragma unroll
            for (int j = 0; j < J; ++j) x[j] = vzero<VV>();
        } else {
            load_row<T, J>(X, i, valid, lane, s, x);
        }
        if (mslot >= 0) {
            cf.apply(d, lane, x);
        } else {
#pragma unroll
            for (int j = 0; j < J; ++j) x[j] = x[j] + d[j];
        }
        store_row<T, J>(X, i, valid, lane, s, x);
    }
}
__global__ __launch_bounds__(kScalar) void k_copy_mat(c64* mats, int s, int from, int to) {
    for (int e = threadIdx.x; e < s * s; e += blockDim.x) mats[(size_t)to * s * s + e] = mats[(size_t)from * s * s + e];
}
__global__ __launch_bounds__(kScalar) void k_sum2(const c64* part, int np, c64* out) {
    __shared__ c64 r[2];
    sum_partials<2>(part, np, r);
    if (threadIdx.x == 0) {
        out[0] = r[0];
        out[1] = r[1];
    }
}
// SDDMM: out[k] = scale * sum_c G[i,c] conj(X[j,c]) over A's pattern (L lanes per row)
template <class T, int J>
__global__ __launch_bounds__(kBlock) void k_sddmm(Layout ly, int n, int rpc, const int* __restrict__ rp,
                                                  const int* __restrict__ ci, const T* __restrict__ G,
                                                  const T* __restrict__ X, double scale, T* __restrict__ out) {
    const int s = ly.s;
    SKR_ROW_LOOP(ly, n, rpc) {
        const int i = base_ + grp;
        const bool valid = i < r1_;
        c64 g[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            int c = lane + ly.L * j;
            g[j] = (valid && c < s) ? up(G[(size_t)i * s + c]) : c64{0.0, 0.0};
        }
        const int k0 = valid ? rp[i] : 0, k1 = valid ? rp[i + 1] : 0;
        for (int k = k0; k < k1; ++k) {
            const int col = ci[k];
            c64 acc = {0.0, 0.0};
#pragma unroll
            for (int j = 0; j < J; ++j) {
                int c = lane + ly.L * j;
                if (c < s) {
                    c64 x = up(X[(size_t)col * s + c]);
                    acc.x = fma(g[j].x, x.x, fma(g[j].y, x.y, acc.x));
                    acc.y = fma(g[j].y, x.x, fma(-g[j].x, x.y, acc.y));
                }
            }
            for (int off = ly.L >> 1; off > 0; off >>= 1) {
                acc.x += __shfl_xor(acc.x, off, ly.L);
                acc.y += __shfl_xor(acc.y, off, ly.L);
            }
            if (lane == 0) out[k] = down<T>(scale * acc);
        }
    }
}

// ============================================================== host structures
struct GraphEntry {
    uint64_t key;
    hipGraphExec_t exec;
};

struct skr_context {
    int device = 0;
    hipStream_t user = nullptr;
    hipStream_t own = nullptr;
    std::string err;
    char* arena = nullptr;
    size_t arena_cap = 0;
    Ctl* hin = nullptr;   // pinned
    Ctl* hout = nullptr;  // pinned
    c64* hsum = nullptr;  // pinned, small
    c64* hmat = nullptr;  // pinned, kMaxS x kMaxS: s x s results of the allocation-free calls
    double* hhist = nullptr;   // pinned residual history of the single-workgroup path (grow-only)
    size_t hhist_cap = 0;      // entries
    char* scratch = nullptr;   // device address of this device's static scratch array (or null)
    int lds_max = 0;           // LDS bytes one workgroup may hold on this device
    std::vector<GraphEntry> graphs;
    std::vector<skr_matrix*> mats;   // live matrices (orphaned when the context goes first)
    void* stage = nullptr;           // cached staging blocks for B and X (grow-only)
    size_t stage_cap = 0;
    hipStream_t stream() const { return user ? user : own; }
};

struct DevSell {
    int C = 0, sigma = 0;
    size_t slots = 0;
    int* cptr = nullptr;
    int* clen = nullptr;
    int* row = nullptr;
    int* ci = nullptr;
    int* idx = nullptr;
    void* va = nullptr;
    void* va32 = nullptr;
};

struct skr_matrix {
    skr_context* ctx = nullptr;
    int device = 0;
    int n = 0, nnz = 0, dtype = 0;
    int *rp = nullptr, *ci = nullptr;
    void *va = nullptr, *va32 = nullptr;
    int *rpH = nullptr, *ciH = nullptr, *perm = nullptr;
    void *vaH = nullptr, *vaH32 = nullptr;
    bool sell = false;
    DevSell SA, SAH;
    double sell_pad = 0.0;
    Ilu* ilu = nullptr;   // right ILU(0) factors (skr_matrix_ilu0), dropped when the values change
};

// ---------------------------------------------------------------- static scratch
// Device memory of the allocation-free entry point (skr_block_qr_noalloc): its
// control block, coefficient slots and reduction partials, at most
// kNoAllocBytes.  Each device holds one copy for the life of the process, and
// every call on that device shares it.  Host code never uses this name as an
// address: the per-device address comes from hipGetSymbolAddress at context
// creation (scratch_addr below).
constexpr size_t kNoAllocBytes = 9u << 20;
constexpr int kNoAllocMaxS = 16;
__device__ __align__(256) char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;

// Address of `scratch` on `device` (which must be current), looked up once per
// device; null if the lookup failed.
char* scratch_addr(int device, std::string* why) {
    static std::mutex mu;
    static char* addr[kMaxDevices] = {};
    static bool tried[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) {
        *why = "device index beyond the scratch table";
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (!tried[device]) {
        tried[device] = true;
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e == hipSuccess) addr[device] = (char*)p;
        else *why = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    }
    if (!addr[device] && why->empty()) *why = "the scratch array of this device could not be located";
    return addr[device];
}

size_t elt(int dtype, bool fp32) {
    if (dtype == SKR_C64) return fp32 ? 8 : 16;
    return fp32 ? 4 : 8;
}

void invalidate_graphs(skr_context* c) {
    for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    c->graphs.clear();
}

template <class T>
void* dmalloc(size_t count) {
    void* p = nullptr;
    if (count == 0) count = 1;
    if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) throw std::bad_alloc();
    return p;
}

uint64_t fnv(const void* p, size_t n, uint64_t h = 1469598103934665603ULL) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ULL;
    }
    return h;
}

// ---------------------------------------------------------------- SELL upload (host build in sell.hpp)
void upload_sell(DevSell& d, const HostSell& h, int C, int sigma, int n) {
    d.C = C;
    d.sigma = sigma;
    d.slots = h.ci.size();
    int nch = (int)h.clen.size();
    d.cptr = (int*)dmalloc<int>(nch + 1);
    d.clen = (int*)dmalloc<int>(nch);
    d.row = (int*)dmalloc<int>(n);
    d.ci = (int*)dmalloc<int>(d.slots);
    d.idx = (int*)dmalloc<int>(d.slots);
    SKR_HIP(hipMemcpy(d.cptr, h.cptr.data(), (nch + 1) * sizeof(int), hipMemcpyHostToDevice));
    SKR_HIP(hipMemcpy(d.clen, h.clen.data(), nch * sizeof(int), hipMemcpyHostToDevice));
    SKR_HIP(hipMemcpy(d.row, h.row.data(), n * sizeof(int), hipMemcpyHostToDevice));
    if (d.slots) {
        SKR_HIP(hipMemcpy(d.ci, h.ci.data(), d.slots * sizeof(int), hipMemcpyHostToDevice));
        SKR_HIP(hipMemcpy(d.idx, h.idx.data(), d.slots * sizeof(int), hipMemcpyHostToDevice));
    }
}

void free_tri(TriDev& t) {
    void* ps[] = {t.rp, t.ci, t.rows, t.dlvl, t.va, t.dg};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    t = TriDev{};
}

void free_ilu(skr_matrix* M) {
    if (!M->ilu) return;
    free_tri(M->ilu->L);
    free_tri(M->ilu->U);
    free_tri(M->ilu->UH);
    free_tri(M->ilu->LH);
    delete M->ilu;
    M->ilu = nullptr;
}

// upload of the level-order copy of a row-ordered operator
template <class T>
void upload_tri(const TriHost<T>& rowwise, int n, TriDev& d, hipStream_t st) {
    TriHost<T> h;
    tri_level_order(rowwise, n, h);
    auto up = [&](void** dst, const void* src, size_t bytes) {
        SKR_HIP(hipMalloc(dst, std::max<size_t>(bytes, 1)));
        if (bytes) SKR_HIP(hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, st));
        d.bytes += bytes;
    };
    up((void**)&d.rp, h.rp.data(), sizeof(int) * (n + 1));
    up((void**)&d.ci, h.ci.data(), sizeof(int) * h.ci.size());
    up((void**)&d.rows, h.rows.data(), sizeof(int) * n);
    up(&d.va, h.va.data(), sizeof(T) * h.va.size());
    if (!h.dg.empty()) up(&d.dg, h.dg.data(), sizeof(T) * n);
    up((void**)&d.dlvl, h.lvl.data(), sizeof(int) * h.lvl.size());
    d.lvl = h.lvl;
    d.maxrows = 0;
    for (size_t l = 0; l + 1 < h.lvl.size(); ++l) d.maxrows = std::max(d.maxrows, h.lvl[l + 1] - h.lvl[l]);
    SKR_HIP(hipStreamSynchronize(st));   // h is released on return
}

// ILU(0) on the host from the device CSR, level schedules, upload of L, U, U^H, L^H.
template <class T>
void build_ilu(skr_matrix* M, hipStream_t st) {
    const int n = M->n, nnz = M->nnz;
    std::vector<int> rp(n + 1), ci(nnz);
    std::vector<T> va(nnz);
    SKR_HIP(hipMemcpyAsync(rp.data(), M->rp, sizeof(int) * (n + 1), hipMemcpyDeviceToHost, st));
    if (nnz) {
        SKR_HIP(hipMemcpyAsync(ci.data(), M->ci, sizeof(int) * nnz, hipMemcpyDeviceToHost, st));
        SKR_HIP(hipMemcpyAsync(va.data(), M->va, sizeof(T) * nnz, hipMemcpyDeviceToHost, st));
    }
    SKR_HIP(hipStreamSynchronize(st));
    TriHost<T> L, U, UH, LH;
    ilu0_factor<T>(n, rp, ci, std::move(va), L, U);
    tri_adjoint(U, n, UH);
    tri_adjoint(L, n, LH);
    tri_levels(L, n, true);
    tri_levels(U, n, false);
    tri_levels(UH, n, true);
    tri_levels(LH, n, false);
    std::unique_ptr<Ilu> p(new Ilu);
    p->dtype = M->dtype;
    try {
        upload_tri(L, n, p->L, st);
        upload_tri(U, n, p->U, st);
        upload_tri(UH, n, p->UH, st);
        upload_tri(LH, n, p->LH, st);
        SKR_HIP(hipStreamSynchronize(st));
    } catch (...) {
        free_tri(p->L);
        free_tri(p->U);
        free_tri(p->UH);
        free_tri(p->LH);
        throw;
    }
    M->ilu = p.release();
}

void free_sell(DevSell& d) {
    (void)hipFree(d.cptr);
    (void)hipFree(d.clen);
    (void)hipFree(d.row);
    (void)hipFree(d.ci);
    (void)hipFree(d.idx);
    (void)hipFree(d.va);
    (void)hipFree(d.va32);
    d = DevSell{};
}

// ---------------------------------------------------------------- value refresh
template <class T, class T32>
void refresh_values_t(skr_matrix* M, hipStream_t st) {
    const int nnz = M->nnz;
    const int tb = 256;
    if (nnz > 0) {
        k_gather_conj<T><<<(nnz + tb - 1) / tb, tb, 0, st>>>(nnz, M->perm, (const T*)M->va, (T*)M->vaH);
        SKR_LAUNCHED();
        if (M->va32) {
            k_convert<T, T32><<<(nnz + tb - 1) / tb, tb, 0, st>>>(nnz, (const T*)M->va, (T32*)M->va32);
            k_convert<T, T32><<<(nnz + tb - 1) / tb, tb, 0, st>>>(nnz, (const T*)M->vaH, (T32*)M->vaH32);
            SKR_LAUNCHED();
        }
    }
    if (M->sell) {
        for (int side = 0; side < 2; ++side) {
            DevSell& d = side ? M->SAH : M->SA;
            const T* src = (const T*)(side ? M->vaH : M->va);
            size_t g = (d.slots + tb - 1) / tb;
            if (d.slots) {
                k_gather_sell<T><<<g, tb, 0, st>>>(d.slots, d.idx, src, (T*)d.va);
                SKR_LAUNCHED();
                if (d.va32) {
                    k_convert<T, T32><<<g, tb, 0, st>>>(d.slots, (const T*)d.va, (T32*)d.va32);
                    SKR_LAUNCHED();
                }
            }
        }
    }
}
void refresh_values(skr_matrix* M, hipStream_t st) {
    if (M->dtype == SKR_C64) refresh_values_t<c64, c32>(M, st);
    else refresh_values_t<double, float>(M, st);
}

void ensure_fp32(skr_matrix* M, hipStream_t st) {
    if (M->va32) return;
    size_t e32 = elt(M->dtype, true);
    SKR_HIP(hipMalloc(&M->va32, std::max<size_t>(1, (size_t)M->nnz) * e32));
    SKR_HIP(hipMalloc(&M->vaH32, std::max<size_t>(1, (size_t)M->nnz) * e32));
    if (M->sell) {
        SKR_HIP(hipMalloc(&M->SA.va32, std::max<size_t>(1, M->SA.slots) * e32));
        SKR_HIP(hipMalloc(&M->SAH.va32, std::max<size_t>(1, M->SAH.slots) * e32));
    }
    refresh_values(M, st);
}

// ---------------------------------------------------------------- operands
template <class T>
Operand<T> operand(const skr_matrix* M, bool hermitian, bool fp32) {
    Operand<T> o;
    if (M->sell) {
        const DevSell& d = hermitian ? M->SAH : M->SA;
        o.sell = true;
        o.sl = SellOp<T>{M->n, d.C, d.cptr, d.clen, d.row, d.ci, (const T*)(fp32 ? d.va32 : d.va)};
    }
    o.csr = CsrOp<T>{M->n, hermitian ? M->rpH : M->rp, hermitian ? M->ciH : M->ci,
                     (const T*)(hermitian ? (fp32 ? M->vaH32 : M->vaH) : (fp32 ? M->va32 : M->va))};
    return o;
}

// common per-solve device state
template <class T>
void take_common(Env<T>& e, Arena& ar, int maxit) {
    const int s = e.s;
    const size_t E = std::max<size_t>(4, 2 * (size_t)s * s);
    e.ctl = (Ctl*)ar.take(sizeof(Ctl));
    e.hist = (double*)ar.take(sizeof(double) * ((size_t)maxit + 2));
    e.sc = (c64*)ar.take(sizeof(c64) * 128);
    e.mats = (c64*)ar.take(sizeof(c64) * (size_t)M_COUNT * s * s);
    e.part = (c64*)ar.take(sizeof(c64) * (size_t)e.nb * E);
    e.part2 = (c64*)ar.take(sizeof(c64) * (size_t)e.p2 * E);
}

void ensure_arena(skr_context* c, size_t bytes) {
    if (bytes <= c->arena_cap) return;
    invalidate_graphs(c);
    if (c->arena) {
        SKR_HIP(hipStreamSynchronize(c->stream()));
        (void)hipFree(c->arena);
        c->arena = nullptr;
        c->arena_cap = 0;
    }
    size_t cap = bytes + bytes / 8 + (1 << 20);
    if (hipMalloc(&c->arena, cap) != hipSuccess) {
        c->arena = nullptr;
        throw std::bad_alloc();
    }
    c->arena_cap = cap;
}

template <class T, int J>
Method<T> make_method(int method, Env<T>& e, Arena& ar, T* rhs, T* x) {
    switch (method) {
        case SKR_GL_BICG: return make_gl_bicg<T>(e, ar, rhs, x);
        case SKR_EGL_BICG: return make_egl_bicg<T>(e, ar, rhs, x);
        case SKR_GL_QMR: return make_gl_qmr<T>(e, ar, rhs, x);
        case SKR_EGL_QMR: return make_egl_qmr<T>(e, ar, rhs, x);
        case SKR_GL_BICGSTAB: return make_gl_bicgstab<T>(e, ar, rhs, x);
        case SKR_BL_BICG_RQ: return make_bl_bicg_rq<T, J>(e, ar, rhs, x);
        case SKR_BL_BICGSTAB_RQ: return make_bl_bicgstab_rq<T, J>(e, ar, rhs, x);
        case SKR_BL_BICG: return make_bl_bicg<T, J>(e, ar, rhs, x, 0);
        case SKR_BL_BICGSTAB: return make_bl_bicgstab<T, J>(e, ar, rhs, x);
        case SKR_LI_BICG: return make_bl_bicg<T, J>(e, ar, rhs, x, 1);
        case SKR_LI_BICGSTAB: return make_li_bicgstab<T, J>(e, ar, rhs, x);
        case SKR_LI_QMR: return make_li_qmr<T, J>(e, ar, rhs, x);
    }
    throw Unsupported{"unknown method"};
}

struct InnerStats {
    int status = 0, iters = 0, bd_iter = -1;
    long long matvecs = 0;
    double rres = 0.0;
    std::vector<double> hist;
};

// Stop state (already copied to c->hout) and history of a finished run (read
// from the device, or from host_hist where the caller has already copied it).
template <class T>
InnerStats inner_stats(skr_context* c, Env<T>& e, long long mv_per_iter, const double* host_hist = nullptr) {
    InnerStats r;
    const Ctl& o = *c->hout;
    r.iters = o.iter;
    r.bd_iter = o.bd_iter;
    r.status = o.status == ST_OK ? SKR_OK : (o.status == ST_BREAKDOWN ? SKR_BREAKDOWN : SKR_NOT_CONVERGED);
    r.matvecs = (long long)o.iter * mv_per_iter;
    r.rres = o.nr0 > 0 ? o.res / o.nr0 : 0.0;
    r.hist.resize((size_t)o.iter + 1);
    if (host_hist)
        std::memcpy(r.hist.data(), host_hist, sizeof(double) * r.hist.size());
    else
        SKR_HIP(hipMemcpy(r.hist.data(), e.hist, sizeof(double) * r.hist.size(), hipMemcpyDeviceToHost));
    return r;
}

// Run a method to completion on A D = rhs (the caller enqueued rhs).
template <class T>
InnerStats iterate(skr_context* c, Env<T>& e, Method<T>& m, int method, double tol, int maxit, int every,
                   bool use_graph, uint64_t key_extra, double div_limit = 0.0) {
    Ctl* h = c->hin;
    std::memset(h, 0, sizeof(Ctl));
    h->done = 0;
    h->status = ST_RUNNING;
    h->bd_iter = -1;
    h->maxit = maxit;
    h->tol = tol;
    h->div_limit = div_limit;
    SKR_HIP(hipMemcpyAsync(e.ctl, h, sizeof(Ctl), hipMemcpyHostToDevice, e.st));
    m.init();
    if (every < 1) every = 1;
    hipGraphExec_t exec = nullptr;
    if (use_graph) {
        struct {
            int method, n, s, nb, rpc, every, sell, tsize;
            const void *a0, *a1, *a2, *h0, *h1, *h2, *ctl, *part;
            uint64_t extra;
        } k{method, e.n, e.s, e.nb, e.rpc, every, e.A.sell ? 1 : 0, (int)sizeof(T),
            e.A.sell ? (const void*)e.A.sl.va : (const void*)e.A.csr.va,
            e.A.sell ? (const void*)e.A.sl.ci : (const void*)e.A.csr.ci,
            e.A.sell ? (const void*)e.A.sl.row : (const void*)e.A.csr.rp,
            e.AH.sell ? (const void*)e.AH.sl.va : (const void*)e.AH.csr.va,
            e.AH.sell ? (const void*)e.AH.sl.ci : (const void*)e.AH.csr.ci,
            e.AH.sell ? (const void*)e.AH.sl.row : (const void*)e.AH.csr.rp,
            e.ctl, e.part, key_extra};
        uint64_t key = fnv(&k, sizeof(k));
        for (auto& g : c->graphs)
            if (g.key == key) exec = g.exec;
        if (!exec) {
            hipGraph_t graph;
            SKR_HIP(hipStreamBeginCapture(e.st, hipStreamCaptureModeRelaxed));
            try {
                for (int i = 0; i < every; ++i) m.iter();
            } catch (...) {
                hipGraph_t g2;
                (void)hipStreamEndCapture(e.st, &g2);
                throw;
            }
            SKR_HIP(hipStreamEndCapture(e.st, &graph));
            SKR_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
            (void)hipGraphDestroy(graph);
            c->graphs.push_back(GraphEntry{key, exec});
        }
    }
    long long launched = 0;
    const long long cap = (long long)maxit + 2LL * every + 2;
    for (;;) {
        if (exec) {
            SKR_HIP(hipGraphLaunch(exec, e.st));
        } else {
            for (int i = 0; i < every; ++i) m.iter();
        }
        launched += every;
        SKR_HIP(hipMemcpyAsync(c->hout, e.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, e.st));
        SKR_HIP(hipStreamSynchronize(e.st));
        if (c->hout->done || launched > cap) break;
    }
    return inner_stats(c, e, m.mv_per_iter);
}

// Dynamic LDS of the single-workgroup kernels: P (n x s), then P^ (n x s) or
// p^ (n) for Gl-BiCG / eGl-BiCG; one n x s block (P, then S) for Gl-BiCGStab.
template <class T>
size_t small_lds_bytes(int n, int s, int method) {
    const size_t blk = (size_t)n * s;
    if (method == SKR_GL_BICGSTAB) return sizeof(T) * blk;
    return sizeof(T) * (blk + (method == SKR_EGL_BICG ? (size_t)n : blk));
}

// A system the single-workgroup kernels take: Gl-BiCG, eGl-BiCG or
// Gl-BiCGStab, CSR operands, no preconditioner, n <= 1024 rows, s within the
// register budget and the LDS blocks within one workgroup's LDS (with 1 KiB left
// for the kernels' reduction slots).
template <class T>
bool small_eligible(const skr_context* c, const Env<T>& e, int method, const skr_opts& o) {
    if (!o.fused_small || (method != SKR_GL_BICG && method != SKR_EGL_BICG && method != SKR_GL_BICGSTAB))
        return false;
    if (e.n < 1 || e.n > kSmallMaxRows || e.s > SmallMaxS<T>::value || e.A.sell || e.AH.sell || e.pc) return false;
    return small_lds_bytes<T>(e.n, e.s, method) + 1024 <= (size_t)c->lds_max;
}

template <class T, int S>
void launch_small(Env<T>& e, int method, size_t lds, const T* rhs, T* D) {
    const bool econ = method == SKR_EGL_BICG;
    if (method == SKR_GL_BICGSTAB) {
        SKR_HIP(hipFuncSetAttribute((const void*)k_small_bicgstab<T, S>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lds));
        k_small_bicgstab<T, S><<<1, kSmallThreads, lds, e.st>>>(e.ctl, e.hist, e.A.csr, rhs, D);
    } else if (econ) {
        SKR_HIP(hipFuncSetAttribute((const void*)k_small_bicg<T, true, S>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        k_small_bicg<T, true, S><<<1, kSmallThreads, lds, e.st>>>(e.ctl, e.hist, e.A.csr, e.AH.csr, rhs, D);
    } else {
        SKR_HIP(hipFuncSetAttribute((const void*)k_small_bicg<T, false, S>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        k_small_bicg<T, false, S><<<1, kSmallThreads, lds, e.st>>>(e.ctl, e.hist, e.A.csr, e.AH.csr, rhs, D);
    }
}

// Enqueue Gl-BiCG, eGl-BiCG or Gl-BiCGStab on A D = rhs as one launch (every
// iteration inside one workgroup; same stopping rule, breakdown rules and
// history as iterate), then the copy of the stop state to c->hout.  The caller
// synchronises and reads the result with inner_stats.
template <class T>
void enqueue_small(skr_context* c, Env<T>& e, int method, double tol, int maxit, const T* rhs, T* D) {
    Ctl* h = c->hin;
    std::memset(h, 0, sizeof(Ctl));
    h->status = ST_RUNNING;
    h->bd_iter = -1;
    h->maxit = maxit;
    h->tol = tol;
    SKR_HIP(hipMemcpyAsync(e.ctl, h, sizeof(Ctl), hipMemcpyHostToDevice, e.st));
    const size_t lds = small_lds_bytes<T>(e.n, e.s, method);
    if constexpr (Tr<T>::cplx) {
        switch (e.s) {
            case 1: launch_small<T, 1>(e, method, lds, rhs, D); break;
            case 2: launch_small<T, 2>(e, method, lds, rhs, D); break;
            default: throw Unsupported{"single-workgroup path: block too wide"};
        }
    } else {
        switch (e.s) {
            case 1: launch_small<T, 1>(e, method, lds, rhs, D); break;
            case 2: launch_small<T, 2>(e, method, lds, rhs, D); break;
            case 3: launch_small<T, 3>(e, method, lds, rhs, D); break;
            case 4: launch_small<T, 4>(e, method, lds, rhs, D); break;
            default: throw Unsupported{"single-workgroup path: block too wide"};
        }
    }
    SKR_LAUNCHED();
    SKR_HIP(hipMemcpyAsync(c->hout, e.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, e.st));
}

// True residual: part = (||B - A X||^2, ||B||^2) -> c->hsum[0..1].x; with
// sync = false only enqueued (the caller synchronises before reading).
template <class T>
void true_residual(skr_context* c, Env<T>& e, const T* B, const T* X, T* tmp, double* rn2, double* bn2,
                   bool sync = true) {
    spmm(e, e.A, e.ly, X, tmp, EpiNone{}, (const Ctl*)nullptr);
    k_resid<T, T><<<e.nb, kBlock, 0, e.st>>>(e.fl, B, tmp, (T*)nullptr, (T*)nullptr, e.part);
    k_sum2<<<1, kScalar, 0, e.st>>>(e.part, e.nb, e.sc + 100);
    SKR_LAUNCHED();
    SKR_HIP(hipMemcpyAsync(c->hsum, e.sc + 100, 2 * sizeof(c64), hipMemcpyDeviceToHost, e.st));
    if (!sync) return;
    SKR_HIP(hipStreamSynchronize(e.st));
    *rn2 = c->hsum[0].x;
    *bn2 = c->hsum[1].x;
}

// Pinned host room for n history entries (grow-only; null when n is beyond
// the cap below, and then the history is read with a blocking copy).
inline double* host_history(skr_context* c, size_t n) {
    constexpr size_t kCap = size_t(1) << 16;   // 512 KB
    if (n > kCap) return nullptr;
    if (n > c->hhist_cap) {
        if (c->hhist) {
            SKR_HIP(hipStreamSynchronize(c->stream()));
            (void)hipHostFree(c->hhist);
            c->hhist = nullptr;
            c->hhist_cap = 0;
        }
        const size_t want = std::max<size_t>(n, 4096);
        SKR_HIP(hipHostMalloc((void**)&c->hhist, sizeof(double) * want, hipHostMallocDefault));
        c->hhist_cap = want;
    }
    return c->hhist;
}

template <class T, int S>
void launch_small_qr(Env<T>& e, T* rhs) {
    k_small_qr<T, S><<<1, kSmallThreads, 0, e.st>>>(e.ctl, e.n, rhs, e.mats, 0x1p-53);
}

// Preprocess rhs in place: rhs = Q with rhs = Q R_R (R_R -> mats M_RB).  Returns
// false if the QR broke down.  small: the system takes the single-workgroup
// path (n <= 1024, s within its limit), and the QR runs as one launch too.
template <class T, int J>
bool preprocess(skr_context* c, Env<T>& e, T* rhs, bool small = false) {
    Ctl* h = c->hin;
    std::memset(h, 0, sizeof(Ctl));
    h->status = ST_RUNNING;
    h->bd_iter = -1;
    SKR_HIP(hipMemcpyAsync(e.ctl, h, sizeof(Ctl), hipMemcpyHostToDevice, e.st));
    if (small) {
        if constexpr (!std::is_same<typename Tr<T>::R, double>::value) {
            throw Unsupported{"single-workgroup path: FP64 only"};
        } else if constexpr (Tr<T>::cplx) {
            switch (e.s) {
                case 1: launch_small_qr<T, 1>(e, rhs); break;
                case 2: launch_small_qr<T, 2>(e, rhs); break;
                default: throw Unsupported{"single-workgroup path: block too wide"};
            }
        } else {
            switch (e.s) {
                case 1: launch_small_qr<T, 1>(e, rhs); break;
                case 2: launch_small_qr<T, 2>(e, rhs); break;
                case 3: launch_small_qr<T, 3>(e, rhs); break;
                case 4: launch_small_qr<T, 4>(e, rhs); break;
                default: throw Unsupported{"single-workgroup path: block too wide"};
            }
        }
    } else {
        k_bl_gram<T, J><<<e.nb, kBlock, 0, e.st>>>(e.ctl, e.tl, rhs, rhs, e.part);
        SKR_LAUNCHED();
        cholqr<T, J>(e, 0, rhs, rhs, 0, nullptr);
        k_copy_mat<<<1, kScalar, 0, e.st>>>(e.mats, e.s, M_S, M_RB);
    }
    SKR_LAUNCHED();
    SKR_HIP(hipMemcpyAsync(c->hout, e.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, e.st));
    SKR_HIP(hipStreamSynchronize(e.st));
    return c->hout->done == 0;
}

template <class T>
struct Lower;
template <>
struct Lower<double> { using type = float; };
template <>
struct Lower<c64> { using type = c32; };

// ---------------------------------------------------------------- FP64 solve
template <class T, int J>
int solve_fp64(skr_context* c, const skr_matrix* M, int s, const T* B, T* X, bool x0zero, int method,
               const skr_opts& o, int adjoint, skr_result* res) {
    Env<T> e;
    env_layout(e, M->n, s);
    e.st = c->stream();
    e.A = operand<T>(M, adjoint != 0, false);
    e.AH = operand<T>(M, adjoint == 0, false);
    if (o.precond == SKR_PRECOND_ILU0) {
        if (!M->ilu) throw Unsupported{"ILU(0) preconditioning requested: call skr_matrix_ilu0 first"};
        if (adjoint) throw Unsupported{"ILU(0) preconditioning of adjoint solves is not available"};
        e.pc = M->ilu;
    }
    auto carve = [&](Arena& ar, T** rhs, T** D, T** tmp, Method<T>* m) {
        take_common(e, ar, o.maxit);
        *rhs = (T*)ar.take(e.blk_bytes());
        *D = (T*)ar.take(e.blk_bytes());
        *tmp = (T*)ar.take(e.blk_bytes());
        if (e.pc) e.pc_tmp = (T*)ar.take(e.blk_bytes());
        *m = make_method<T, J>(method, e, ar, *rhs, *D);
    };
    T *rhs, *D, *tmp;
    Method<T> m;
    Arena sz;
    carve(sz, &rhs, &D, &tmp, &m);
    ensure_arena(c, sz.off);
    Arena ar;
    ar.base = c->arena;
    ar.cap = c->arena_cap;
    carve(ar, &rhs, &D, &tmp, &m);

    // R0 = B - A X0
    if (x0zero) {
        k_fill0<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, X, nullptr, nullptr, nullptr);
        k_copy<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, B, rhs, nullptr, nullptr);
    } else {
        spmm(e, e.A, e.ly, X, tmp, EpiNone{}, (const Ctl*)nullptr);
        k_resid<T, T><<<e.nb, kBlock, 0, e.st>>>(e.fl, B, tmp, rhs, (T*)nullptr, e.part);
    }
    SKR_LAUNCHED();
    bool pre = o.preprocess_qr != 0;
    const bool small = small_eligible<T>(c, e, method, o);
    if (pre && !preprocess<T, J>(c, e, rhs, small)) {
        res->status = SKR_BREAKDOWN;
        res->iterations = 0;
        res->breakdown_iter = 0;
        return SKR_BREAKDOWN;
    }
    e.pc_on = e.pc != nullptr;
    InnerStats st;
    double rn2, bn2;
    if (small) {
        // one launch, then X = X0 + D R_R, the true residual and the history
        // copy, all enqueued behind it, and one synchronisation for the lot
        enqueue_small<T>(c, e, method, o.tol, o.maxit, rhs, D);
        k_xupd<T, T, J><<<e.nb, kBlock, mat_lds(s, 1, 1), e.st>>>(e.tl, e.mats, pre ? M_RB : -1, X, D, 0);
        SKR_LAUNCHED();
        true_residual<T>(c, e, B, X, tmp, &rn2, &bn2, false);
        double* hh = host_history(c, (size_t)o.maxit + 1);
        if (hh) SKR_HIP(hipMemcpyAsync(hh, e.hist, sizeof(double) * ((size_t)o.maxit + 1), hipMemcpyDeviceToHost, e.st));
        SKR_HIP(hipStreamSynchronize(e.st));
        rn2 = c->hsum[0].x;
        bn2 = c->hsum[1].x;
        st = inner_stats(c, e, method == SKR_EGL_BICG ? (long long)e.s + 1 : 2LL * e.s, hh);
    } else {
        st = iterate<T>(c, e, m, method, o.tol, o.maxit, o.check_every, o.use_graph != 0,
                        fnv(&e.pc, sizeof(e.pc), fnv(&ar, sizeof(ar), 0)));
        e.pc_on = false;
        if (e.pc) {   // the method solved A M^-1 D = Q: the correction is M^-1 D
            prec_apply(e, s, D, e.pc_tmp, false, nullptr);
            D = e.pc_tmp;
        }
        // X = X0 + D R_R  (or X0 + D)
        k_xupd<T, T, J><<<e.nb, kBlock, mat_lds(s, 1, 1), e.st>>>(e.tl, e.mats, pre ? M_RB : -1, X, D, 0);
        SKR_LAUNCHED();
        true_residual<T>(c, e, B, X, tmp, &rn2, &bn2);
    }
    res->single_workgroup = small ? 1 : 0;
    e.pc_on = false;
    double rel = bn2 > 0 ? std::sqrt(rn2 / bn2) : 0.0;
    res->status = st.status;
    if (st.status != SKR_BREAKDOWN && rel > 1.0) res->status = SKR_DIVERGED;
    res->iterations = st.iters;
    res->matvecs = st.matvecs;
    res->outer_iterations = 0;
    res->fp64_outer_iterations = 0;
    res->breakdown_iter = st.bd_iter;
    res->rel_res_recursive = st.rres;
    res->rel_res_true = rel;
    if (res->history && res->history_cap > 0) {
        int len = std::min<int>(res->history_cap, (int)st.hist.size());
        std::memcpy(res->history, st.hist.data(), sizeof(double) * len);
        res->history_len = len;
    } else {
        res->history_len = 0;
    }
    return res->status;
}

// ---------------------------------------------------------------- FP32 inner + FP64 refinement
template <class T, int J>
int solve_mixed(skr_context* c, skr_matrix* M, int s, const T* B, T* X, bool x0zero, int method,
                const skr_opts& o, int adjoint, skr_result* res) {
    using L = typename Lower<T>::type;
    ensure_fp32(M, c->stream());
    Env<T> e;
    env_layout(e, M->n, s);
    e.st = c->stream();
    e.A = operand<T>(M, adjoint != 0, false);
    e.AH = operand<T>(M, adjoint == 0, false);
    Env<L> f;
    env_layout(f, M->n, s);
    f.st = c->stream();
    f.A = operand<L>(M, adjoint != 0, true);
    f.AH = operand<L>(M, adjoint == 0, true);
    // FP32 method on (r32, d32); the same method in FP64 on (r64, d64) runs an
    // outer step whose FP32 inner solve made no progress.
    auto carve = [&](Arena& ar, T** tmp, L** r32, L** d32, Method<L>* m, T** r64, T** d64, Method<T>* m64) {
        take_common(e, ar, o.maxit);
        take_common(f, ar, o.maxit);
        *tmp = (T*)ar.take(e.blk_bytes());
        *r32 = (L*)ar.take(f.blk_bytes());
        *d32 = (L*)ar.take(f.blk_bytes());
        *m = make_method<L, J>(method, f, ar, *r32, *d32);
        *r64 = (T*)ar.take(e.blk_bytes());
        *d64 = (T*)ar.take(e.blk_bytes());
        *m64 = make_method<T, J>(method, e, ar, *r64, *d64);
    };
    T *tmp, *r64, *d64;
    L *r32, *d32;
    Method<L> m;
    Method<T> m64;
    Arena sz;
    carve(sz, &tmp, &r32, &d32, &m, &r64, &d64, &m64);
    ensure_arena(c, sz.off);
    Arena ar;
    ar.base = c->arena;
    ar.cap = c->arena_cap;
    carve(ar, &tmp, &r32, &d32, &m, &r64, &d64, &m64);

    if (x0zero) {
        k_fill0<T><<<e.nb, kBlock, 0, e.st>>>(e.fl, X, nullptr, nullptr, nullptr);
        SKR_LAUNCHED();
    }
    std::vector<double> hist;
    int iters = 0, outer = 0, status = SKR_NOT_CONVERGED, bd = -1, outer64 = 0;
    long long mv = 0;
    double rel = 0.0, rres = 0.0, prev_rel = -1.0;
    bool use64 = false;   // once an FP32 step fails to halve the true residual, stay in FP64
    const bool pre = o.preprocess_qr != 0;
    for (;;) {
        spmm(e, e.A, e.ly, X, tmp, EpiNone{}, (const Ctl*)nullptr);
        k_resid<T, L><<<e.nb, kBlock, 0, e.st>>>(e.fl, B, tmp, (T*)nullptr, r32, e.part);
        k_sum2<<<1, kScalar, 0, e.st>>>(e.part, e.nb, e.sc + 100);
        SKR_LAUNCHED();
        SKR_HIP(hipMemcpyAsync(c->hsum, e.sc + 100, 2 * sizeof(c64), hipMemcpyDeviceToHost, e.st));
        SKR_HIP(hipStreamSynchronize(e.st));
        double rn = std::sqrt(c->hsum[0].x), bn = std::sqrt(c->hsum[1].x);
        rel = bn > 0 ? rn / bn : 0.0;
        hist.push_back(rel);
        if (rel <= o.tol || !(bn > 0)) {
            status = SKR_OK;
            break;
        }
        if (!std::isfinite(rel)) {
            status = SKR_BREAKDOWN;
            break;
        }
        if (outer >= o.max_outer) {
            status = SKR_NOT_CONVERGED;
            break;
        }
        if (prev_rel > 0.0 && !(rel < 0.5 * prev_rel)) use64 = true;
        prev_rel = rel;
        ++outer;
        // inner target: inner_tol, relaxed on the last step to what is still
        // needed (half of tol / current relative residual), never above 0.5
        const double inner = std::max(o.inner_tol, std::min(0.5, 0.5 * o.tol / rel));
        mv += s;  // the outer residual product
        if (!use64 && (!pre || preprocess<L, J>(c, f, r32))) {
            // an FP32 inner solve whose residual grows 1e4-fold is abandoned early
            InnerStats st = iterate<L>(c, f, m, method, inner, o.maxit, o.check_every, o.use_graph != 0,
                                       fnv(&ar, sizeof(ar), 1), 1e4);
            iters += st.iters;
            mv += st.matvecs;
            rres = st.rres;
            if (st.rres < 1.0 && std::isfinite(st.rres)) {
                k_xupd<T, L, J><<<e.nb, kBlock, mat_lds(s, 1, 1), e.st>>>(e.tl, f.mats, pre ? M_RB : -1, X, d32, 0);
                SKR_LAUNCHED();
                continue;
            }
        }
        // This step in FP64: the FP32 QR of the residual or the FP32 inner solve
        // failed (X is unchanged and tmp still holds A X), or FP32 steps stopped
        // paying off.
        ++outer64;
        k_resid<T, T><<<e.nb, kBlock, 0, e.st>>>(e.fl, B, tmp, r64, (T*)nullptr, e.part);
        SKR_LAUNCHED();
        if (pre && !preprocess<T, J>(c, e, r64)) {
            status = SKR_BREAKDOWN;
            bd = iters;
            break;
        }
        InnerStats s64 = iterate<T>(c, e, m64, method, inner, o.maxit, o.check_every, o.use_graph != 0,
                                    fnv(&ar, sizeof(ar), 2));
        iters += s64.iters;
        mv += s64.matvecs;
        rres = s64.rres;
        if (!(s64.rres < 1.0) || !std::isfinite(s64.rres)) {
            status = SKR_BREAKDOWN;   // no progress in FP64 either: keep X and stop
            bd = iters;
            break;
        }
        k_xupd<T, T, J><<<e.nb, kBlock, mat_lds(s, 1, 1), e.st>>>(e.tl, e.mats, pre ? M_RB : -1, X, d64, 0);
        SKR_LAUNCHED();
    }
    res->status = status;
    if (status != SKR_BREAKDOWN && rel > 1.0) res->status = SKR_DIVERGED;
    res->iterations = iters;
    res->matvecs = mv;
    res->outer_iterations = outer;
    res->fp64_outer_iterations = outer64;
    res->breakdown_iter = bd;
    res->rel_res_recursive = rres;
    res->rel_res_true = rel;
    if (res->history && res->history_cap > 0) {
        int len = std::min<int>(res->history_cap, (int)hist.size());
        std::memcpy(res->history, hist.data(), sizeof(double) * len);
        res->history_len = len;
    } else {
        res->history_len = 0;
    }
    return res->status;
}

bool finite_block(skr_context* c, const void* P, int n, int w) {
    Env<double> e;
    env_layout(e, n, w);
    e.st = c->stream();
    Arena sz;
    take_common(e, sz, 1);
    ensure_arena(c, sz.off);
    Arena ar;
    ar.base = c->arena;
    take_common(e, ar, 1);
    k_flat_nrm_dot<double><<<e.nb, kBlock, 0, e.st>>>(e.fl, (const double*)P, nullptr, e.part);
    k_sum2<<<1, kScalar, 0, e.st>>>(e.part, e.nb, e.sc + 100);
    SKR_LAUNCHED();
    SKR_HIP(hipMemcpyAsync(c->hsum, e.sc + 100, 2 * sizeof(c64), hipMemcpyDeviceToHost, e.st));
    SKR_HIP(hipStreamSynchronize(e.st));
    return std::isfinite(c->hsum[0].x);
}

template <class T>
int solve_dispatch(skr_context* c, skr_matrix* M, int s, const T* B, T* X, bool x0zero, int method,
                   const skr_opts& o, int adjoint, skr_result* res) {
    const bool mixed = o.precision == SKR_PREC_FP32_REFINE;
    if (mixed && o.precond != SKR_PRECOND_NONE)
        throw Unsupported{"ILU(0) preconditioning is available for FP64 solves only"};
    if (s <= 16) {
        return mixed ? solve_mixed<T, 1>(c, M, s, B, X, x0zero, method, o, adjoint, res)
                     : solve_fp64<T, 1>(c, M, s, B, X, x0zero, method, o, adjoint, res);
    }
    return mixed ? solve_mixed<T, 2>(c, M, s, B, X, x0zero, method, o, adjoint, res)
                 : solve_fp64<T, 2>(c, M, s, B, X, x0zero, method, o, adjoint, res);
}

int fail(skr_context* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

template <class F>
int guarded(skr_context* c, F&& f) {
    try {
        return f();
    } catch (const HipError& h) {
        return fail(c, SKR_E_HIP, std::string("HIP error in ") + h.what + ": " + hipGetErrorString(h.e));
    } catch (const std::bad_alloc&) {
        return fail(c, SKR_E_ALLOC, "device or host memory allocation failed");
    } catch (const Unsupported& u) {
        return fail(c, SKR_E_UNSUPPORTED, u.what);
    } catch (const IluError& u) {
        return fail(c, SKR_E_INVALID, u.what);
    } catch (...) {
        return fail(c, SKR_E_INVALID, "unexpected error");
    }
}

}  // namespace

// ============================================================== C ABI
extern "C" {

void skr_opts_default(skr_opts* o) {
    if (!o) return;
    o->tol = 1e-8;
    o->maxit = 10000;
    o->precision = SKR_PREC_FP64;
    o->inner_tol = 1e-4;
    o->max_outer = 10;
    o->preprocess_qr = 1;
    o->zero_x0 = 1;
    o->precond = SKR_PRECOND_NONE;
    o->check_every = 16;
    o->use_graph = 1;
    o->fused_small = 1;
}

int skr_context_create(int device, void* hip_stream, skr_context** out) {
    if (!out) return SKR_E_INVALID;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return SKR_E_INVALID;
    if (hipSetDevice(device) != hipSuccess) return SKR_E_HIP;
    skr_context* c = new (std::nothrow) skr_context();
    if (!c) return SKR_E_ALLOC;
    c->device = device;
    c->user = (hipStream_t)hip_stream;
    if (hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking) != hipSuccess ||
        hipHostMalloc((void**)&c->hin, sizeof(Ctl), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->hout, sizeof(Ctl), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->hsum, 4 * sizeof(c64), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->hmat, sizeof(c64) * kMaxS * kMaxS, hipHostMallocDefault) != hipSuccess) {
        if (c->hin) (void)hipHostFree(c->hin);
        if (c->hout) (void)hipHostFree(c->hout);
        if (c->hsum) (void)hipHostFree(c->hsum);
        if (c->hmat) (void)hipHostFree(c->hmat);
        if (c->own) (void)hipStreamDestroy(c->own);
        delete c;
        return SKR_E_HIP;
    }
    // the allocation-free entry point's scratch on this device (once per device;
    // a failed lookup only disables that entry point, which then reports it)
    if (hipDeviceGetAttribute(&c->lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess)
        c->lds_max = 0;   // the single-workgroup small-system path stays off
    std::string why;
    c->scratch = scratch_addr(device, &why);
    if (!c->scratch) c->err = why;
    *out = c;
    return SKR_OK;
}

int skr_context_destroy(skr_context* c) {
    if (!c) return SKR_E_INVALID;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream());
    invalidate_graphs(c);
    for (skr_matrix* M : c->mats) M->ctx = nullptr;
    if (c->arena) (void)hipFree(c->arena);
    if (c->stage) (void)hipFree(c->stage);
    if (c->hin) (void)hipHostFree(c->hin);
    if (c->hout) (void)hipHostFree(c->hout);
    if (c->hsum) (void)hipHostFree(c->hsum);
    if (c->hmat) (void)hipHostFree(c->hmat);
    if (c->hhist) (void)hipHostFree(c->hhist);
    if (c->own) (void)hipStreamDestroy(c->own);
    delete c;
    return SKR_OK;
}

int skr_context_set_stream(skr_context* c, void* hip_stream) {
    if (!c) return SKR_E_INVALID;
    if ((hipStream_t)hip_stream != c->user) invalidate_graphs(c);
    c->user = (hipStream_t)hip_stream;
    return SKR_OK;
}

const char* skr_last_error(skr_context* c) { return c ? c->err.c_str() : "null context"; }

int skr_matrix_create(skr_context* c, int64_t n64, int64_t nnz64, const int64_t* row_ptr, const int32_t* col_idx,
                      const void* values, int32_t dtype, int32_t mem, const skr_format_opts* fmt, skr_matrix** out) {
    if (!c || !out) return SKR_E_INVALID;
    *out = nullptr;
    // the kernels' row sweeps step int row indices up to one grid stride past n
    if (n64 < 1 || n64 > kMaxRows || nnz64 < 0 || nnz64 >= (1LL << 31))
        return fail(c, SKR_E_INVALID, "n must be in [1, 2^31 - 2^20] and nnz in [0, 2^31)");
    if (dtype != SKR_F64 && dtype != SKR_C64) return fail(c, SKR_E_INVALID, "dtype must be SKR_F64 or SKR_C64");
    if (mem != SKR_MEM_HOST && mem != SKR_MEM_DEVICE) return fail(c, SKR_E_INVALID, "bad mem");
    if (!row_ptr || (nnz64 > 0 && (!col_idx || !values))) return fail(c, SKR_E_INVALID, "null array");
    int C = 32, sigma = 256, fmtk = SKR_FMT_CSR, mk32 = 0;
    if (fmt) {
        fmtk = fmt->format;
        C = fmt->sell_C;
        sigma = fmt->sell_sigma;
        mk32 = fmt->make_fp32;
        if (fmtk != SKR_FMT_CSR && fmtk != SKR_FMT_SELL) return fail(c, SKR_E_INVALID, "bad format");
        if (fmtk == SKR_FMT_SELL && ((C != 16 && C != 32 && C != 64) || sigma < C || sigma % C != 0))
            return fail(c, SKR_E_INVALID, "SELL needs C in {16,32,64} and sigma a positive multiple of C");
    }
    return guarded(c, [&]() -> int {
        SKR_HIP(hipSetDevice(c->device));
        const int n = (int)n64, nnz = (int)nnz64;
        std::vector<int64_t> rp64(n + 1);
        std::vector<int> ci(nnz);
        if (mem == SKR_MEM_HOST) {
            std::memcpy(rp64.data(), row_ptr, sizeof(int64_t) * (n + 1));
            if (nnz) std::memcpy(ci.data(), col_idx, sizeof(int) * nnz);
        } else {
            SKR_HIP(hipMemcpy(rp64.data(), row_ptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost));
            if (nnz) SKR_HIP(hipMemcpy(ci.data(), col_idx, sizeof(int) * nnz, hipMemcpyDeviceToHost));
        }
        std::vector<int> rp;
        if (const char* why = validate_csr(n, nnz64, rp64, ci, rp)) return fail(c, SKR_E_INVALID, why);
        std::vector<int> rpH, ciH, perm;
        adjoint_pattern(n, rp, ci, rpH, ciH, perm);
        std::unique_ptr<skr_matrix> M(new skr_matrix());
        M->ctx = c;
        M->device = c->device;
        M->n = n;
        M->nnz = nnz;
        M->dtype = dtype;
        const size_t es = elt(dtype, false);
        M->rp = (int*)dmalloc<int>(n + 1);
        M->ci = (int*)dmalloc<int>(nnz);
        M->rpH = (int*)dmalloc<int>(n + 1);
        M->ciH = (int*)dmalloc<int>(nnz);
        M->perm = (int*)dmalloc<int>(nnz);
        SKR_HIP(hipMalloc(&M->va, es * std::max<size_t>(1, nnz)));   // at least one element
        SKR_HIP(hipMalloc(&M->vaH, es * std::max<size_t>(1, nnz)));
        SKR_HIP(hipMemcpy(M->rp, rp.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice));
        SKR_HIP(hipMemcpy(M->rpH, rpH.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice));
        if (nnz == 0) {
            // the sparse kernels read a clamped entry even for empty rows: keep one
            // valid (column 0, value 0) slot
            SKR_HIP(hipMemset(M->ci, 0, sizeof(int)));
            SKR_HIP(hipMemset(M->ciH, 0, sizeof(int)));
            SKR_HIP(hipMemset(M->perm, 0, sizeof(int)));
            SKR_HIP(hipMemset(M->va, 0, es));
            SKR_HIP(hipMemset(M->vaH, 0, es));
        }
        if (nnz) {
            SKR_HIP(hipMemcpy(M->ci, ci.data(), sizeof(int) * nnz, hipMemcpyHostToDevice));
            SKR_HIP(hipMemcpy(M->ciH, ciH.data(), sizeof(int) * nnz, hipMemcpyHostToDevice));
            SKR_HIP(hipMemcpy(M->perm, perm.data(), sizeof(int) * nnz, hipMemcpyHostToDevice));
            SKR_HIP(hipMemcpy(M->va, values, es * nnz,
                              mem == SKR_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice));
        }
        if (fmtk == SKR_FMT_SELL) {
            M->sell = true;
            HostSell hs, hsh;
            if (!build_sell(n, rp, ci, C, sigma, hs) || !build_sell(n, rpH, ciH, C, sigma, hsh))
                throw Unsupported{"the SELL-C-sigma copy would need 2^31 or more stored slots; use CSR"};
            upload_sell(M->SA, hs, C, sigma, n);
            upload_sell(M->SAH, hsh, C, sigma, n);
            SKR_HIP(hipMalloc(&M->SA.va, es * std::max<size_t>(1, M->SA.slots)));
            SKR_HIP(hipMalloc(&M->SAH.va, es * std::max<size_t>(1, M->SAH.slots)));
            M->sell_pad = nnz ? (double)M->SA.slots / nnz : 0.0;
        }
        hipStream_t st = c->stream();
        refresh_values(M.get(), st);
        if (mk32) ensure_fp32(M.get(), st);
        SKR_HIP(hipStreamSynchronize(st));
        *out = M.release();
        c->mats.push_back(*out);
        return SKR_OK;
    });
}

int skr_matrix_update_values(skr_matrix* M, const void* values, int32_t mem) {
    if (!M || !values || !M->ctx) return SKR_E_INVALID;
    skr_context* c = M->ctx;
    if (mem != SKR_MEM_HOST && mem != SKR_MEM_DEVICE) return fail(c, SKR_E_INVALID, "bad mem");
    return guarded(c, [&]() -> int {
        SKR_HIP(hipSetDevice(c->device));
        size_t es = elt(M->dtype, false);
        if (M->nnz)
            SKR_HIP(hipMemcpyAsync(M->va, values, es * M->nnz,
                                   mem == SKR_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                                   c->stream()));
        refresh_values(M, c->stream());
        SKR_HIP(hipStreamSynchronize(c->stream()));
        if (M->ilu) {   // the factors belong to the old values
            invalidate_graphs(c);
            free_ilu(M);
        }
        return SKR_OK;
    });
}

int skr_matrix_destroy(skr_matrix* M) {
    if (!M) return SKR_E_INVALID;
    skr_context* c = M->ctx;
    (void)hipSetDevice(M->device);
    if (c) {
        (void)hipStreamSynchronize(c->stream());
        invalidate_graphs(c);
        c->mats.erase(std::remove(c->mats.begin(), c->mats.end(), M), c->mats.end());
    } else {
        (void)hipDeviceSynchronize();
    }
    void* ps[] = {M->rp, M->ci, M->va, M->va32, M->rpH, M->ciH, M->perm, M->vaH, M->vaH32};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    if (M->sell) {
        free_sell(M->SA);
        free_sell(M->SAH);
    }
    free_ilu(M);
    delete M;
    return SKR_OK;
}

double skr_matrix_sell_padding(const skr_matrix* M) { return M ? M->sell_pad : 0.0; }

int skr_solve(skr_context* c, const skr_matrix* Mc, int32_t s, const void* B, int64_t ldb, void* X, int64_t ldx,
              int32_t mem, int32_t method, const skr_opts* opts, int32_t adjoint, skr_result* res) {
    if (!c) return SKR_E_INVALID;
    if (!Mc || !B || !X || !res) return fail(c, SKR_E_INVALID, "null argument");
    if (Mc->ctx != c) return fail(c, SKR_E_INVALID, "matrix belongs to another (or a destroyed) context");
    skr_matrix* M = const_cast<skr_matrix*>(Mc);
    if (s < 1 || s > kMaxS) return fail(c, SKR_E_INVALID, "s must be in [1, 32]");
    if (ldb < s || ldx < s) return fail(c, SKR_E_INVALID, "leading dimensions must be >= s");
    if (method < SKR_GL_BICG || method > SKR_LI_QMR) return fail(c, SKR_E_INVALID, "unknown method");
    if (mem != SKR_MEM_HOST && mem != SKR_MEM_DEVICE) return fail(c, SKR_E_INVALID, "bad mem");
    skr_opts o;
    skr_opts_default(&o);
    if (opts) o = *opts;
    if (!(o.tol >= 0.0) || o.maxit < 0 || o.max_outer < 0 || !(o.inner_tol > 0.0) || o.check_every < 1)
        return fail(c, SKR_E_INVALID, "bad options");
    if (o.precision != SKR_PREC_FP64 && o.precision != SKR_PREC_FP32_REFINE)
        return fail(c, SKR_E_INVALID, "bad precision");
    if (o.precond != SKR_PRECOND_NONE && o.precond != SKR_PRECOND_ILU0)
        return fail(c, SKR_E_INVALID, "bad precond");
    double* hist = res->history;
    int cap = res->history_cap;
    std::memset(res, 0, sizeof(*res));
    res->history = hist;
    res->history_cap = cap;
    res->breakdown_iter = -1;
    return guarded(c, [&]() -> int {
        SKR_HIP(hipSetDevice(c->device));
        const int n = M->n;
        const size_t es = elt(M->dtype, false);
        const size_t bytes = (size_t)n * s * es;
        hipStream_t st = c->stream();
        // stage B and X into contiguous device blocks
        const size_t half = (std::max<size_t>(bytes, 1) + 255) & ~size_t(255);
        if (c->stage_cap < 2 * half) {
            SKR_HIP(hipStreamSynchronize(st));
            if (c->stage) (void)hipFree(c->stage);
            c->stage = nullptr;
            c->stage_cap = 0;
            SKR_HIP(hipMalloc(&c->stage, 2 * half));
            c->stage_cap = 2 * half;
        }
        void* Bd = c->stage;
        void* Xd = (char*)c->stage + half;
        auto stage_in = [&](const void* src, int64_t ld, void* dst) {
            if (mem == SKR_MEM_HOST) {
                SKR_HIP(hipMemcpy2DAsync(dst, s * es, src, ld * es, s * es, n, hipMemcpyHostToDevice, st));
            } else {
                SKR_HIP(hipMemcpy2DAsync(dst, s * es, src, ld * es, s * es, n, hipMemcpyDeviceToDevice, st));
            }
        };
        stage_in(B, ldb, Bd);
        bool x0zero = o.zero_x0 != 0;
        if (!x0zero) stage_in(X, ldx, Xd);
        // reject NaN / Inf in B (and in X0)
        if (!finite_block(c, Bd, n, s * (int)(es / 8)) || (!x0zero && !finite_block(c, Xd, n, s * (int)(es / 8))))
            return fail(c, SKR_E_INVALID, "B or X0 contains NaN or Inf");
        int rc;
        if (M->dtype == SKR_C64)
            rc = solve_dispatch<c64>(c, M, s, (const c64*)Bd, (c64*)Xd, x0zero, method, o, adjoint, res);
        else
            rc = solve_dispatch<double>(c, M, s, (const double*)Bd, (double*)Xd, x0zero, method, o, adjoint, res);
        if (rc < 0) return rc;
        if (mem == SKR_MEM_HOST) {
            SKR_HIP(hipMemcpy2DAsync(X, ldx * es, Xd, s * es, s * es, n, hipMemcpyDeviceToHost, st));
        } else {
            SKR_HIP(hipMemcpy2DAsync(X, ldx * es, Xd, s * es, s * es, n, hipMemcpyDeviceToDevice, st));
        }
        SKR_HIP(hipStreamSynchronize(st));
        if (!std::isfinite(res->rel_res_true) && res->status == SKR_OK) res->status = SKR_BREAKDOWN;
        return res->status;
    });
}

int skr_spmm(skr_context* c, const skr_matrix* M, int32_t s, const void* X, int64_t ldx, void* Y, int64_t ldy,
             int32_t mem, int32_t adjoint) {
    if (!c) return SKR_E_INVALID;
    if (!M || !X || !Y) return fail(c, SKR_E_INVALID, "null argument");
    if (M->ctx != c) return fail(c, SKR_E_INVALID, "matrix belongs to another (or a destroyed) context");
    if (s < 1 || s > kMaxS || ldx < s || ldy < s) return fail(c, SKR_E_INVALID, "bad s or leading dimension");
    if (mem != SKR_MEM_HOST && mem != SKR_MEM_DEVICE) return fail(c, SKR_E_INVALID, "bad mem");
    return guarded(c, [&]() -> int {
        SKR_HIP(hipSetDevice(c->device));
        const int n = M->n;
        const size_t es = elt(M->dtype, false);
        const size_t bytes = (size_t)n * s * es;
        hipStream_t st = c->stream();
        const bool direct = mem == SKR_MEM_DEVICE && ldx == s && ldy == s;
        void *Xd = (void*)X, *Yd = Y;
        if (!direct) {
            SKR_HIP(hipMalloc(&Xd, std::max<size_t>(bytes, 1)));
            SKR_HIP(hipMalloc(&Yd, std::max<size_t>(bytes, 1)));
            SKR_HIP(hipMemcpy2DAsync(Xd, s * es, X, ldx * es, s * es, n,
                                     mem == SKR_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, st));
        }
        if (M->dtype == SKR_C64) {
            Env<c64> e;
            env_layout(e, n, s);
            e.st = st;
            Operand<c64> op = operand<c64>(M, adjoint != 0, false);
            spmm(e, op, e.ly, (const c64*)Xd, (c64*)Yd, EpiNone{}, (const Ctl*)nullptr);
        } else {
            Env<double> e;
            env_layout(e, n, s);
            e.st = st;
            Operand<double> op = operand<double>(M, adjoint != 0, false);
            spmm(e, op, e.ly, (const double*)Xd, (double*)Yd, EpiNone{}, (const Ctl*)nullptr);
        }
        if (!direct) {
            SKR_HIP(hipMemcpy2DAsync(Y, ldy * es, Yd, s * es, s * es, n,
                                     mem == SKR_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, st));
            SKR_HIP(hipStreamSynchronize(st));
            (void)hipFree(Xd);
            (void)hipFree(Yd);
        }
        return SKR_OK;
    });
}

int skr_matrix_ilu0(skr_context* c, skr_matrix* M) {
    if (!c) return SKR_E_INVALID;
    if (!M) return fail(c, SKR_E_INVALID, "null argument");
    if (M->ctx != c) return fail(c, SKR_E_INVALID, "matrix belongs to another (or a destroyed) context");
    return guarded(c, [&]() -> int {
        SKR_HIP(hipSetDevice(c->device));
        hipStream_t st = c->stream();
        SKR_HIP(hipStreamSynchronize(st));
        invalidate_graphs(c);
        free_ilu(M);
        if (M->dtype == SKR_C64) build_ilu<c64>(M, st);
        else build_ilu<double>(M, st);
        return SKR_OK;
    });
}

int skr_precond_apply(skr_context* c, const skr_matrix* M, int32_t s, const void* Z, int64_t ldz, void* Y,
                      int64_t ldy, int32_t mem, int32_t adjoint) {
    if (!c) return SKR_E_INVALID;
    if (!M || !Z || !Y) return fail(c, SKR_E_INVALID, "null argument");
    if (M->ctx != c) return fail(c, SKR_E_INVALID, "matrix belongs to another (or a destroyed) context");
    if (!M->ilu) return fail(c, SKR_E_INVALID, "no ILU(0) factors: call skr_matrix_ilu0 first");
    if (s < 1 || s > kMaxS || ldz < s || ldy < s) return fail(c, SKR_E_INVALID, "bad s or leading dimension");
    if (mem != SKR_MEM_HOST && mem != SKR_MEM_DEVICE) return fail(c, SKR_E_INVALID, "bad mem");
    return guarded(c, [&]() -> int {
        SKR_HIP(hipSetDevice(c->device));
        const int n = M->n;
        const size_t es = elt(M->dtype, false);
        const size_t bytes = (size_t)n * s * es;
        hipStream_t st = c->stream();
        const bool direct = mem == SKR_MEM_DEVICE && ldz == s && ldy == s;
        void *Zd = (void*)Z, *Yd = Y;
        if (!direct) {
            SKR_HIP(hipMalloc(&Zd, std::max<size_t>(bytes, 1)));
            SKR_HIP(hipMalloc(&Yd, std::max<size_t>(bytes, 1)));
            SKR_HIP(hipMemcpy2DAsync(Zd, s * es, Z, ldz * es, s * es, n,
                                     mem == SKR_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, st));
        }
        if (M->dtype == SKR_C64) {
            Env<c64> e;
            env_layout(e, n, s);
            e.st = st;
            e.pc = M->ilu;
            prec_apply(e, s, (const c64*)Zd, (c64*)Yd, adjoint != 0, nullptr);
        } else {
            Env<double> e;
            env_layout(e, n, s);
            e.st = st;
            e.pc = M->ilu;
            prec_apply(e, s, (const double*)Zd, (double*)Yd, adjoint != 0, nullptr);
        }
        if (!direct) {
            SKR_HIP(hipMemcpy2DAsync(Y, ldy * es, Yd, s * es, s * es, n,
                                     mem == SKR_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, st));
            SKR_HIP(hipStreamSynchronize(st));
            (void)hipFree(Zd);
            (void)hipFree(Yd);
        } else {
            SKR_HIP(hipStreamSynchronize(st));
        }
        return SKR_OK;
    });
}

int skr_sddmm(skr_context* c, const skr_matrix* M, int32_t s, const void* G, const void* X, void* out_vals,
              double scale, int32_t mem) {
    if (!c) return SKR_E_INVALID;
    if (!M || !G || !X || !out_vals) return fail(c, SKR_E_INVALID, "null argument");
    if (M->ctx != c) return fail(c, SKR_E_INVALID, "matrix belongs to another (or a destroyed) context");
    if (s < 1 || s > kMaxS) return fail(c, SKR_E_INVALID, "s must be in [1, 32]");
    if (mem != SKR_MEM_HOST && mem != SKR_MEM_DEVICE) return fail(c, SKR_E_INVALID, "bad mem");
    return guarded(c, [&]() -> int {
        SKR_HIP(hipSetDevice(c->device));
        const int n = M->n;
        const size_t es = elt(M->dtype, false);
        const size_t bytes = (size_t)n * s * es;
        hipStream_t st = c->stream();
        void *Gd = (void*)G, *Xd = (void*)X, *Od = out_vals;
        if (mem == SKR_MEM_HOST) {
            SKR_HIP(hipMalloc(&Gd, std::max<size_t>(bytes, 1)));
            SKR_HIP(hipMalloc(&Xd, std::max<size_t>(bytes, 1)));
            SKR_HIP(hipMalloc(&Od, std::max<size_t>(es * M->nnz, 1)));
            SKR_HIP(hipMemcpyAsync(Gd, G, bytes, hipMemcpyHostToDevice, st));
            SKR_HIP(hipMemcpyAsync(Xd, X, bytes, hipMemcpyHostToDevice, st));
        }
        auto launch = [&](auto tag) {
            using T = decltype(tag);
            Env<T> e;
            env_layout(e, n, s);
            if (e.J == 1)
                k_sddmm<T, 1><<<e.nb, kBlock, 0, st>>>(e.ly, n, e.rpc, M->rp, M->ci, (const T*)Gd, (const T*)Xd,
                                                      scale, (T*)Od);
            else
                k_sddmm<T, 2><<<e.nb, kBlock, 0, st>>>(e.ly, n, e.rpc, M->rp, M->ci, (const T*)Gd, (const T*)Xd,
                                                      scale, (T*)Od);
            SKR_LAUNCHED();
        };
        if (M->dtype == SKR_C64) launch(c64{});
        else launch(double{});
        if (mem == SKR_MEM_HOST) {
            SKR_HIP(hipMemcpyAsync(out_vals, Od, es * M->nnz, hipMemcpyDeviceToHost, st));
            SKR_HIP(hipStreamSynchronize(st));
            (void)hipFree(Gd);
            (void)hipFree(Xd);
            (void)hipFree(Od);
        }
        return SKR_OK;
    });
}

int skr_block_qr(skr_context* c, int64_t n64, int32_t s, int32_t dtype, const void* Z, void* Q, double* Cout,
                 int32_t mem) {
    if (!c) return SKR_E_INVALID;
    if (!Z || !Q || !Cout) return fail(c, SKR_E_INVALID, "null argument");
    if (n64 < 1 || n64 > kMaxRows || s < 1 || s > kMaxS || n64 < s)
        return fail(c, SKR_E_INVALID, "need 1 <= s <= 32 and s <= n <= 2^31 - 2^20");
    if (dtype != SKR_F64 && dtype != SKR_C64) return fail(c, SKR_E_INVALID, "bad dtype");
    if (mem != SKR_MEM_HOST && mem != SKR_MEM_DEVICE) return fail(c, SKR_E_INVALID, "bad mem");
    return guarded(c, [&]() -> int {
        SKR_HIP(hipSetDevice(c->device));
        const int n = (int)n64;
        const size_t es = elt(dtype, false);
        const size_t bytes = (size_t)n * s * es;
        hipStream_t st = c->stream();
        auto run = [&](auto tag) -> int {
            using T = decltype(tag);
            Env<T> e;
            env_layout(e, n, s);
            e.st = st;
            Arena sz;
            take_common(e, sz, 1);
            T* buf = (T*)sz.take(bytes);
            ensure_arena(c, sz.off);
            Arena ar;
            ar.base = c->arena;
            take_common(e, ar, 1);
            buf = (T*)ar.take(bytes);
            SKR_HIP(hipMemcpyAsync(buf, Z, bytes, mem == SKR_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                                   st));
            bool ok = (s <= 16) ? preprocess<T, 1>(c, e, buf) : preprocess<T, 2>(c, e, buf);
            SKR_HIP(hipMemcpyAsync(Q, buf, bytes, mem == SKR_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                                   st));
            std::vector<c64> Cm((size_t)s * s);
            SKR_HIP(hipMemcpyAsync(Cm.data(), e.mats + (size_t)M_RB * s * s, sizeof(c64) * s * s,
                                   hipMemcpyDeviceToHost, st));
            SKR_HIP(hipStreamSynchronize(st));
            for (int k = 0; k < s * s; ++k) {
                if (dtype == SKR_C64) {
                    Cout[2 * k] = Cm[k].x;
                    Cout[2 * k + 1] = Cm[k].y;
                } else {
                    Cout[k] = Cm[k].x;
                }
            }
            return ok ? SKR_OK : SKR_BREAKDOWN;
        };
        return dtype == SKR_C64 ? run(c64{}) : run(double{});
    });
}

int skr_block_qr_noalloc(skr_context* c, int64_t n64, int32_t s, int32_t dtype, const void* Z, void* Q,
                         double* Cout) {
    if (!c) return SKR_E_INVALID;
    if (!Z || !Q || !Cout) return fail(c, SKR_E_INVALID, "null argument");
    if (n64 < 1 || n64 > kMaxRows || s < 1 || s > kNoAllocMaxS || n64 < s)
        return fail(c, SKR_E_INVALID, "skr_block_qr_noalloc needs 1 <= s <= 16 and s <= n <= 2^31 - 2^20 "
                                      "(its static scratch holds the partials of s <= 16; use skr_block_qr)");
    if (dtype != SKR_F64 && dtype != SKR_C64) return fail(c, SKR_E_INVALID, "bad dtype");
    if (!c->scratch) return fail(c, SKR_E_HIP, "the static scratch array of this device could not be located");
    return guarded(c, [&]() -> int {
        SKR_HIP(hipSetDevice(c->device));
        const int n = (int)n64;
        const size_t bytes = (size_t)n * s * elt(dtype, false);
        hipStream_t st = c->stream();
        auto run = [&](auto tag) -> int {
            using T = decltype(tag);
            Env<T> e;
            env_layout(e, n, s);
            e.st = st;
            // the QR's state in the static scratch: control block, coefficient
            // slots, s x s partials of every workgroup and the second stage
            const size_t ss = (size_t)s * s;
            Arena ar;
            ar.base = c->scratch;
            ar.cap = kNoAllocBytes;
            e.ctl = (Ctl*)ar.take(sizeof(Ctl));
            e.hist = (double*)ar.take(4 * sizeof(double));
            e.sc = (c64*)ar.take(sizeof(c64) * 128);
            e.mats = (c64*)ar.take(sizeof(c64) * (size_t)M_COUNT * ss);
            e.part = (c64*)ar.take(sizeof(c64) * (size_t)e.nb * ss);
            e.part2 = (c64*)ar.take(sizeof(c64) * (size_t)e.p2 * ss);
            if (ar.off > kNoAllocBytes) throw Unsupported{"scratch layout exceeds the static array"};
            if (Q != Z) SKR_HIP(hipMemcpyAsync(Q, Z, bytes, hipMemcpyDeviceToDevice, st));
            const bool ok = preprocess<T, 1>(c, e, (T*)Q);   // s <= 16: one 16-column tile
            SKR_HIP(hipMemcpyAsync(c->hmat, e.mats + (size_t)M_RB * ss, sizeof(c64) * ss, hipMemcpyDeviceToHost,
                                   st));
            SKR_HIP(hipStreamSynchronize(st));
            for (size_t k = 0; k < ss; ++k) {
                if (dtype == SKR_C64) {
                    Cout[2 * k] = c->hmat[k].x;
                    Cout[2 * k + 1] = c->hmat[k].y;
                } else {
                    Cout[k] = c->hmat[k].x;
                }
            }
            return ok ? SKR_OK : SKR_BREAKDOWN;
        };
        return dtype == SKR_C64 ? run(c64{}) : run(double{});
    });
}

}  // extern "C"
