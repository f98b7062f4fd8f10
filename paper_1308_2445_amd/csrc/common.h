// Internal declarations shared by the HIP translation units of liblabpsd.
#pragma once

#include <hip/hip_runtime.h>
#include <algorithm>

#include <cstdint>
#include <cstring>
#include <functional>
#include <string>
#include <utility>
#include <vector>

#include "../../include/labpsd.h"
#include "factor.h"
#include "serve_policy.h"

namespace labpsd {

// ------------------------------------------------------------------ errors

void set_error(const std::string& msg);
const char* get_error();

struct Error {
    labpsd_status code;
    std::string msg;
};

#define LABPSD_HIP(call)                                                                      \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            throw ::labpsd::Error{LABPSD_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define LABPSD_REQUIRE(cond, msg)                                                             \
    do {                                                                                      \
        if (!(cond)) throw ::labpsd::Error{LABPSD_EINVAL, (msg)};                             \
    } while (0)

// ------------------------------------------------------------------ device memory

template <typename T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    ~DBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    void alloc(size_t count) {
        if (count <= n && p) return;
        release();
        if (count == 0) return;
        hipError_t e = hipMalloc(&p, count * sizeof(T));
        if (e != hipSuccess) {
            p = nullptr;
            throw Error{LABPSD_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) +
                                           " bytes failed: " + hipGetErrorString(e)};
        }
        n = count;
    }
    void swap(DBuf& o) noexcept {
        std::swap(p, o.p);
        std::swap(n, o.n);
    }
    void upload(const T* h, size_t count, hipStream_t s) {
        alloc(count);
        if (count) LABPSD_HIP(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, s));
    }
};

// Cross-lane sums with DPP moves (VALU latency, no LDS round trip).  A DPP source lane
// that is inactive contributes 0.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}
// sum over the 16 lanes of a DPP row, in every lane of the row
__device__ __forceinline__ double row16_allsum(double v) {
    v += dpp_d<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_d<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_d<0x124>(v);   // row_ror 4
    v += dpp_d<0x128>(v);   // row_ror 8
    return v;
}
// sum over each group of 8 lanes (half a DPP row), in every lane of the group
__device__ __forceinline__ double row8_allsum(double v) {
    v += dpp_d<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_d<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_d<0x141>(v);   // row_half_mirror
    return v;
}
__device__ __forceinline__ double readlane_d(double v, int l) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | (uint64_t)lo);
}
// sum over the wavefront, in every lane; all 64 lanes must be active
__device__ __forceinline__ double wave_allsum(double v) {
    v = row16_allsum(v);
    return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// Pinned (page-locked, device-mapped) host memory that only grows.
template <typename T>
struct HBuf {
    T* p = nullptr;
    size_t n = 0;
    HBuf() = default;
    HBuf(const HBuf&) = delete;
    HBuf& operator=(const HBuf&) = delete;
    ~HBuf() {
        if (p) (void)hipHostFree(p);
    }
    void alloc(size_t count) {
        if (count <= n && p) return;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        n = 0;
        LABPSD_HIP(hipHostMalloc((void**)&p, std::max<size_t>(count, 1) * sizeof(T), hipHostMallocDefault));
        n = count;
        std::memset((void*)p, 0, std::max<size_t>(count, 1) * sizeof(T));
    }
};

// A few events without timing, created on first use.
struct EventSet {
    hipEvent_t e[3] = {nullptr, nullptr, nullptr};
    EventSet() = default;
    EventSet(const EventSet&) = delete;
    EventSet& operator=(const EventSet&) = delete;
    ~EventSet() {
        for (auto& x : e)
            if (x) (void)hipEventDestroy(x);
    }
    void ensure() {
        for (auto& x : e)
            if (!x) LABPSD_HIP(hipEventCreateWithFlags(&x, hipEventDisableTiming));
    }
};

// ------------------------------------------------------------------ sliced ELL

// Rows in slices of 64 (one wavefront, one row per lane); each slice is padded to
// its longest row and stored slot-major (64 consecutive entries per slot), so the
// loads of col/values across a wavefront are contiguous.
constexpr int kSlice = 64;

// Map a linear work-group index to a slice-block index so that each XCD (work-groups
// are dealt round-robin to the 8 XCDs) receives a contiguous range of slice blocks, and
// neighbouring rows' gathers hit the same L2.  A bijection on [0, nblocks).
__device__ __forceinline__ int64_t xcd_block(int64_t bid, int64_t nblocks) {
    constexpr int kXcd = 8;
    if (nblocks < 2 * kXcd) return bid;
    const int64_t per = nblocks / kXcd, rem = nblocks % kXcd;
    const int64_t xcd = bid % kXcd, idx = bid / kXcd;
    // XCDs 0..rem-1 own per+1 blocks, the rest own per
    const int64_t start = xcd * per + (xcd < rem ? xcd : rem);
    const int64_t own = per + (xcd < rem ? 1 : 0);
    if (idx < own) return start + idx;
    return bid;  // unreachable for bid < nblocks; kept total
}

struct Sell;

// Launch shape of the sliced-ELL kernels over many right-hand-side columns.  One slice
// per work-group of kSellWaves wavefronts: the slice's pattern (column indices, H and S
// values) is staged in LDS, in segments of at most `lseg` slots, and each wavefront takes
// CW columns of every round of kSellWaves * CW columns from there, so the pattern leaves
// HBM once per band of columns instead of once per few columns.  grid.y splits the
// columns into `bands` of about 96: the neighbouring slices' gathers of a band's X
// columns then meet in the caches.
constexpr int kSellWaves = 8;
constexpr size_t kSellLdsBytes = 80 * 1024;   // two work-groups per CU
struct SellShape {
    int cw;
    int bands;
    int lseg;
    size_t lds_bytes;
};
SellShape sell_shape(const Sell& A, int w, size_t value_bytes);
// Raise a kernel's dynamic-LDS limit on the current device to the device's maximum
// per work-group, once (under a lock; never lowered again).  Every kernel launched with
// more than 64 KB of dynamic LDS calls this first: setting the limit per launch to that
// launch's size would let a concurrent launch of the same kernel on another stream lower
// it between another thread's setting and its launch.
void allow_dynamic_lds(const void* kernel);

template <typename T>
struct SliceLds {
    T* h;
    T* s;
    int32_t* c;
};

template <typename T>
__device__ __forceinline__ SliceLds<T> slice_lds(void* base, int lseg) {
    T* h = (T*)base;
    T* s = h + (int64_t)lseg * kSlice;
    return SliceLds<T>{h, s, (int32_t*)(s + (int64_t)lseg * kSlice)};
}

// Copy slots s0 .. s0 + ns - 1 of the slice whose entries start at e0 into LDS (every
// thread of the work-group takes part).
template <typename T>
__device__ __forceinline__ void sell_stage(const int32_t* __restrict__ col, const T* __restrict__ hv,
                                           const T* __restrict__ sv, int64_t e0, int s0, int ns,
                                           SliceLds<T> L) {
    const int64_t b = e0 + (int64_t)s0 * kSlice;
    for (int i = threadIdx.x; i < ns * kSlice; i += blockDim.x) {
        L.c[i] = col[b + i];
        L.h[i] = hv[b + i];
        L.s[i] = sv[b + i];
    }
}

// ah[j] += H(row, :) x_j and as[j] += S(row, :) x_j over the ns staged slots, for the CW
// columns whose bases xp[j] gives (row = the lane's row of the slice).  Four slots at a
// time: all four slots' gathers of every column are issued before the products (two at a
// time left a wavefront waiting on each pair's gathers: 296k-dof cell, 410 columns, 4.32
// against 4.10 ms per product; eight gain nothing more).  Padding slots hold the lane's
// own row and zero values.
template <typename T, int CW>
__device__ __forceinline__ void sell_lds_accumulate(SliceLds<T> L, int ns, const T* const (&xp)[CW],
                                                    T (&ah)[CW], T (&as)[CW]) {
    const int lane = threadIdx.x & 63;
    constexpr int U = 4;
    int k = 0;
    for (; k + U <= ns; k += U) {
        int32_t c[U];
        T h[U], s[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            c[u] = L.c[(k + u) * kSlice + lane];
            h[u] = L.h[(k + u) * kSlice + lane];
            s[u] = L.s[(k + u) * kSlice + lane];
        }
        T x[U][CW];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < CW; ++j) x[u][j] = xp[j][c[u]];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < CW; ++j) {
                ah[j] = fma(h[u], x[u][j], ah[j]);
                as[j] = fma(s[u], x[u][j], as[j]);
            }
    }
    for (; k < ns; ++k) {
        const int32_t c = L.c[k * kSlice + lane];
        const T h = L.h[k * kSlice + lane], s = L.s[k * kSlice + lane];
#pragma unroll
        for (int j = 0; j < CW; ++j) {
            const T x = xp[j][c];
            ah[j] = fma(h, x, ah[j]);
            as[j] = fma(s, x, as[j]);
        }
    }
}

// The nonlocal term H_nl = F G F^T of a product (Section 4, eq. (fgf)), added to the H
// part of a sliced-ELL product row by row: the kernel's row i gains
// sum_e F[i, c_e] W[c_e, j] over the entries of row i of F, with W = G F^T X formed
// beforehand (k x w, column stride ldw).  rp == nullptr: no nonlocal term.
template <typename T, typename TW>
struct NlEpi {
    const int64_t* rp = nullptr;   // F rows: row pointers (n + 1)
    const int32_t* ci = nullptr;   // projector index of every entry
    const T* fv = nullptr;         // F values
    const TW* W = nullptr;         // G F^T X, k x w
    int64_t ldw = 0;
};

template <typename T, typename TW>
__device__ __forceinline__ T nl_row_term(const NlEpi<T, TW>& nl, int64_t row, int col) {
    T s = T(0);
    const int64_t e1 = nl.rp[row + 1];
    for (int64_t e = nl.rp[row]; e < e1; ++e) s += nl.fv[e] * (T)nl.W[nl.ci[e] + (int64_t)col * nl.ldw];
    return s;
}

struct Sell {
    int64_t n = 0;
    int64_t nslices = 0;
    int64_t stored = 0;          // padded entries
    int max_slots = 0;           // slots of the longest slice
    DBuf<int64_t> slice_off;     // nslices + 1 offsets (entries)
    DBuf<int32_t> col;
    DBuf<double> hv, sv;         // FP64 values
    DBuf<float> hv32, sv32;      // FP32 copies for the mixed-precision preconditioner
    std::vector<int64_t> h_slice_off;   // host copies of the layout (for update_h)
    std::vector<int64_t> h_map;         // stored entry -> CSR entry (-1 for padding)
};

// ------------------------------------------------------------------ device factor

// One work-group task of the supernodal apply: a 64-row output tile of one supernode's
// product and one 64-wide chunk of its reduction dimension, with the supernode's
// metadata folded in so a work-group needs a single (scalar) load to start.
// reduction depth of a task in the sweep over wide right-hand-side blocks
constexpr int kDeepChunk = 256;

struct SnTask {
    int64_t idx_off;   // offset of the supernode's row list in DevFactor::rows
    int64_t val_off;   // offset of its panel [G ; F] (ld nrow)
    int32_t ncol;      // |D|
    int32_t nrow;      // |D| + |B|
    int32_t r0;        // first output row of the tile
    int32_t k0;        // first reduction index of the chunk
};
static_assert(sizeof(SnTask) == 32, "SnTask is two 16-byte words");

// A task of the single-launch sweep (launch_precond_solve): a product task and its
// place in the supernode tree; op 2 forward, 0 diagonal, 3 backward.
struct SweepTask {
    SnTask t;
    int32_t op;       // which product
    int32_t sn;       // its supernode
    int32_t parent;   // the supernode's parent (-1 for a root)
    int32_t pad;
};
static_assert(sizeof(SweepTask) == 48, "sweep task layout");

struct DevFactor {
    int64_t n = 0;
    int nsn = 0;
    int nlevels = 0;
    double eps_bar = 0.0;
    DBuf<int32_t> rows;          // row lists (dof ids)
    DBuf<double> panels64;
    DBuf<float> panels32;
    // work-group tasks: per level [level][op] with op 1 the forward off-diagonal product
    // (r_B -= F r_D) and op 2 the backward one (x_D -= F^T x_B) (ops 0 and 3 unused),
    // and one list of the diagonal products x_D = G r_D of all supernodes
    std::vector<int64_t> lev_off, lev_count;   // 4 * nlevels each
    int64_t diag_off = 0, diag_count = 0;
    DBuf<SnTask> tasks;
    // The same products as one launch: every task in dependency order (forward level by
    // level from the leaves, the diagonal products, backward level by level from the
    // roots), each waiting on counters of its supernode's children or parent.  The
    // initial counters per supernode are (children, forward tasks, diagonal and backward
    // tasks); sweep_cnt holds an error word (4 ints) and then their live copy for each
    // group of 16 right-hand sides.
    DBuf<SweepTask> sweep;
    DBuf<int32_t> sweep_init;            // 3 nsn
    DBuf<SweepTask> sweep_deep;          // the same sweep with kDeepChunk-deep reductions
    DBuf<int32_t> sweep_init_deep;
    mutable DBuf<int32_t> sweep_cnt;     // 4 + 3 nsn groups
    bool use_sweep = true;
    labpsd_factor_info info{};
};

// Raise an error if a preconditioner sweep on F gave up waiting for a dependency (a
// counter that never reached zero) since the last check; synchronises with s.
void check_precond_sweep(const DevFactor& F, hipStream_t s);

// ------------------------------------------------------------------ context / problem

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int cu_count = 256;
    DBuf<double> scratch;        // small reductions
    DBuf<char> rr_ws;            // Rayleigh-Ritz workspace
};

struct LocalParams {
    double tau1 = 0.1, tau2 = 0.1, eta = 0.25;
    int max_inner = 20;
    int mode = LABPSD_HYBRID;
    int method = LABPSD_REFINE_MINRES;
};

struct Problem;

}  // namespace labpsd

struct labpsd_ctx : labpsd::Ctx {};

namespace labpsd {

// The nonlocal term H_nl = F G F^T (Section 4, eq. (fgf)) on the device: F by columns
// (for F^T X) and by rows (for the product epilogues) in FP64 and FP32, G in both, and
// for the global apply the SMW factor Ft = (H_loc - eps_bar S)^{-1} F T^{-1} G with
// T = I + G F^T (H_loc - eps_bar S)^{-1} F (n x k row-major, built with the factor), so
// that P = P_loc - Ft (F^T P_loc) (the update that ends the SMW outline of Section 4).
struct NonLocal {
    int k = 0;
    std::vector<int64_t> h_colptr, h_rowptr;
    std::vector<int32_t> h_rowidx, h_colidx;
    std::vector<double> h_cval, h_rval, h_G;
    DBuf<int64_t> colptr, rowptr;
    DBuf<int32_t> rowidx, colidx;
    DBuf<double> cval64, rval64, G64;
    DBuf<float> cval32, rval32, G32;
    DBuf<double> Ft64;
    DBuf<float> Ft32;
    bool smw_ready = false;
    // W = F^T X and G W for the products (k x w FP64 or FP32)
    mutable DBuf<double> w64a, w64b;
    mutable DBuf<float> w32a, w32b;
    template <typename T, typename TW>
    NlEpi<T, TW> epi(const TW* W, int64_t ldw) const {
        NlEpi<T, TW> e;
        if (k == 0) return e;
        e.rp = rowptr.p;
        e.ci = colidx.p;
        if constexpr (sizeof(T) == 8) e.fv = rval64.p;
        else e.fv = rval32.p;
        e.W = W;
        e.ldw = ldw;
        return e;
    }
};

// G F^T X for the w columns of X (column-major, ld ldx; xcols[j] selects column j, or the
// identity when null) into nl.w*b (k x w), and the epilogue view of it; a view with
// rp == nullptr when there is no nonlocal term.
template <typename T>
NlEpi<T, T> nl_prepare(const NonLocal& nl, const T* X, int64_t ldx, const int32_t* xcols, int w,
                       hipStream_t s);
// Row-major forms for the global apply: W (k x m, row-major) = F^T X for X n x m row-major;
// D = alpha A B + beta D for A n x k, B k x m, D n x m, all row-major.
template <typename T>
void launch_nl_ftx_rm(const NonLocal& nl, const T* X, int m, T* W, hipStream_t s);
template <typename T>
void launch_rm_gemm(int64_t n, int k, int m, const T* A, const T* B, T* D, double alpha, double beta,
                    hipStream_t s);

struct Problem {
    labpsd_ctx* ctx = nullptr;
    int64_t n = 0, nnz = 0;
    HostCSR csr;
    std::vector<double> h_val, s_val;
    Sell sell;
    DevFactor* factor = nullptr;
    NonLocal nl;
    // a complex Hermitian pencil stored as its real embedding (interleaved, n = 2 nc)
    bool hermitian = false;
    int64_t nc = 0;
    LocalParams local;
    // solver workspace (kept between solves)
    DBuf<double> ws64;
    DBuf<float> ws32;
    DBuf<double> red;            // FP64 preconditioner arena
    DBuf<int32_t> iws;
    // host side of the solve loop (kept between solves): read-back blocks, the selection
    // upload block, the MINRES done flags, and the loop's events
    HBuf<double> h_rb, h_sel;
    HBuf<int32_t> h_ib, h_flags;
    EventSet events;
    // the last solve's full block (n x b, all Ritz vectors incl. guards) and Ritz
    // values, kept resident for warm starts of the next GHEP of the sequence
    DBuf<double> resident_X;
    std::vector<double> resident_E;
    int resident_b = 0;
    ~Problem();
};

}  // namespace labpsd

struct labpsd_problem : labpsd::Problem {};

namespace labpsd {

// Resolve the device address of the allocation-free entry points' static scratch array
// on `device` (must be the current device); idempotent.
void noalloc_setup(int device);
size_t noalloc_scratch_doubles();

// Run one LABPSD solve of P on `stream` (the driver of labpsd_solve).
labpsd_status run_solve(Problem& P, const labpsd_solve_params& prm, const double* X0,
                        const double* E0, labpsd_mem in_where, double* lambda, double* X,
                        double* res_hist, double* ritz_hist, int* n_hist, labpsd_mem out_where, labpsd_stats* stats,
                        hipStream_t stream);
// The solve arenas of one solve (carve() cuts them up) and the device bytes one solve
// reserves beyond the resident problem (the arenas plus the resident block it leaves).
ArenaElems solve_arena_elems(int64_t n, int nev, int m0, int precision, int cu_count);
size_t solve_footprint_bytes(int64_t n, int nev, int m0, int precision, int cu_count);

// ------------------------------------------------------------------ kernel launchers
// All launchers enqueue on `s` and check the launch.

void build_sell(Sell& S, const HostCSR& A, const double* hv, const double* sv, hipStream_t s);
void refresh_sell_h(Sell& S, const double* hv, hipStream_t s);
// the guarded-call wrapper of the C ABI (maps exceptions to status codes)
labpsd_status abi_guard(const std::function<labpsd_status()>& f);

// YH = H X, YS = S X (FP64); nl: the nonlocal term of H (null: none)
void launch_spmm_hs(const Sell& A, const double* X, int64_t ldx, int w, double* YH, double* YS,
                    int64_t ldy, hipStream_t s, const NonLocal* nl = nullptr);
// Y = (H - shift_j S) X (T = double or float; shift in double)
template <typename T>
void launch_spmm_shift(const Sell& A, const T* X, int64_t ldx, int w, const double* shift, T* Y,
                       int64_t ldy, hipStream_t s, const NonLocal* nl = nullptr);

// Interleaved complex columns (nc complex entries each): dst = J src, or J^T src, with J the
// real form of multiplication by i
void launch_apply_j(int64_t nc, int ncols, const double* src, int64_t lds, double* dst, int64_t ldd, bool transpose,
                    hipStream_t s);

// X (n x b, ld ldx) := i.i.d. standard normals, entry (i, j) from counter i + n j of `seed`
void launch_random_block(int64_t n, int b, uint64_t seed, double* X, int64_t ldx, hipStream_t s);

// residual and per-column norms (partials reduced by launch_residual_finish)
void launch_residual(int64_t n, int m, const double* PsiH, const double* PsiS, int64_t ld,
                     const double* E, double sigma0, double* R, int64_t ldr, double* partial,
                     int nblk, hipStream_t s);
// host: optional device-mapped pinned memory that also receives [Res | norms] (2 m);
// flag_dst (optional, device-visible) receives *flag_src (0 if flag_src is null)
void launch_residual_finish(int m, const double* partial, int nblk, double* res, double* rnorm,
                            hipStream_t s, double* host = nullptr, const int32_t* flag_src = nullptr,
                            int32_t* flag_dst = nullptr);
int residual_blocks(int64_t n);

// Gram: HR = Z^T ZH, SR = Z^T ZS (symmetric parts); partial workspace sized by gram_ws
size_t gram_ws_doubles(int64_t n, int k, int cu_count);
// out (device-visible) = max |SR - I| over the b x b matrix SR (ld ld)
void launch_orth_deviation(int b, const double* SR, int64_t ld, double* out, hipStream_t s);
void launch_gram(int64_t n, int k, const double* Z, const double* ZH, const double* ZS, int64_t ldz,
                 double* HR, double* SR, int64_t ldr, double* ws, int cu_count, hipStream_t s);

// MFMA tiles per wavefront of the wide block update for b output columns (6, 8 or 9)
int block_update_ct(int b);
// Block update: out_i = in_i W for i = 0..2
void launch_block_update(int64_t n, int k, int b, const double* Z, const double* ZH,
                         const double* ZS, int64_t ldz, const double* W, int64_t ldw, double* Psi,
                         double* PsiH, double* PsiS, int64_t ldo, hipStream_t s);

// Rayleigh-Ritz (single work-group, k <= kRRMax)
constexpr int kRRMax = 4096;
size_t rr_ws_bytes(int k);
// gamma_host, info_host: optional device-mapped pinned memory that also receives the
// nwant Ritz values and the two report words
void launch_rayleigh_ritz(int k, int nwant, const double* HR, const double* SR, int64_t ldr,
                          double* gamma, double* W, int64_t ldw, int32_t* info, void* ws,
                          hipStream_t s, double* gamma_host = nullptr, int32_t* info_host = nullptr);

// Gathers / casts
// row-major blocks (the ncols values of a row contiguous) for the global preconditioner:
// dst[i * ncols + j] = (TD) src[i + cols[j] * lds] * scale  (cols may be null: identity)
template <typename TS, typename TD>
void launch_cast_to_rm(int64_t n, int ncols, const TS* src, int64_t lds, const int32_t* cols,
                       double scale, TD* dst, hipStream_t s);
// dst[i + j * ldd] = (TD) src[i * ncols + j] * scale
template <typename TS, typename TD>
void launch_cast_from_rm(int64_t n, int ncols, const TS* src, double scale, TD* dst, int64_t ldd,
                         hipStream_t s);
// dst[:, j] = (T) src[:, cols[j]] * scale  (cols may be null: identity)
template <typename TS, typename TD>
void launch_gather_cast(int64_t n, int ncols, const TS* src, int64_t lds, const int32_t* cols,
                        double scale, TD* dst, int64_t ldd, hipStream_t s);

// dst[:, cols[j]] = (TD) src[:, j] * scale
template <typename TS, typename TD>
void launch_scatter_cast(int64_t n, int ncols, const TS* src, int64_t lds, const int32_t* cols,
                         double scale, TD* dst, int64_t ldd, hipStream_t s);
// out[j] = ||src[:, cols[j]]|| (cols may be null); partial holds residual_blocks(n) * q doubles
template <typename T>
void launch_colnorms(int64_t n, int q, const T* src, int64_t ld, const int32_t* cols,
                     double* partial, double* out, hipStream_t s);

// Global preconditioner: W2 := K^{-1} Y for n x ncols row-major blocks (element (i, j)
// at i * ncols + j) of precision T; Y is consumed, W1 is scratch
// With nl (its SMW factor built), the result is corrected to (H - eps_bar S)^{-1} Y for
// H = H_loc + F G F^T: W2 -= Ft (F^T W2), with W1 holding F^T W2 (k x ncols).
template <typename T>
void launch_precond_solve(const DevFactor& F, T* Y, T* W1, T* W2, int64_t n, int ncols,
                          hipStream_t s, const NonLocal* nl = nullptr);
// Build the SMW factor of P's nonlocal term with its global factor (synchronises).
void nonlocal_smw_setup(Problem& P);

// MINRES batched refinement (T = double or float). P (n x *, ld ldp) in precision T is
// refined in place on the columns cols[0..q), with the residual columns R[:, cols[j]] in
// precision T, shifts shift[j] and stopping norms eta * rnorm[j].  ws holds
// minres_ws_elems(n, q) elements of T, scal_ws minres_scal_doubles(q) doubles.
size_t minres_ws_elems(int64_t n, int q);
size_t minres_scal_doubles(int q);
// flag_host_pinned: pinned host memory of 2 q ints (the done flags of the checked
// iterations); ev0, ev1: two events for pipelined checks (else a synchronisation per check)
template <typename T>
void run_minres(const Sell& A, T* P, int64_t ldp, const T* R, int64_t ldr, int q,
                const int32_t* cols_dev, const double* shift_dev, const double* rnorm_dev,
                double eta, int max_inner, int32_t* its_dev, T* ws, double* scal_ws,
                int32_t* flag_host_pinned, hipStream_t s, int64_t* launches, hipEvent_t ev0 = nullptr,
                hipEvent_t ev1 = nullptr, unsigned long long* its_total = nullptr,
                int method = LABPSD_REFINE_MINRES, const NonLocal* nl = nullptr);

// Wait until everything enqueued on s so far has finished.  With an event the host polls
// it (spins) instead of blocking, which shortens the wake-up after the small read-backs
// the solve loop waits on; without one it falls back to hipStreamSynchronize.
void spin_sync(hipStream_t s, hipEvent_t ev);
// Wait for an event recorded earlier by polling it.
void spin_event(hipEvent_t ev);

}  // namespace labpsd
