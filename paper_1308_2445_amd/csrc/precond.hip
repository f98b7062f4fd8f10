// Application of the global preconditioner K = (H - eps_bar S)^{-1} (eq. (k1p)) with the
// supernodal Cholesky factor P^T K P = L L^T computed once on the host (eq. (ldl)).
//
// Each supernode t owns columns D_t (its separator or leaf) and row set D_t + B_t
// (B_t in ancestors).  Its panel holds G = (L11 L11^T)^{-1} on top and F = L21 L11^{-1}
// below, which makes the two substitutions
//   forward   r_B -= F r_D         level by level, leaves to root (atomic: siblings share
//                                   ancestor rows)
//   diagonal  x_D  = G r_D          every supernode at once
//   backward  x_D -= F^T x_B       level by level, root to leaves
// (with y = L^{-1} r and x = L^{-T} y this is x_D = L11^{-T} (L11^{-1} r_D - L21^T x_B)).
// Every product reads only right-hand-side rows that are final when it starts: either
// all tasks run in one launch ordered by dependency (k_sn_sweep, the default), or one
// launch per level and phase (k_sn_product).
// The permutation is folded into the row lists (dof ids), so every block is read and
// written in the caller's ordering.  Right-hand-side blocks are row-major, so a gathered
// or updated row's 16 values are one contiguous segment.  The 64 x 64 by 64 x 16 product
// of a task runs on the matrix cores (16x16x4 MFMA, one 16-row tile per wavefront).
// Work-group task: 64 output rows x 16 right-hand sides x one 64-wide chunk of the
// reduction dimension, staged through LDS in a single round (every load of the task is
// in flight at once: the work is latency-bound at these sizes); chunks of one output
// tile accumulate with atomics, so the large separators at the top of the tree spread
// over many work-groups.  Outputs are zeroed first.  T is double (FP64 mode) or float
// (mixed mode: FP32 panels, FP32 accumulation).
#include <algorithm>

#include "common.h"

namespace labpsd {

namespace {

constexpr int TR = 64;   // output rows per work-group
constexpr int TC = 16;   // right-hand sides per work-group
constexpr int TCW = 64;  // the same for wide blocks (at least kWideCols columns)
constexpr int kWideCols = 128;
// FP64 blocks of at least kWide64Cols columns: 128 right-hand sides per deep task (each
// panel chunk read half as often; 512 columns of the 296k-dof factor: 39.1 against
// 41.4 ms per apply.  In FP32 the 128-wide tiles lose: 28.0 against 23.8 ms)
constexpr int TCW64 = 128;
constexpr int kWide64Cols = 256;
static_assert(kDeepChunk % 64 == 0, "deep tasks stage 64 reduction indices at a time");
constexpr int KS = 64;   // reduction chunk per work-group (one LDS stage)
constexpr int64_t kLevelsMaxNnz = 30000000;   // factors up to this nnz(L) apply level by level (narrow blocks)

enum { OP_DIAG = 0, OP_OFFD = 2, OP_OFFD_T = 3 };

// Tiled product for one task (supernode, output tile, reduction chunk); every op
// accumulates atomically into its output:
//  OP_DIAG   out[D[r]] += sum_k G[r,k] in[D[k]]
//  OP_OFFD   out[B[r]] -= sum_k F[r,k] in[D[k]]
//  OP_OFFD_T out[D[r]] -= sum_k F[k,r] in[B[k]]
template <typename T, int NC = TC>
struct SnTiles {
    T M[KS][TR + 1];   // M[k][r] = M(r0 + r, kb + k)
    T X[KS][NC + 1];   // X[k][c] = in[row(kb + k), c0 + c]
};

struct NoWait {
    __device__ void operator()() const {}
};

// One task on right-hand sides c0 .. c0 + NC - 1 (in and out may be the same block).
// Every thread of the work-group calls it.  The panel tile and the row indices are requested
// first; wait() (called by every thread) runs while they are in flight, and only then
// are the right-hand-side rows read.  CO: those rows are read with device-scope
// (coherent) loads, for rows other work-groups of the same launch have updated.
template <typename T, int OP, bool CO = false, typename Wait = NoWait, int NC = TC, int KD = KS>
__device__ __forceinline__ void sn_task(const SnTask& tk, const int32_t* __restrict__ rows,
                                        const T* __restrict__ panels, const T* in, T* out, int nrhs,
                                        int c0, SnTiles<T, NC>& st, Wait wait = Wait{}) {
    const int ncol = tk.ncol, nrow = tk.nrow;
    const int nb = nrow - ncol;
    const int32_t* rl = rows + tk.idx_off;
    const T* P = panels + tk.val_off;   // nrow x ncol, ld nrow
    const int nc = min(NC, nrhs - c0);

    // output and reduction extents
    int nout, nred;
    if (OP == OP_OFFD) { nout = nb; nred = ncol; }
    else if (OP == OP_OFFD_T) { nout = ncol; nred = nb; }
    else { nout = ncol; nred = ncol; }
    const int r0 = tk.r0;
    // the task's reduction range, staged KS at a time
    const int kb0 = tk.k0;
    const int k_all = min(nred, kb0 + KD);

    auto& sM = st.M;
    auto& sX = st.X;
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    constexpr int NJ = NC / 16;
    typedef T acc_t __attribute__((ext_vector_type(4)));
    acc_t acc[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[j] = acc_t{T(0), T(0), T(0), T(0)};
    for (int kb = kb0; kb < k_all; kb += KS) {
        const int k_end = min(k_all, kb + KS);
        // stage M(r, k) for r in [r0, r0+TR), k in [kb, kb+KS); every load issued before any use
        T mv[TR * KS / 256];
#pragma unroll
        for (int i = 0; i < TR * KS / 256; ++i) {
            const int e = t + 256 * i;
            T v = T(0);
            if (OP != OP_OFFD_T) {
                // column-major panel: consecutive threads walk rows (contiguous)
                const int r = r0 + (e % TR), k = kb + e / TR;
                if (r < nout && k < k_end) {
                    const int prow = (OP == OP_OFFD) ? ncol + r : r;
                    v = P[prow + (int64_t)k * nrow];
                }
            } else {
                // transposed: M(r, k) = F(k, r); consecutive threads walk k
                const int k = kb + (e % KS), r = r0 + e / KS;
                if (r < nout && k < k_end) v = P[(ncol + k) + (int64_t)r * nrow];
            }
            mv[i] = v;
        }
        // gathered right-hand sides: 16 consecutive lanes read 16 values of one row
        int gi[KS * NC / 256];
#pragma unroll
        for (int i = 0; i < KS * NC / 256; ++i) {
            const int e = t + 256 * i;
            const int c = e % NC, k = kb + e / NC;
            gi[i] = (k < k_end && c < nc) ? ((OP == OP_OFFD_T) ? rl[ncol + k] : rl[k]) : -1;
        }
        if (kb == kb0) wait();   // the dependencies, once per task (uniform)
        T xv[KS * NC / 256];
#pragma unroll
        for (int i = 0; i < KS * NC / 256; ++i) {
            const int c = (t + 256 * i) % NC;
            T v = T(0);
            if (gi[i] >= 0) {
                const T* src = in + (int64_t)gi[i] * nrhs + c0 + c;
                if constexpr (CO) v = __hip_atomic_load(const_cast<T*>(src), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                else v = *src;
            }
            xv[i] = v;
        }
        if (kb != kb0) __syncthreads();   // the previous stage's products have read the tiles
#pragma unroll
        for (int i = 0; i < TR * KS / 256; ++i) {
            const int e = t + 256 * i;
            if (OP != OP_OFFD_T) sM[e / TR][e % TR] = mv[i];
            else sM[e % KS][e / KS] = mv[i];
        }
#pragma unroll
        for (int i = 0; i < KS * NC / 256; ++i) {
            const int e = t + 256 * i;
            sX[e / NC][e % NC] = xv[i];
        }
        __syncthreads();
        // the 64 x NC output tile: wavefront w takes rows 16 w .. 16 w + 15, one 16 x 16
        // matrix-core tile per 16 columns; operands: A lane l = M(16 w + l % 16, k0 + l / 16),
        // B lane l = X(k0 + l / 16, 16 j + l % 16); staged zeros cover the chunk beyond k_end
        const int kn = k_end - kb;
        for (int k0 = 0; k0 < kn; k0 += 4) {
            const T a = sM[k0 + (lane >> 4)][16 * wave + (lane & 15)];
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const T b = sX[k0 + (lane >> 4)][16 * j + (lane & 15)];
                if constexpr (sizeof(T) == 8) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
                else acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[j], 0, 0, 0);
            }
        }
    }
    const bool sub = (OP == OP_OFFD || OP == OP_OFFD_T);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        // accumulator layout: register q of lane l holds row 4q + l / 16 (FP64) or
        // 4 (l / 16) + q (FP32) of the tile, column l % 16
        const int rt = (sizeof(T) == 8) ? 4 * q + (lane >> 4) : 4 * (lane >> 4) + q;
        const int r = r0 + 16 * wave + rt;
        if (r < nout) {
            const int64_t g = (OP == OP_OFFD) ? rl[ncol + r] : rl[r];
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const int c = 16 * j + (lane & 15);
                if (c < nc) atomicAdd(&out[g * nrhs + c0 + c], sub ? -acc[j][q] : acc[j][q]);
            }
        }
    }
}

template <typename T, int OP>
__global__ __launch_bounds__(256) void k_sn_product(const SnTask* __restrict__ tasks,
                                                    const int32_t* __restrict__ rows,
                                                    const T* __restrict__ panels,
                                                    const T* __restrict__ in, T* __restrict__ out,
                                                    int nrhs) {
    __shared__ SnTiles<T> st;
    sn_task<T, OP>(tasks[blockIdx.x], rows, panels, in, out, nrhs, blockIdx.y * TC, st);
}

// Upper bound on the polls of one dependency wait (with a short sleep between polls,
// seconds); a wait that runs out sets the error word and goes on, so every work-group
// finishes whatever happens.
constexpr int kSweepSpinLimit = 1 << 20;

// The whole solve in one launch.  A work-group's logical index b is a ticket it takes
// from a counter when it starts; it runs task b / groups on right-hand-side group
// b % groups (the groups of a task side by side, so they advance together).  Before its
// product a task waits until (forward and diagonal) every child supernode has finished
// its forward products, or (backward) the parent has finished its diagonal and backward
// products.  Every dependency has a lower task index, and a work-group holding ticket b
// started after every holder of a lower ticket had started, so those are resident and
// the lowest unfinished one can always run -- whatever order the XCDs dispatch the grid
// in and whatever other kernels share the device (the hardware index order gives no such
// guarantee on a multi-XCD part).  Results pass between work-groups only through
// device-scope atomics: a task's
// outputs are atomic adds, which it waits for (vmcnt) before counting itself off with an
// atomic; the last forward task of a supernode counts the supernode off at its parent;
// a waiting task polls its counter and reads right-hand-side rows with device-scope
// loads.  (Device-scope fences would write back or invalidate a whole L2 per task.)
template <typename T, int NC, int KD>
__global__ __launch_bounds__(256) void k_sn_sweep(const SweepTask* __restrict__ tasks, int64_t ntasks,
                                                  const int32_t* __restrict__ rows,
                                                  const T* __restrict__ panels, T* Y, T* W2, int nrhs,
                                                  int32_t* cnt, int nsn, int groups) {
    __shared__ SnTiles<T, NC> st;
    __shared__ int32_t s_ticket;
    if (threadIdx.x == 0)
        s_ticket = __hip_atomic_fetch_add(cnt + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int64_t b = s_ticket;
    const int64_t ti = b / groups;
    const int cg = (int)(b - ti * groups);
    const SweepTask tk = tasks[ti];
    int32_t* err = cnt;
    int32_t* ch_f = cnt + 4 + (int64_t)cg * 3 * nsn;   // children yet to finish forward
    int32_t* tk_f = ch_f + nsn;                          // forward tasks left
    int32_t* tk_b = ch_f + 2 * nsn;                      // diagonal and backward tasks left
    auto wait = [&]() {
        if (threadIdx.x == 0) {
            int32_t* w = tk.op == OP_OFFD_T ? tk_b + tk.parent : ch_f + tk.sn;
            // poll with a growing pause (waiting work-groups keep their polls off the
            // lines the producers update)
            int spins = 0, pause = 1;
            while (__hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                for (int i = 0; i < pause; ++i) __builtin_amdgcn_s_sleep(4);
                pause = pause < 4 ? 2 * pause : 4;
                if (++spins > kSweepSpinLimit) {
                    __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
        }
        __syncthreads();
    };
    const int c0 = cg * NC;
    if (tk.op == OP_OFFD)
        sn_task<T, OP_OFFD, true, decltype(wait), NC, KD>(tk.t, rows, panels, Y, Y, nrhs, c0, st, wait);
    else if (tk.op == OP_DIAG)
        sn_task<T, OP_DIAG, true, decltype(wait), NC, KD>(tk.t, rows, panels, Y, W2, nrhs, c0, st, wait);
    else
        sn_task<T, OP_OFFD_T, true, decltype(wait), NC, KD>(tk.t, rows, panels, W2, W2, nrhs, c0, st, wait);
    // every wavefront's atomic adds have completed (s_waitcnt vmcnt(0)) before the barrier
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (tk.op == OP_OFFD) {
            if (__hip_atomic_fetch_add(tk_f + tk.sn, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 1 &&
                tk.parent >= 0)
                __hip_atomic_fetch_add(ch_f + tk.parent, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_fetch_add(tk_b + tk.sn, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// W2 = 0, the ticket counter = 0 and the sweep counters of `groups` right-hand-side
// groups from their template (the error word, cnt[0], is left for the host to read)
template <typename T>
__global__ __launch_bounds__(256) void k_sweep_init(int64_t count, T* __restrict__ W2,
                                                    const int32_t* __restrict__ init, int64_t ninit,
                                                    int32_t* __restrict__ cnt, int groups) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    if (blockIdx.x == 0 && threadIdx.x == 0) cnt[1] = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += stride) W2[i] = T(0);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < ninit * groups; i += stride)
        cnt[4 + i] = init[i % ninit];
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill_copy(int64_t count, T* __restrict__ dst,
                                                   const T* __restrict__ src) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256)
        dst[i] = src ? src[i] : T(0);
}

template <typename T>
void fill_copy(T* dst, const T* src, int64_t count, hipStream_t s) {
    if (count <= 0) return;
    const int64_t blocks = std::min<int64_t>((count + 255) / 256, 2048);
    hipLaunchKernelGGL((k_fill_copy<T>), dim3((unsigned)blocks), dim3(256), 0, s, count, dst, src);
    LABPSD_HIP(hipGetLastError());
}

template <typename T, int OP>
void launch_level(const DevFactor& F, const SnTask* tasks, int64_t ntasks, const T* panels,
                  const T* in, T* out, int nrhs, hipStream_t s) {
    if (ntasks <= 0 || nrhs <= 0) return;
    LABPSD_REQUIRE(tasks != nullptr && panels != nullptr && in != nullptr && out != nullptr,
                   "supernodal product launched without its task list or buffers");
    dim3 grid((unsigned)ntasks, (unsigned)((nrhs + TC - 1) / TC));
    hipLaunchKernelGGL((k_sn_product<T, OP>), grid, dim3(256), 0, s, tasks, F.rows.p, panels, in, out,
                       nrhs);
    LABPSD_HIP(hipGetLastError());
}

}  // namespace

// Y: right-hand sides on entry (consumed); W2: result K^{-1} Y; W1 is not used.
// All are n x ncols row-major.
// The SMW step of the nonlocal term: W2 -= Ft (F^T W2), with W1 as the k x ncols scratch
template <typename T>
static void smw_correct(const NonLocal* nl, T* W1, T* W2, int64_t n, int ncols, hipStream_t s) {
    if (!nl || nl->k == 0 || ncols <= 0) return;
    LABPSD_REQUIRE(nl->smw_ready, "nonlocal term set but its SMW factor is not built");
    const T* Ft;
    if constexpr (sizeof(T) == 8) Ft = nl->Ft64.p;
    else Ft = nl->Ft32.p;
    launch_nl_ftx_rm<T>(*nl, W2, ncols, W1, s);
    launch_rm_gemm<T>(n, nl->k, ncols, Ft, W1, W2, -1.0, 1.0, s);
}

template <typename T>
void launch_precond_solve(const DevFactor& F, T* Y, T* W1, T* W2, int64_t n, int ncols,
                          hipStream_t s, const NonLocal* nl) {
    const T* panels;
    if constexpr (sizeof(T) == 8) panels = F.panels64.p;
    else panels = F.panels32.p;
    // the single-launch sweep pays a dependency hop between work-groups per tree level; on
    // a small factor with a narrow block the launch boundaries of the level-by-level route
    // are cheaper (16k-dof cell, 32 columns: FP64 0.24 against 0.31 ms, FP32 0.16 against
    // 0.38 ms per apply; the 296k-dof cell's sweep is twice as fast as its levels)
    const bool small = F.info.nnz_factor <= kLevelsMaxNnz && ncols < kWideCols;
    if (F.use_sweep && F.sweep.n > 0 && ncols > 0 && !small) {
        // wide blocks: 64 right-hand sides and a 256-deep reduction per task (the second
        // task list), so each panel chunk is read a quarter as often and each output tile
        // takes a quarter of the atomic adds
        const bool wide = ncols >= kWideCols && F.sweep_deep.n > 0;
        const bool wide128 = wide && sizeof(T) == 8 && ncols >= kWide64Cols;
        const int nc = wide128 ? TCW64 : wide ? TCW : TC;
        const int groups = (ncols + nc - 1) / nc;
        const int64_t ninit = 3 * (int64_t)F.nsn;
        const size_t need = 4 + (size_t)ninit * groups;
        if (F.sweep_cnt.n < need) {
            F.sweep_cnt.alloc(need);
            LABPSD_HIP(hipMemsetAsync(F.sweep_cnt.p, 0, 4 * sizeof(int32_t), s));
        }
        const int64_t count = n * ncols;
        const int64_t blocks = std::min<int64_t>((std::max<int64_t>(count, ninit * groups) + 255) / 256, 2048);
        hipLaunchKernelGGL((k_sweep_init<T>), dim3((unsigned)blocks), dim3(256), 0, s, count, W2,
                           wide ? F.sweep_init_deep.p : F.sweep_init.p, ninit, F.sweep_cnt.p, groups);
        const int64_t ntasks = (int64_t)(wide ? F.sweep_deep.n : F.sweep.n);
        if (wide128) {
            if constexpr (sizeof(T) == 8)
                hipLaunchKernelGGL((k_sn_sweep<T, TCW64, kDeepChunk>), dim3((unsigned)(ntasks * groups)), dim3(256),
                                   0, s, F.sweep_deep.p, ntasks, F.rows.p, panels, Y, W2, ncols, F.sweep_cnt.p,
                                   F.nsn, groups);
        } else if (wide)
            hipLaunchKernelGGL((k_sn_sweep<T, TCW, kDeepChunk>), dim3((unsigned)(ntasks * groups)), dim3(256), 0,
                               s, F.sweep_deep.p, ntasks, F.rows.p, panels, Y, W2, ncols, F.sweep_cnt.p, F.nsn,
                               groups);
        else
            hipLaunchKernelGGL((k_sn_sweep<T, TC, KS>), dim3((unsigned)(ntasks * groups)), dim3(256), 0, s,
                               F.sweep.p, ntasks, F.rows.p, panels, Y, W2, ncols, F.sweep_cnt.p, F.nsn, groups);
        LABPSD_HIP(hipGetLastError());
        smw_correct<T>(nl, W1, W2, n, ncols, s);
        return;
    }
    const int L = F.nlevels;
    fill_copy<T>(W2, nullptr, n * ncols, s);
    for (int l = 0; l < L; ++l)
        launch_level<T, OP_OFFD>(F, F.tasks.p + F.lev_off[4 * l + 1], F.lev_count[4 * l + 1], panels, Y, Y,
                                 ncols, s);
    launch_level<T, OP_DIAG>(F, F.tasks.p + F.diag_off, F.diag_count, panels, Y, W2, ncols, s);
    for (int l = L - 1; l >= 0; --l)
        launch_level<T, OP_OFFD_T>(F, F.tasks.p + F.lev_off[4 * l + 2], F.lev_count[4 * l + 2], panels, W2,
                                   W2, ncols, s);
    smw_correct<T>(nl, W1, W2, n, ncols, s);
}

void check_precond_sweep(const DevFactor& F, hipStream_t s) {
    if (!F.sweep_cnt.p) return;
    int32_t e = 0;
    LABPSD_HIP(hipMemcpyAsync(&e, F.sweep_cnt.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    LABPSD_HIP(hipStreamSynchronize(s));
    if (e != 0) {
        LABPSD_HIP(hipMemsetAsync(F.sweep_cnt.p, 0, sizeof(int32_t), s));
        LABPSD_HIP(hipStreamSynchronize(s));
        throw Error{LABPSD_EHIP, "preconditioner sweep: a dependency wait ran out"};
    }
}

template void launch_precond_solve<double>(const DevFactor&, double*, double*, double*, int64_t, int,
                                           hipStream_t, const NonLocal*);
template void launch_precond_solve<float>(const DevFactor&, float*, float*, float*, int64_t, int,
                                          hipStream_t, const NonLocal*);

}  // namespace labpsd
