// Application of the global preconditioner K = (H - eps_bar S)^{-1} (eq. (k1p)) with the
// supernodal Cholesky factor P^T K P = L L^T computed once on the host (eq. (ldl)).
//
// Each supernode t owns columns D_t (its separator or leaf) and row set D_t + B_t
// (B_t in ancestors).  Its panel holds inv(L11) (lower) on top and L21 below, so the
// substitutions become small dense products.  Supernodes of one tree level are
// independent; levels run leaves to root (forward) and root to leaves (backward):
//   forward  level l:  y[D] <- inv(L11) y[D]          (diag kernel, assign)
//                      r[B] -= L21 y[D]               (off-diag kernel, atomic: siblings
//                                                      share ancestor rows)
//   backward level l:  z[D] <- y[D] - L21^T x[B]      (gather kernel)
//                      x[D] <- inv(L11)^T z[D]        (diag kernel)
// The permutation is folded into the row lists (dof ids), so every block is read and
// written in the caller's ordering.  Right-hand-side blocks are row-major, so a gathered
// or updated row's 16 values are one contiguous segment.  Work-group task: 64 output rows x 16 right-hand
// sides x one 64-wide chunk of the reduction dimension, staged through LDS in a single
// round (every load of the task is in flight at once: the work is latency-bound at
// these sizes); chunks of one output tile accumulate with atomics, so the large
// separators at the top of the tree spread over many work-groups.  Outputs are zeroed
// (or seeded) first.  T is double (FP64 mode) or float (mixed mode: FP32 panels, FP32
// accumulation).
#include <algorithm>

#include "common.h"

namespace labpsd {

namespace {

constexpr int TR = 64;   // output rows per work-group
constexpr int TC = 16;   // right-hand sides per work-group
constexpr int KS = 64;   // reduction chunk per work-group (one LDS stage)

enum { OP_DIAG = 0, OP_DIAG_T = 1, OP_OFFD = 2, OP_OFFD_T = 3 };

// Tiled product for one task (supernode, output tile, reduction chunk) of a level;
// every op accumulates atomically into its output:
//  OP_DIAG   out[D[r]] += sum_{k<=r} inv(L11)[r,k] in[D[k]]
//  OP_DIAG_T out[D[r]] += sum_{k>=r} inv(L11)[k,r] in[D[k]]
//  OP_OFFD   out[B[r]] -= sum_k L21[r,k] in[D[k]]
//  OP_OFFD_T out[D[r]] -= sum_k L21[k,r] in[B[k]]
template <typename T, int OP>
__global__ __launch_bounds__(256) void k_sn_product(const SnTask* __restrict__ tasks,
                                                    const int32_t* __restrict__ rows,
                                                    const T* __restrict__ panels,
                                                    const T* __restrict__ in, T* __restrict__ out,
                                                    int nrhs) {
    const SnTask tk = tasks[blockIdx.x];
    const int ncol = tk.ncol, nrow = tk.nrow;
    const int nb = nrow - ncol;
    const int32_t* rl = rows + tk.idx_off;
    const T* P = panels + tk.val_off;   // nrow x ncol, ld nrow
    const int c0 = blockIdx.y * TC;
    const int nc = min(TC, nrhs - c0);

    // output and reduction extents
    int nout, nred;
    if (OP == OP_OFFD) { nout = nb; nred = ncol; }
    else if (OP == OP_OFFD_T) { nout = ncol; nred = nb; }
    else { nout = ncol; nred = ncol; }
    const int r0 = tk.r0;
    const int kb = tk.k0;
    // reduction range of the chunk (triangular blocks skip the zero half)
    int k_end = min(nred, kb + KS);
    if (OP == OP_DIAG) k_end = min(k_end, r0 + TR);

    __shared__ T sM[KS][TR + 1];      // sM[k][r] = M(r0 + r, kb + k)
    __shared__ T sX[KS][TC];          // sX[k][c] = in[row(kb + k), c0 + c]
    const int t = threadIdx.x;
    // stage M(r, k) for r in [r0, r0+TR), k in [kb, kb+KS); every load issued before any use
    T mv[TR * KS / 256];
#pragma unroll
    for (int i = 0; i < TR * KS / 256; ++i) {
        const int e = t + 256 * i;
        T v = T(0);
        if (OP == OP_DIAG || OP == OP_OFFD) {
            // column-major panel: consecutive threads walk rows (contiguous)
            const int r = r0 + (e % TR), k = kb + e / TR;
            if (r < nout && k < k_end) {
                const int prow = (OP == OP_OFFD) ? ncol + r : r;
                if (OP == OP_OFFD || k <= r) v = P[prow + (int64_t)k * nrow];
            }
        } else {
            // transposed: M(r, k) = panel(krow, r); consecutive threads walk k
            const int k = kb + (e % KS), r = r0 + e / KS;
            if (r < nout && k < k_end) {
                const int krow = (OP == OP_OFFD_T) ? ncol + k : k;
                if (OP == OP_OFFD_T || k >= r) v = P[krow + (int64_t)r * nrow];
            }
        }
        mv[i] = v;
    }
    // gathered right-hand sides: 16 consecutive lanes read the 16 values of one row
    T xv[KS * TC / 256];
#pragma unroll
    for (int i = 0; i < KS * TC / 256; ++i) {
        const int e = t + 256 * i;
        const int c = e % TC, kk = e / TC;
        const int k = kb + kk;
        T v = T(0);
        if (k < k_end && c < nc) {
            const int grow = (OP == OP_OFFD_T) ? rl[ncol + k] : rl[k];
            v = in[(int64_t)grow * nrhs + c0 + c];
        }
        xv[i] = v;
    }
#pragma unroll
    for (int i = 0; i < TR * KS / 256; ++i) {
        const int e = t + 256 * i;
        if (OP == OP_DIAG || OP == OP_OFFD) sM[e / TR][e % TR] = mv[i];
        else sM[e % KS][e / KS] = mv[i];
    }
#pragma unroll
    for (int i = 0; i < KS * TC / 256; ++i) {
        const int e = t + 256 * i;
        sX[e / TC][e % TC] = xv[i];
    }
    __syncthreads();
    // thread: right-hand side c, output rows rb, rb + 16, rb + 32, rb + 48 of the tile
    const int c = t % TC, rb = t / TC;
    T acc[TR / 16] = {};
    const int kn = k_end - kb;
#pragma unroll 8
    for (int kk = 0; kk < kn; ++kk) {
        const T x = sX[kk][c];
#pragma unroll
        for (int j = 0; j < TR / 16; ++j) acc[j] = fma(sM[kk][rb + 16 * j], x, acc[j]);
    }
    if (c >= nc) return;
    const bool sub = (OP == OP_OFFD || OP == OP_OFFD_T);
#pragma unroll
    for (int j = 0; j < TR / 16; ++j) {
        const int r = r0 + rb + 16 * j;
        if (r < nout) {
            const int64_t g = (OP == OP_OFFD) ? rl[ncol + r] : rl[r];
            atomicAdd(&out[g * nrhs + c0 + c], sub ? -acc[j] : acc[j]);
        }
    }
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

// Y: right-hand sides on entry (consumed); W1: forward solution; W2: result K^{-1} Y.
// All three are n x ncols row-major.
template <typename T>
void launch_precond_solve(const DevFactor& F, T* Y, T* W1, T* W2, int64_t n, int ncols,
                          hipStream_t s) {
    const T* panels;
    if constexpr (sizeof(T) == 8) panels = F.panels64.p;
    else panels = F.panels32.p;
    const int L = F.nlevels;
    const int64_t nb = n * ncols;
    fill_copy<T>(W1, nullptr, nb, s);
    fill_copy<T>(W2, nullptr, nb, s);
    for (int l = 0; l < L; ++l) {
        const int64_t* o = &F.lev_off[4 * l];
        launch_level<T, OP_DIAG>(F, F.tasks.p + o[0], F.lev_count[4 * l + 0], panels, Y, W1, ncols, s);
        launch_level<T, OP_OFFD>(F, F.tasks.p + o[1], F.lev_count[4 * l + 1], panels, W1, Y, ncols, s);
    }
    // z = y - L21^T x accumulates into a copy of the forward solution, held in Y
    fill_copy<T>(Y, W1, nb, s);
    for (int l = L - 1; l >= 0; --l) {
        const int64_t* o = &F.lev_off[4 * l];
        launch_level<T, OP_OFFD_T>(F, F.tasks.p + o[2], F.lev_count[4 * l + 2], panels, W2, Y, ncols, s);
        launch_level<T, OP_DIAG_T>(F, F.tasks.p + o[3], F.lev_count[4 * l + 3], panels, Y, W2, ncols, s);
    }
}

template void launch_precond_solve<double>(const DevFactor&, double*, double*, double*, int64_t, int,
                                           hipStream_t);
template void launch_precond_solve<float>(const DevFactor&, float*, float*, float*, int64_t, int,
                                          hipStream_t);

}  // namespace labpsd
