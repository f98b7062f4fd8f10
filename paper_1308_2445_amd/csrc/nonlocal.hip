// The nonlocal part of the Hamiltonian, H = H_loc + F G F^T (Section 4, eqs. (k1),
// (fgf)): its rank-k products and the Sherman-Morrison-Woodbury form of the global
// preconditioner.
//
// Products: W = F^T X (one work-group per projector and column chunk, a reduction over the
// projector's rows), W2 = G W (k x k times k x w), then the sliced-ELL kernels add row i's
// sum_e F[i, c_e] W2[c_e, j] in their epilogue (NlEpi), so H X costs one pattern pass
// plus the small rank-k work.
//
// Global apply (eq. (k1p) with eq. (k1)): the factorisation (eq. (ldl)) is of
// H_loc - eps_bar S only.  With Fh = (H_loc - eps_bar S)^{-1} F and T = I + G F^T Fh, the
// SMW formula gives (H - eps_bar S)^{-1} = (H_loc - eps_bar S)^{-1} - Fh T^{-1} G F^T
// (H_loc - eps_bar S)^{-1}; Ft = Fh T^{-1} G is formed once (the section's first four
// steps), and every apply ends with P -= Ft (F^T P) (its last step).
#include <cmath>

#include "common.h"

namespace labpsd {

namespace {

constexpr int kNlCols = 8;   // columns per work-group of the F^T X reduction

// W[a + j ldw] = sum_i F[i, a] X[i, xcols ? xcols[j] : j] for columns j0 .. j0 + 7
template <typename T>
__global__ __launch_bounds__(256) void k_nl_ftx(const int64_t* __restrict__ colptr,
                                                const int32_t* __restrict__ rowidx,
                                                const T* __restrict__ cval, const T* __restrict__ X,
                                                int64_t ldx, const int32_t* __restrict__ xcols, int w,
                                                T* __restrict__ W, int64_t ldw) {
    const int a = blockIdx.x;
    const int j0 = blockIdx.y * kNlCols;
    const int nc = min(kNlCols, w - j0);
    const T* xp[kNlCols];
#pragma unroll
    for (int j = 0; j < kNlCols; ++j) {
        const int jj = j < nc ? j0 + j : j0;
        xp[j] = X + (int64_t)(xcols ? xcols[jj] : jj) * ldx;
    }
    T acc[kNlCols];
#pragma unroll
    for (int j = 0; j < kNlCols; ++j) acc[j] = T(0);
    for (int64_t e = colptr[a] + threadIdx.x; e < colptr[a + 1]; e += 256) {
        const int64_t i = rowidx[e];
        const T f = cval[e];
#pragma unroll
        for (int j = 0; j < kNlCols; ++j) acc[j] = fma(f, xp[j][i], acc[j]);
    }
    __shared__ T red[4][kNlCols];
#pragma unroll
    for (int j = 0; j < kNlCols; ++j) {
        T v = acc[j];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][j] = v;
    }
    __syncthreads();
    if (threadIdx.x < nc) {
        const int j = threadIdx.x;
        W[a + (int64_t)(j0 + j) * ldw] = (red[0][j] + red[1][j]) + (red[2][j] + red[3][j]);
    }
}

// W2[a + j k] = sum_b G[a + b k] W[b + j k]
template <typename T>
__global__ __launch_bounds__(256) void k_nl_gw(int k, int w, const T* __restrict__ G,
                                               const T* __restrict__ W, T* __restrict__ W2) {
    const int a = blockIdx.x * 256 + threadIdx.x;
    const int j = blockIdx.y;
    if (a >= k) return;
    const T* wj = W + (int64_t)j * k;
    T s = T(0);
    for (int b = 0; b < k; ++b) s = fma(G[a + (int64_t)b * k], wj[b], s);
    W2[a + (int64_t)j * k] = s;
}

// Row-major F^T X: W[a m + c] = sum_i F[i, a] X[i m + c]; one work-group per projector and
// 64-column chunk, four row groups reduced through LDS
template <typename T>
__global__ __launch_bounds__(256) void k_nl_ftx_rm(const int64_t* __restrict__ colptr,
                                                   const int32_t* __restrict__ rowidx,
                                                   const T* __restrict__ cval, const T* __restrict__ X,
                                                   int m, T* __restrict__ W) {
    const int a = blockIdx.x;
    const int c = blockIdx.y * 64 + (threadIdx.x & 63);
    const int g = threadIdx.x >> 6;
    T acc = T(0);
    if (c < m)
        for (int64_t e = colptr[a] + g; e < colptr[a + 1]; e += 4)
            acc = fma(cval[e], X[(int64_t)rowidx[e] * m + c], acc);
    __shared__ T red[4][64];
    red[g][threadIdx.x & 63] = acc;
    __syncthreads();
    if (g == 0 && c < m)
        W[(int64_t)a * m + c] = (red[0][threadIdx.x] + red[1][threadIdx.x]) +
                                (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

// D = alpha A B + beta D, A n x k, B k x m, D n x m, all row-major; 64 x 64 output tiles,
// 16-deep operand slabs in LDS, a 4 x 4 register tile per thread
template <typename T>
__global__ __launch_bounds__(256) void k_rm_gemm(int64_t n, int k, int m, const T* __restrict__ A,
                                                 const T* __restrict__ B, T* __restrict__ D, T alpha,
                                                 T beta) {
    __shared__ T sA[16][65];
    __shared__ T sB[16][64];
    const int64_t r0 = (int64_t)blockIdx.x * 64;
    const int c0 = blockIdx.y * 64;
    const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;   // 16 x 16 threads, 4 x 4 each
    T acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = T(0);
    for (int k0 = 0; k0 < k; k0 += 16) {
        // A slab 64 x 16 (transposed into sA[kk][row]), B slab 16 x 64
        for (int e = threadIdx.x; e < 64 * 16; e += 256) {
            const int rr = e >> 4, kk = e & 15;
            const int64_t row = r0 + rr;
            sA[kk][rr] = (row < n && k0 + kk < k) ? A[row * k + k0 + kk] : T(0);
            const int br = e >> 6, bc = e & 63;
            sB[br][bc] = (k0 + br < k && c0 + bc < m) ? B[(int64_t)(k0 + br) * m + c0 + bc] : T(0);
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < 16; ++kk) {
            T a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) a[u] = sA[kk][tr * 4 + u];
#pragma unroll
            for (int v = 0; v < 4; ++v) b[v] = sB[kk][tc * 4 + v];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t row = r0 + tr * 4 + u;
        if (row >= n) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int c = c0 + tc * 4 + v;
            if (c >= m) continue;
            T* d = D + row * m + c;
            *d = beta == T(0) ? alpha * acc[u][v] : fma(alpha, acc[u][v], beta * *d);
        }
    }
}

// dst[i k + a] = F[i, a] (a dense row-major copy of F; dst zeroed first)
template <typename T>
__global__ __launch_bounds__(256) void k_nl_dense_rm(int k, const int64_t* __restrict__ colptr,
                                                     const int32_t* __restrict__ rowidx,
                                                     const T* __restrict__ cval, T* __restrict__ dst) {
    const int a = blockIdx.x;
    for (int64_t e = colptr[a] + threadIdx.x; e < colptr[a + 1]; e += 256)
        dst[(int64_t)rowidx[e] * k + a] = cval[e];
}

}  // namespace

template <typename T>
NlEpi<T, T> nl_prepare(const NonLocal& nl, const T* X, int64_t ldx, const int32_t* xcols, int w,
                       hipStream_t s) {
    if (nl.k == 0 || w <= 0) return NlEpi<T, T>{};
    const size_t need = (size_t)nl.k * w;
    T* W;
    T* W2;
    const T* cval;
    const T* G;
    if constexpr (sizeof(T) == 8) {
        nl.w64a.alloc(need);
        nl.w64b.alloc(need);
        W = nl.w64a.p; W2 = nl.w64b.p; cval = nl.cval64.p; G = nl.G64.p;
    } else {
        nl.w32a.alloc(need);
        nl.w32b.alloc(need);
        W = nl.w32a.p; W2 = nl.w32b.p; cval = nl.cval32.p; G = nl.G32.p;
    }
    hipLaunchKernelGGL((k_nl_ftx<T>), dim3(nl.k, (w + kNlCols - 1) / kNlCols), dim3(256), 0, s, nl.colptr.p,
                       nl.rowidx.p, cval, X, ldx, xcols, w, W, (int64_t)nl.k);
    hipLaunchKernelGGL((k_nl_gw<T>), dim3((nl.k + 255) / 256, w), dim3(256), 0, s, nl.k, w, G,
                       (const T*)W, W2);
    LABPSD_HIP(hipGetLastError());
    return nl.epi<T, T>(W2, nl.k);
}

template NlEpi<double, double> nl_prepare<double>(const NonLocal&, const double*, int64_t, const int32_t*, int,
                                                  hipStream_t);
template NlEpi<float, float> nl_prepare<float>(const NonLocal&, const float*, int64_t, const int32_t*, int,
                                               hipStream_t);

template <typename T>
void launch_nl_ftx_rm(const NonLocal& nl, const T* X, int m, T* W, hipStream_t s) {
    if (nl.k == 0 || m <= 0) return;
    const T* cval;
    if constexpr (sizeof(T) == 8) cval = nl.cval64.p;
    else cval = nl.cval32.p;
    hipLaunchKernelGGL((k_nl_ftx_rm<T>), dim3(nl.k, (m + 63) / 64), dim3(256), 0, s, nl.colptr.p, nl.rowidx.p,
                       cval, X, m, W);
    LABPSD_HIP(hipGetLastError());
}

template void launch_nl_ftx_rm<double>(const NonLocal&, const double*, int, double*, hipStream_t);
template void launch_nl_ftx_rm<float>(const NonLocal&, const float*, int, float*, hipStream_t);

template <typename T>
void launch_rm_gemm(int64_t n, int k, int m, const T* A, const T* B, T* D, double alpha, double beta,
                    hipStream_t s) {
    if (n <= 0 || m <= 0) return;
    const dim3 g((unsigned)((n + 63) / 64), (unsigned)((m + 63) / 64));
    hipLaunchKernelGGL((k_rm_gemm<T>), g, dim3(256), 0, s, n, k, m, A, B, D, (T)alpha, (T)beta);
    LABPSD_HIP(hipGetLastError());
}

template void launch_rm_gemm<double>(int64_t, int, int, const double*, const double*, double*, double, double,
                                     hipStream_t);
template void launch_rm_gemm<float>(int64_t, int, int, const float*, const float*, float*, double, double,
                                    hipStream_t);

// Solve T C = G (k x k, row-major) on the host by Gaussian elimination with partial pivoting
static bool solve_small(int k, std::vector<double>& T, std::vector<double>& C) {
    for (int c = 0; c < k; ++c) {
        int piv = c;
        for (int r = c + 1; r < k; ++r)
            if (std::fabs(T[(size_t)r * k + c]) > std::fabs(T[(size_t)piv * k + c])) piv = r;
        if (T[(size_t)piv * k + c] == 0.0) return false;
        if (piv != c)
            for (int j = 0; j < k; ++j) {
                std::swap(T[(size_t)piv * k + j], T[(size_t)c * k + j]);
                std::swap(C[(size_t)piv * k + j], C[(size_t)c * k + j]);
            }
        const double d = T[(size_t)c * k + c];
        for (int r = c + 1; r < k; ++r) {
            const double f = T[(size_t)r * k + c] / d;
            if (f == 0.0) continue;
            for (int j = c; j < k; ++j) T[(size_t)r * k + j] -= f * T[(size_t)c * k + j];
            for (int j = 0; j < k; ++j) C[(size_t)r * k + j] -= f * C[(size_t)c * k + j];
        }
    }
    for (int c = k - 1; c >= 0; --c) {
        const double d = T[(size_t)c * k + c];
        for (int j = 0; j < k; ++j) {
            double v = C[(size_t)c * k + j];
            for (int r = c + 1; r < k; ++r) v -= T[(size_t)c * k + r] * C[(size_t)r * k + j];
            C[(size_t)c * k + j] = v / d;
        }
    }
    return true;
}

void nonlocal_smw_setup(Problem& P) {
    NonLocal& nl = P.nl;
    nl.smw_ready = false;
    if (nl.k == 0 || !P.factor) return;
    const DevFactor& F = *P.factor;
    hipStream_t s = P.ctx->stream;
    const int64_t n = P.n;
    const int k = nl.k;
    // Fh = (H_loc - eps_bar S)^{-1} F in FP64 when the FP64 panels are there, else in FP32
    const bool f64 = F.panels64.p != nullptr;
    DBuf<double> Y, W1, Fh, M, C;
    Y.alloc((size_t)n * k);
    W1.alloc((size_t)n * k);
    Fh.alloc((size_t)n * k);
    M.alloc((size_t)k * k);
    C.alloc((size_t)k * k);
    LABPSD_HIP(hipMemsetAsync(Y.p, 0, (size_t)n * k * sizeof(double), s));
    hipLaunchKernelGGL((k_nl_dense_rm<double>), dim3(k), dim3(256), 0, s, k, nl.colptr.p, nl.rowidx.p,
                       nl.cval64.p, Y.p);
    LABPSD_HIP(hipGetLastError());
    if (f64) {
        launch_precond_solve<double>(F, Y.p, W1.p, Fh.p, n, k, s);
    } else {
        DBuf<float> y32, w32, f32;
        y32.alloc((size_t)n * k);
        w32.alloc((size_t)n * k);
        f32.alloc((size_t)n * k);
        launch_gather_cast<double, float>((int64_t)n * k, 1, Y.p, (int64_t)n * k, nullptr, 1.0, y32.p,
                                          (int64_t)n * k, s);
        launch_precond_solve<float>(F, y32.p, w32.p, f32.p, n, k, s);
        launch_gather_cast<float, double>((int64_t)n * k, 1, f32.p, (int64_t)n * k, nullptr, 1.0, Fh.p,
                                          (int64_t)n * k, s);
        LABPSD_HIP(hipStreamSynchronize(s));
    }
    check_precond_sweep(F, s);
    // T = I + G (F^T Fh); C = T^{-1} G on the host
    launch_nl_ftx_rm<double>(nl, Fh.p, k, M.p, s);
    std::vector<double> Mh((size_t)k * k), T((size_t)k * k), Ch((size_t)k * k);
    LABPSD_HIP(hipMemcpyAsync(Mh.data(), M.p, Mh.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    LABPSD_HIP(hipStreamSynchronize(s));
    for (int a = 0; a < k; ++a)
        for (int c = 0; c < k; ++c) {
            double v = a == c ? 1.0 : 0.0;
            for (int b = 0; b < k; ++b) v += nl.h_G[(size_t)a + (size_t)b * k] * Mh[(size_t)b * k + c];
            T[(size_t)a * k + c] = v;
            Ch[(size_t)a * k + c] = nl.h_G[(size_t)a + (size_t)c * k];
        }
    if (!solve_small(k, T, Ch)) throw Error{LABPSD_EINVAL, "I + G F^T (H_loc - eps_bar S)^{-1} F is singular"};
    LABPSD_HIP(hipMemcpyAsync(C.p, Ch.data(), Ch.size() * sizeof(double), hipMemcpyHostToDevice, s));
    // Ft = Fh C
    nl.Ft64.alloc((size_t)n * k);
    launch_rm_gemm<double>(n, k, k, Fh.p, C.p, nl.Ft64.p, 1.0, 0.0, s);
    nl.Ft32.alloc((size_t)n * k);
    launch_gather_cast<double, float>((int64_t)n * k, 1, nl.Ft64.p, (int64_t)n * k, nullptr, 1.0, nl.Ft32.p,
                                      (int64_t)n * k, s);
    LABPSD_HIP(hipStreamSynchronize(s));
    nl.smw_ready = true;
}

}  // namespace labpsd

using namespace labpsd;

extern "C" labpsd_status labpsd_problem_set_nonlocal(labpsd_problem* p, int k, const int64_t* colptr,
                                                     const int32_t* rowidx, const double* fval,
                                                     const double* G) {
    return abi_guard([&]() -> labpsd_status {
        LABPSD_REQUIRE(p != nullptr, "problem is NULL");
        LABPSD_REQUIRE(!p->hermitian, "the nonlocal term is real here; Hermitian problems take none");
        LABPSD_REQUIRE(k >= 0 && k <= 65536, "k out of range (0 .. 65536)");
        NonLocal& nl = p->nl;
        LABPSD_HIP(hipSetDevice(p->ctx->device));
        if (k == 0) {
            nl.k = 0;
            nl.smw_ready = false;
            return LABPSD_OK;
        }
        LABPSD_REQUIRE(colptr && rowidx && fval && G, "NULL argument");
        const int64_t n = p->n;
        LABPSD_REQUIRE(colptr[0] == 0, "colptr[0] must be 0");
        for (int a = 0; a < k; ++a) {
            LABPSD_REQUIRE(colptr[a + 1] >= colptr[a], "colptr not non-decreasing");
            for (int64_t e = colptr[a]; e < colptr[a + 1]; ++e) {
                LABPSD_REQUIRE(rowidx[e] >= 0 && rowidx[e] < n, "row index out of range in column " + std::to_string(a));
                if (e > colptr[a])
                    LABPSD_REQUIRE(rowidx[e] > rowidx[e - 1], "rows not strictly increasing in column " + std::to_string(a));
            }
        }
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < a; ++b) {
                const double x = G[a + (size_t)b * k], y = G[b + (size_t)a * k];
                LABPSD_REQUIRE(std::fabs(x - y) <= 1e-14 * (std::fabs(x) + std::fabs(y)), "G is not symmetric");
            }
        const int64_t nnz = colptr[k];
        LABPSD_REQUIRE(nnz >= 1, "F has no entries");
        LABPSD_REQUIRE(k <= n, "more projectors than rows");
        nl.k = k;
        nl.smw_ready = false;
        nl.h_colptr.assign(colptr, colptr + k + 1);
        nl.h_rowidx.assign(rowidx, rowidx + nnz);
        nl.h_cval.assign(fval, fval + nnz);
        nl.h_G.assign(G, G + (size_t)k * k);
        // the same matrix by rows
        nl.h_rowptr.assign(n + 1, 0);
        for (int64_t e = 0; e < nnz; ++e) ++nl.h_rowptr[rowidx[e] + 1];
        for (int64_t i = 0; i < n; ++i) nl.h_rowptr[i + 1] += nl.h_rowptr[i];
        nl.h_colidx.assign(nnz, 0);
        nl.h_rval.assign(nnz, 0.0);
        std::vector<int64_t> fill(nl.h_rowptr.begin(), nl.h_rowptr.end() - 1);
        for (int a = 0; a < k; ++a)
            for (int64_t e = colptr[a]; e < colptr[a + 1]; ++e) {
                const int64_t d = fill[rowidx[e]]++;
                nl.h_colidx[d] = a;
                nl.h_rval[d] = fval[e];
            }
        hipStream_t s = p->ctx->stream;
        std::vector<float> cv32(nl.h_cval.begin(), nl.h_cval.end()), rv32(nl.h_rval.begin(), nl.h_rval.end()),
            g32(nl.h_G.begin(), nl.h_G.end());
        nl.colptr.upload(nl.h_colptr.data(), nl.h_colptr.size(), s);
        nl.rowidx.upload(nl.h_rowidx.data(), std::max<size_t>(nl.h_rowidx.size(), 1), s);
        nl.cval64.upload(nl.h_cval.data(), std::max<size_t>(nl.h_cval.size(), 1), s);
        nl.cval32.upload(cv32.data(), std::max<size_t>(cv32.size(), 1), s);
        nl.rowptr.upload(nl.h_rowptr.data(), nl.h_rowptr.size(), s);
        nl.colidx.upload(nl.h_colidx.data(), std::max<size_t>(nl.h_colidx.size(), 1), s);
        nl.rval64.upload(nl.h_rval.data(), std::max<size_t>(nl.h_rval.size(), 1), s);
        nl.rval32.upload(rv32.data(), std::max<size_t>(rv32.size(), 1), s);
        nl.G64.upload(nl.h_G.data(), nl.h_G.size(), s);
        nl.G32.upload(g32.data(), g32.size(), s);
        LABPSD_HIP(hipStreamSynchronize(s));
        if (p->factor) nonlocal_smw_setup(*p);
        return LABPSD_OK;
    });
}
