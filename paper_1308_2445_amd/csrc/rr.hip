// Rayleigh-Ritz step with S-orthonormalisation (outline step 9; the conclusions ask for a
// rank-revealing treatment when [Psi P] loses rank).
//
// One work-group solves the reduced pencil (H_R, S_R) of order k:
//   1. diagonal scaling D = diag(S_R)^{-1/2}, so the scaled S_R has unit diagonal;
//   2. Cholesky of the scaled S_R (the S-orthonormalisation of the search space) and the
//      explicit inverse of its factor; if a pivot falls below 1e-14 the scaled S_R is
//      instead diagonalised and only eigen-directions above 1e-14 of its largest
//      eigenvalue are kept;
//   3. C = T^T (D H_R D) T with T = L^{-T} (or the kept scaled eigenvectors) is
//      diagonalised by the cyclic Jacobi method in round-robin order: each round applies
//      r/2 disjoint rotations at once, as independent 2 x 2 block transforms of C;
//   4. the lowest nwant eigenvalues (ascending) and W = D T V are written out.
// Matrices live in LDS when they fit, otherwise in a global workspace.
#include "common.h"

namespace labpsd {

namespace {

constexpr int kRRThreads = 1024;
constexpr double kPivotTol = 1e-14;
constexpr double kRankTol = 1e-14;

__device__ double block_sum(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[wv] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red[i];
    __syncthreads();
    return s;
}

// Cyclic Jacobi on the symmetric r x r matrix M (column-major, ld r).  V (vrows x r,
// ld ldv) is multiplied by every rotation (it holds the identity or a start basis).
// rcs holds r/2 + 1 (cos, sin) pairs and rpq the matching (p, q) index pairs.
__device__ void jacobi(double* M, int r, double* V, int ldv, int vrows, double* red, double2* rcs,
                       int2* rpq) {
    const int tid = threadIdx.x, nt = blockDim.x;
    if (r < 2) return;
    const int re = r + (r & 1);
    const int npair = re / 2;
    double f = 0.0;
    for (int j = 0; j < r; ++j)
        for (int i = tid; i < r; i += nt) f += M[i + (int64_t)j * r] * M[i + (int64_t)j * r];
    const double fro = sqrt(block_sum(f, red));
    if (fro == 0.0) return;
    const double skip = 1e-18 * fro;
    // work items of a round, spread evenly over the threads: npair^2 2 x 2 blocks and
    // npair * vrows vector pairs; the quotient by npair / vrows comes from a float
    // reciprocal (exact: the fractional part stays at least 1 / (2 npair) from an integer)
    const int nblk = npair * npair, nvec = npair * vrows;
    const float inv_np = 1.0f / (float)npair, inv_vr = 1.0f / (float)vrows;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int j = 0; j < r; ++j)
            for (int i = tid; i < r; i += nt)
                if (i != j) off += M[i + (int64_t)j * r] * M[i + (int64_t)j * r];
        off = block_sum(off, red);
        if (sqrt(off) <= 1e-13 * fro) break;
        for (int round = 0; round < re - 1; ++round) {
            for (int a = tid; a < npair; a += nt) {
                int p, q;
                if (a == 0) {
                    p = re - 1;
                    q = round;
                } else {
                    p = round + a;
                    if (p >= re - 1) p -= re - 1;
                    q = round - a;
                    if (q < 0) q += re - 1;
                }
                if (p > q) { const int t = p; p = q; q = t; }
                double c = 1.0, s = 0.0;
                if (q < r) {
                    const double apq = M[p + (int64_t)q * r];
                    if (fabs(apq) > skip) {
                        const double app = M[p + (int64_t)p * r], aqq = M[q + (int64_t)q * r];
                        const double th = (aqq - app) / (2.0 * apq);
                        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        s = t * c;
                    }
                }
                rcs[a] = make_double2(c, s);
                rpq[a] = make_int2(p, q);
            }
            __syncthreads();
            // A' = J^T A J on every 2 x 2 block (rows of pair a, columns of pair b)
            for (int e = tid; e < nblk; e += nt) {
                const int b = (int)(((float)e + 0.5f) * inv_np);
                const int a = e - b * npair;
                const double2 csa = rcs[a], csb = rcs[b];
                if (csa.y == 0.0 && csb.y == 0.0) continue;
                const int2 pqa = rpq[a], pqb = rpq[b];
                const int pa = pqa.x, qa = pqa.y, pb = pqb.x, qb = pqb.y;
                const bool va = qa < r, vb = qb < r;   // pa, pb always < r
                double m00 = M[pa + (int64_t)pb * r];
                double m01 = vb ? M[pa + (int64_t)qb * r] : 0.0;
                double m10 = va ? M[qa + (int64_t)pb * r] : 0.0;
                double m11 = (va && vb) ? M[qa + (int64_t)qb * r] : 0.0;
                // columns: (p, q) <- (c p - s q, s p + c q); then the same on rows
                const double n00 = csb.x * m00 - csb.y * m01, n01 = csb.y * m00 + csb.x * m01;
                const double n10 = csb.x * m10 - csb.y * m11, n11 = csb.y * m10 + csb.x * m11;
                m00 = csa.x * n00 - csa.y * n10;
                m10 = csa.y * n00 + csa.x * n10;
                m01 = csa.x * n01 - csa.y * n11;
                m11 = csa.y * n01 + csa.x * n11;
                if (a == b) { m01 = 0.0; m10 = 0.0; }
                M[pa + (int64_t)pb * r] = m00;
                if (vb) M[pa + (int64_t)qb * r] = m01;
                if (va) M[qa + (int64_t)pb * r] = m10;
                if (va && vb) M[qa + (int64_t)qb * r] = m11;
            }
            // V' = V J
            for (int e = tid; e < nvec; e += nt) {
                const int a = (int)(((float)e + 0.5f) * inv_vr);
                const int i = e - a * vrows;
                const double2 cs = rcs[a];
                if (cs.y == 0.0) continue;
                const int2 pq = rpq[a];
                const double vp = V[i + (int64_t)pq.x * ldv], vq = V[i + (int64_t)pq.y * ldv];
                V[i + (int64_t)pq.x * ldv] = cs.x * vp - cs.y * vq;
                V[i + (int64_t)pq.y * ldv] = cs.y * vp + cs.x * vq;
            }
            __syncthreads();
        }
    }
}

// Y = X^T Z or X Z (k x k blocks, column-major, ld k; op selects the transpose of X)
__device__ void small_gemm(const double* X, bool xt, const double* Z, bool zt, double* Y, int rows,
                           int cols, int inner, int ldx, int ldz, int ldy) {
    for (int64_t e = threadIdx.x; e < (int64_t)rows * cols; e += blockDim.x) {
        const int i = (int)(e % rows), j = (int)(e / rows);
        double acc = 0.0;
        for (int p = 0; p < inner; ++p) {
            const double x = xt ? X[p + (int64_t)i * ldx] : X[i + (int64_t)p * ldx];
            const double z = zt ? Z[j + (int64_t)p * ldz] : Z[p + (int64_t)j * ldz];
            acc = fma(x, z, acc);
        }
        Y[i + (int64_t)j * ldy] = acc;
    }
}

// ALL_LDS: every matrix and the rotation table in LDS (pointers derived from the LDS base
// only, so the compiler emits LDS instructions); otherwise lds_mask picks what fits.
template <bool ALL_LDS>
__global__ __launch_bounds__(kRRThreads) void k_rayleigh_ritz(int k, int nwant,
                                                              const double* __restrict__ HR,
                                                              const double* __restrict__ SR,
                                                              int64_t ldr, double* __restrict__ gamma,
                                                              double* __restrict__ W, int64_t ldw,
                                                              int32_t* __restrict__ info,
                                                              double* gws, int lds_mask) {
    extern __shared__ double lds[];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int64_t kk = (int64_t)k * k;
    double* small = gws + 5 * kk;
    double* D = small;                    // k
    double* theta = D + k;                // k
    double* after_theta = theta + k;
    if ((uintptr_t)after_theta & 15) after_theta += 1;   // 16-byte alignment for double2
    double2* rcs = (double2*)after_theta;          // k/2+1 rotations (cos, sin)
    int2* rpq = (int2*)(rcs + (k / 2 + 1));        //       their index pairs
    int* sel = (int*)(rpq + (k / 2 + 1));          // k
    int* flag = sel + k;                           // 4
    __shared__ double red[kRRThreads / 64];
    // placement: bit 0 the rotation table, bit 1 B (H_R, then C: the Jacobi matrix),
    // bit 2 V, bit 3 A, bit 4 T -- each in LDS when set, else in the global workspace
    if (ALL_LDS) lds_mask = 31;
    double* nextl = lds;
    if (lds_mask & 1) {
        rcs = (double2*)nextl;
        rpq = (int2*)(rcs + (k / 2 + 1));
        nextl += 3 * (k / 2 + 1);
    }
    double* B;
    double* V;
    double* A;
    double* T;
    if (ALL_LDS) {
        B = nextl;
        V = B + kk;
        A = V + kk;
        T = A + kk;
    } else {
        B = (lds_mask & 2) ? (nextl += kk) - kk : gws + kk;
        V = (lds_mask & 4) ? (nextl += kk) - kk : gws + 2 * kk;
        A = (lds_mask & 8) ? (nextl += kk) - kk : gws;
        T = (lds_mask & 16) ? (nextl += kk) - kk : gws + 3 * kk;
    }
    double* U = gws + 4 * kk;    // scratch (global)

    for (int i = tid; i < k; i += nt) {
        const double d = SR[i + (int64_t)i * ldr];
        D[i] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
    }
    if (tid == 0) { flag[0] = 0; flag[1] = 0; }
    __syncthreads();
    for (int64_t e = tid; e < kk; e += nt) {
        const int i = (int)(e % k), j = (int)(e / k);
        A[e] = D[i] * SR[i + (int64_t)j * ldr] * D[j];
        B[e] = D[i] * HR[i + (int64_t)j * ldr] * D[j];
    }
    __syncthreads();
    // Cholesky of the scaled S_R, right-looking, lower triangle in place
    for (int j = 0; j < k; ++j) {
        const double piv = A[j + (int64_t)j * k];
        if (!(piv > kPivotTol)) {
            if (tid == 0) flag[0] = 1;
            break;   // uniform: every thread read the same pivot
        }
        const double l = sqrt(piv);
        __syncthreads();
        for (int i = j + 1 + tid; i < k; i += nt) A[i + (int64_t)j * k] /= l;
        if (tid == 0) A[j + (int64_t)j * k] = l;
        __syncthreads();
        // trailing update of the lower triangle, columns over thread rows, rows over lanes
        {
            const int tx = tid & 31, ty = tid >> 5, tys = nt >> 5;
            for (int cc = j + 1 + ty; cc < k; cc += tys) {
                const double lc = A[cc + (int64_t)j * k];
                for (int i = cc + tx; i < k; i += 32) A[i + (int64_t)cc * k] -= A[i + (int64_t)j * k] * lc;
            }
        }
        __syncthreads();
    }
    __syncthreads();
    const bool fallback = flag[0] != 0;
    int r = k;
    if (!fallback) {
        // T = inv(L): one column per wavefront, forward substitution on e_c with the
        // dot product of each row spread over the lanes
        {
            const int lane = tid & 63, wave = tid >> 6, nwave = nt >> 6;
            for (int c = wave; c < k; c += nwave) {
                double* t = T + (int64_t)c * k;
                for (int i = lane; i < c; i += 64) t[i] = 0.0;
                for (int i = c; i < k; ++i) {
                    double part = 0.0;
                    for (int p = c + lane; p < i; p += 64) part += A[i + (int64_t)p * k] * t[p];
                    for (int o = 32; o > 0; o >>= 1) part += __shfl_down(part, o, 64);
                    part = __shfl(part, 0, 64);
                    if (lane == 0) t[i] = (((i == c) ? 1.0 : 0.0) - part) / A[i + (int64_t)i * k];
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                }
            }
        }
        __syncthreads();
        // C = inv(L) B inv(L)^T  (U = B inv(L)^T, then C = inv(L) U into B)
        small_gemm(B, false, T, true, U, k, k, k, k, k, k);
        __syncthreads();
        small_gemm(T, false, U, false, B, k, k, k, k, k, k);
        __syncthreads();
    } else {
        // rank-revealing: eigen-decompose the scaled S_R (V accumulates its vectors)
        for (int64_t e = tid; e < kk; e += nt) {
            const int i = (int)(e % k), j = (int)(e / k);
            A[e] = D[i] * SR[i + (int64_t)j * ldr] * D[j];
            V[e] = (i == j) ? 1.0 : 0.0;
        }
        __syncthreads();
        jacobi(A, k, V, k, k, red, rcs, rpq);
        __syncthreads();
        double mx = 0.0;
        for (int i = 0; i < k; ++i) mx = fmax(mx, A[i + (int64_t)i * k]);
        if (tid == 0) {
            int c = 0;
            for (int i = 0; i < k; ++i)
                if (A[i + (int64_t)i * k] > kRankTol * mx) sel[c++] = i;
            flag[1] = c;
        }
        __syncthreads();
        r = flag[1];
        // T = Q_keep / sqrt(lambda_keep) (k x r, ld k)
        for (int64_t e = tid; e < (int64_t)k * r; e += nt) {
            const int i = (int)(e % k), c = (int)(e / k);
            const int src = sel[c];
            T[i + (int64_t)c * k] = V[i + (int64_t)src * k] / sqrt(A[src + (int64_t)src * k]);
        }
        __syncthreads();
        // C = T^T B T (r x r, ld r) into B, via U = B T (k x r)
        small_gemm(B, false, T, false, U, k, r, k, k, k, k);
        __syncthreads();
        small_gemm(T, true, U, false, B, r, r, k, k, k, r);
        __syncthreads();
    }
    if (r < nwant) {
        if (tid == 0) { info[0] = k - r; info[1] = (int)LABPSD_ERANK; }
        return;
    }
    // symmetrise C (r x r, ld r), V = I
    for (int64_t e = tid; e < (int64_t)r * r; e += nt) {
        const int i = (int)(e % r), j = (int)(e / r);
        if (i < j) {
            const double a = 0.5 * (B[i + (int64_t)j * r] + B[j + (int64_t)i * r]);
            B[i + (int64_t)j * r] = a;
            B[j + (int64_t)i * r] = a;
        }
        V[e] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    jacobi(B, r, V, r, r, red, rcs, rpq);
    __syncthreads();
    for (int i = tid; i < r; i += nt) theta[i] = B[i + (int64_t)i * r];
    __syncthreads();
    for (int i = tid; i < r; i += nt) {
        const double ti = theta[i];
        int rank = 0;
        for (int j = 0; j < r; ++j) {
            const double tj = theta[j];
            if (tj < ti || (tj == ti && j < i)) ++rank;
        }
        if (rank < nwant) sel[rank] = i;
    }
    __syncthreads();
    for (int q = tid; q < nwant; q += nt) gamma[q] = theta[sel[q]];
    // W = D T_eff V(:, sel): T_eff = inv(L)^T (k x k) or the fallback basis (k x r)
    for (int64_t e = tid; e < (int64_t)k * nwant; e += nt) {
        const int i = (int)(e % k), q = (int)(e / k);
        const int src = sel[q];
        double acc = 0.0;
        if (!fallback) {
            for (int p = i; p < k; ++p) acc = fma(T[p + (int64_t)i * k], V[p + (int64_t)src * r], acc);
        } else {
            for (int p = 0; p < r; ++p) acc = fma(T[i + (int64_t)p * k], V[p + (int64_t)src * r], acc);
        }
        W[i + (int64_t)q * ldw] = D[i] * acc;
    }
    if (tid == 0) { info[0] = k - r; info[1] = 0; }
}

}  // namespace

size_t rr_ws_bytes(int k) {
    const size_t kk = (size_t)k * k;
    return sizeof(double) * (5 * kk + 2 * (size_t)k + 2 * (size_t)(k / 2 + 1)) +
           sizeof(int) * (2 * (size_t)(k / 2 + 1) + (size_t)k + 4) + 256;
}

void launch_rayleigh_ritz(int k, int nwant, const double* HR, const double* SR, int64_t ldr,
                          double* gamma, double* W, int64_t ldw, int32_t* info, void* ws,
                          hipStream_t s) {
    if (k <= 0 || nwant <= 0) return;
    LABPSD_REQUIRE(k <= kRRMax, "Rayleigh-Ritz order exceeds the supported maximum");
    LABPSD_REQUIRE(nwant <= k, "more Ritz pairs requested than the search space holds");
    // A, B, V, T and the rotation table in LDS when they fit the device's per-block limit
    static int lds_limit = -1;
    if (lds_limit < 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            v = 64 * 1024;
        (void)hipGetLastError();
        lds_limit = v;
    }
    // fill LDS greedily: rotation table, the Jacobi matrix, its vectors, then L and inv(L)
    const size_t mat = (size_t)k * k * sizeof(double);
    size_t bytes = (size_t)(k / 2 + 1) * 24;
    int mask = 1;
    const size_t cap = lds_limit > 2048 ? (size_t)lds_limit - 1024 : 0;
    for (int bit : {2, 4, 8, 16}) {
        if (bytes + mat <= cap) {
            bytes += mat;
            mask |= bit;
        }
    }
    if (bytes <= cap) {
        const void* fn = mask == 31 ? (const void*)k_rayleigh_ritz<true> : (const void*)k_rayleigh_ritz<false>;
        if (bytes > 64 * 1024)
            (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        (void)hipGetLastError();
        if (mask == 31)
            hipLaunchKernelGGL(k_rayleigh_ritz<true>, dim3(1), dim3(kRRThreads), bytes, s, k, nwant, HR,
                               SR, ldr, gamma, W, ldw, info, (double*)ws, mask);
        else
            hipLaunchKernelGGL(k_rayleigh_ritz<false>, dim3(1), dim3(kRRThreads), bytes, s, k, nwant, HR,
                               SR, ldr, gamma, W, ldw, info, (double*)ws, mask);
        if (hipGetLastError() == hipSuccess) return;
        // the launch was refused (nothing ran): use the global-memory variant
    }
    hipLaunchKernelGGL(k_rayleigh_ritz<false>, dim3(1), dim3(kRRThreads), 0, s, k, nwant, HR, SR, ldr,
                       gamma, W, ldw, info, (double*)ws, 0);
    LABPSD_HIP(hipGetLastError());
}

}  // namespace labpsd
