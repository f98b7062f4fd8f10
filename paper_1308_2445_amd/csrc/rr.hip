// Rayleigh-Ritz step with S-orthonormalisation (outline step 9; the conclusions ask for a
// rank-revealing treatment when [Psi P] loses rank).
//
// One work-group solves the reduced pencil (H_R, S_R) of order k:
//   1. diagonal scaling D = diag(S_R)^{-1/2}, so the scaled S_R has unit diagonal;
//   2. Cholesky of the scaled S_R (the S-orthonormalisation of the search space);
//      if a pivot falls below 1e-14 the scaled S_R is instead diagonalised by
//      Jacobi and only eigen-directions above 1e-14 of its largest eigenvalue kept;
//   3. the reduced standard matrix C = T^T (D H_R D) T with T = L^{-T} (or the kept
//      scaled eigenvectors) is diagonalised by the cyclic Jacobi method with a
//      round-robin ordering, k/2 disjoint rotations applied in parallel per round;
//   4. the lowest nwant eigenvalues (ascending) and W = D T V are written out.
// Matrices live in LDS when they fit, otherwise in a global workspace.
#include "common.h"

namespace labpsd {

namespace {

constexpr int kRRThreads = 1024;
constexpr double kPivotTol = 1e-14;
constexpr double kRankTol = 1e-14;

struct RRPtrs {
    double* A;   // scaled S_R, then its Cholesky factor (or eigenvectors in the fallback)
    double* B;   // scaled H_R, then C
    double* V;   // eigenvectors of C
    double* T;   // fallback basis (k x r)
};

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

// Cyclic Jacobi on the symmetric r x r matrix M (column-major, ld r); V (ld r)
// accumulates the rotations and must hold the identity (or a start basis) on entry.
__device__ void jacobi(double* M, double* V, int ldv, int vrows, int r, double* red, double* rc,
                       double* rs, int* rp, int* rq) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int re = r + (r & 1);
    const int npair = re / 2;
    // Frobenius norm for the thresholds
    double f = 0.0;
    for (int64_t i = tid; i < (int64_t)r * r; i += nt) f += M[i] * M[i];
    const double fro = sqrt(block_sum(f, red));
    if (fro == 0.0 || r < 2) return;
    const double skip = 1e-18 * fro;
    for (int sweep = 0; sweep < 60; ++sweep) {
        // stop once the off-diagonal part is negligible
        double off = 0.0;
        for (int64_t i = tid; i < (int64_t)r * r; i += nt) {
            const int a = (int)(i % r), b = (int)(i / r);
            if (a != b) off += M[i] * M[i];
        }
        off = block_sum(off, red);
        if (sqrt(off) <= 1e-15 * fro) break;
        for (int round = 0; round < re - 1; ++round) {
            for (int pi = tid; pi < npair; pi += nt) {
                int p, q;
                if (pi == 0) { p = re - 1; q = round; }
                else { p = (round + pi) % (re - 1); q = (round - pi + (re - 1)) % (re - 1); }
                if (p > q) { int t = p; p = q; q = t; }
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
                rc[pi] = c; rs[pi] = s; rp[pi] = p; rq[pi] = q;
            }
            __syncthreads();
            // columns of M and V
            const int64_t ncolw = (int64_t)npair * (r > vrows ? r : vrows);
            for (int64_t it = tid; it < ncolw; it += nt) {
                const int pi = (int)(it % npair);
                const int i = (int)(it / npair);
                const double s = rs[pi];
                if (s == 0.0) continue;
                const double c = rc[pi];
                const int p = rp[pi], q = rq[pi];
                if (i < r) {
                    const double mp = M[i + (int64_t)p * r], mq = M[i + (int64_t)q * r];
                    M[i + (int64_t)p * r] = c * mp - s * mq;
                    M[i + (int64_t)q * r] = s * mp + c * mq;
                }
                if (i < vrows) {
                    const double vp = V[i + (int64_t)p * ldv], vq = V[i + (int64_t)q * ldv];
                    V[i + (int64_t)p * ldv] = c * vp - s * vq;
                    V[i + (int64_t)q * ldv] = s * vp + c * vq;
                }
            }
            __syncthreads();
            // rows of M
            for (int64_t it = tid; it < (int64_t)npair * r; it += nt) {
                const int pi = (int)(it % npair);
                const int j = (int)(it / npair);
                const double s = rs[pi];
                if (s == 0.0) continue;
                const double c = rc[pi];
                const int p = rp[pi], q = rq[pi];
                const double mp = M[p + (int64_t)j * r], mq = M[q + (int64_t)j * r];
                M[p + (int64_t)j * r] = c * mp - s * mq;
                M[q + (int64_t)j * r] = s * mp + c * mq;
            }
            __syncthreads();
            for (int pi = tid; pi < npair; pi += nt) {
                if (rs[pi] != 0.0) {
                    const int p = rp[pi], q = rq[pi];
                    M[p + (int64_t)q * r] = 0.0;
                    M[q + (int64_t)p * r] = 0.0;
                }
            }
            __syncthreads();
        }
    }
}

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
    // small arrays at the end of the global workspace
    double* small = gws + 4 * kk;
    double* D = small;                    // k
    double* theta = D + k;                // k
    double* rc = theta + k;               // k/2+1
    double* rs = rc + (k / 2 + 1);
    int* rp = (int*)(rs + (k / 2 + 1));
    int* rq = rp + (k / 2 + 1);
    int* sel = rq + (k / 2 + 1);          // k
    int* flag = sel + k;                  // 4
    __shared__ double red[kRRThreads / 64];
    RRPtrs m;
    int used = 0;
    m.A = (lds_mask & 1) ? lds + (used++) * kk : gws;
    m.B = (lds_mask & 2) ? lds + (used++) * kk : gws + kk;
    m.V = (lds_mask & 4) ? lds + (used++) * kk : gws + 2 * kk;
    m.T = gws + 3 * kk;

    // 1. scaling
    for (int i = tid; i < k; i += nt) {
        const double d = SR[i + (int64_t)i * ldr];
        D[i] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
    }
    if (tid == 0) { flag[0] = 0; flag[1] = 0; }
    __syncthreads();
    for (int64_t e = tid; e < kk; e += nt) {
        const int i = (int)(e % k), j = (int)(e / k);
        m.A[e] = D[i] * SR[i + (int64_t)j * ldr] * D[j];
        m.B[e] = D[i] * HR[i + (int64_t)j * ldr] * D[j];
    }
    __syncthreads();
    // 2. Cholesky of the scaled S_R (lower, in place), right-looking
    for (int j = 0; j < k; ++j) {
        const double piv = m.A[j + (int64_t)j * k];
        if (!(piv > kPivotTol)) {
            if (tid == 0) flag[0] = 1;
            break;   // uniform: every thread reads the same pivot
        }
        const double l = sqrt(piv);
        __syncthreads();
        for (int i = j + 1 + tid; i < k; i += nt) m.A[i + (int64_t)j * k] /= l;
        __syncthreads();
        if (tid == 0) m.A[j + (int64_t)j * k] = l;
        const int64_t rem = (int64_t)(k - j - 1);
        for (int64_t it = tid; it < rem * rem; it += nt) {
            const int i = j + 1 + (int)(it % rem), c = j + 1 + (int)(it / rem);
            if (i >= c) m.A[i + (int64_t)c * k] -= m.A[i + (int64_t)j * k] * m.A[c + (int64_t)j * k];
        }
        __syncthreads();
    }
    __syncthreads();
    const bool fallback = flag[0] != 0;
    int r = k;
    if (!fallback) {
        // 3a. C = L^{-1} B L^{-T}: columns, then rows, by triangular substitution
        for (int c = tid; c < k; c += nt) {
            for (int i = 0; i < k; ++i) {
                double v = m.B[i + (int64_t)c * k];
                for (int p = 0; p < i; ++p) v -= m.A[i + (int64_t)p * k] * m.B[p + (int64_t)c * k];
                m.B[i + (int64_t)c * k] = v / m.A[i + (int64_t)i * k];
            }
        }
        __syncthreads();
        for (int rr = tid; rr < k; rr += nt) {
            for (int i = 0; i < k; ++i) {
                double v = m.B[rr + (int64_t)i * k];
                for (int p = 0; p < i; ++p) v -= m.A[i + (int64_t)p * k] * m.B[rr + (int64_t)p * k];
                m.B[rr + (int64_t)i * k] = v / m.A[i + (int64_t)i * k];
            }
        }
        __syncthreads();
    } else {
        // 3b. rank-revealing: eigen-decompose the scaled S_R
        for (int64_t e = tid; e < kk; e += nt) {
            const int i = (int)(e % k), j = (int)(e / k);
            m.A[e] = D[i] * SR[i + (int64_t)j * ldr] * D[j];
            m.T[e] = (i == j) ? 1.0 : 0.0;
        }
        __syncthreads();
        jacobi(m.A, m.T, k, k, k, red, rc, rs, rp, rq);
        __syncthreads();
        double mx = 0.0;
        for (int i = 0; i < k; ++i) mx = fmax(mx, m.A[i + (int64_t)i * k]);
        // kept directions, in index order
        if (tid == 0) {
            int c = 0;
            for (int i = 0; i < k; ++i)
                if (m.A[i + (int64_t)i * k] > kRankTol * mx) sel[c++] = i;
            flag[1] = c;
        }
        __syncthreads();
        r = flag[1];
        // T_keep = Q_keep / sqrt(lambda) into V (k x r), then Y = B T_keep into A
        for (int64_t e = tid; e < (int64_t)k * r; e += nt) {
            const int i = (int)(e % k), c = (int)(e / k);
            const int src = sel[c];
            m.V[i + (int64_t)c * k] = m.T[i + (int64_t)src * k] / sqrt(m.A[src + (int64_t)src * k]);
        }
        __syncthreads();
        for (int64_t e = tid; e < (int64_t)k * r; e += nt) {
            const int i = (int)(e % k), c = (int)(e / k);
            double v = 0.0;
            for (int p = 0; p < k; ++p) v += m.B[i + (int64_t)p * k] * m.V[p + (int64_t)c * k];
            m.A[i + (int64_t)c * k] = v;
        }
        __syncthreads();
        // C = T_keep^T Y (r x r, ld r) into B; keep T_keep in T
        for (int64_t e = tid; e < (int64_t)r * r; e += nt) {
            const int i = (int)(e % r), j = (int)(e / r);
            double v = 0.0;
            for (int p = 0; p < k; ++p) v += m.V[p + (int64_t)i * k] * m.A[p + (int64_t)j * k];
            m.B[e] = v;
        }
        for (int64_t e = tid; e < (int64_t)k * r; e += nt) m.T[e] = m.V[e];
        __syncthreads();
        for (int64_t e = tid; e < (int64_t)r * r; e += nt) {
            const int i = (int)(e % r), j = (int)(e / r);
            if (i < j) {
                const double a = 0.5 * (m.B[e] + m.B[j + (int64_t)i * r]);
                m.B[e] = a;
                m.B[j + (int64_t)i * r] = a;
            }
        }
        __syncthreads();
    }
    if (r < nwant) {
        if (tid == 0) { info[0] = k - r; info[1] = (int)LABPSD_ERANK; }
        return;
    }
    // symmetrise C (r x r, ld r) and reset V to the identity
    for (int64_t e = tid; e < (int64_t)r * r; e += nt) {
        const int i = (int)(e % r), j = (int)(e / r);
        if (i < j) {
            const double a = 0.5 * (m.B[i + (int64_t)j * r] + m.B[j + (int64_t)i * r]);
            m.B[i + (int64_t)j * r] = a;
            m.B[j + (int64_t)i * r] = a;
        }
        m.V[e] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    // 4. eigen-decomposition of C
    jacobi(m.B, m.V, r, r, r, red, rc, rs, rp, rq);
    __syncthreads();
    for (int i = tid; i < r; i += nt) theta[i] = m.B[i + (int64_t)i * r];
    __syncthreads();
    // ascending order: rank of every eigenvalue
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
    if (!fallback) {
        // W(:, q) = D L^{-T} V(:, sel[q]) by back substitution, one column per thread
        for (int q = tid; q < nwant; q += nt) {
            const int src = sel[q];
            double* wq = W + (int64_t)q * ldw;
            for (int i = k - 1; i >= 0; --i) {
                double v = m.V[i + (int64_t)src * r];
                for (int p = i + 1; p < k; ++p) v -= m.A[p + (int64_t)i * k] * wq[p];
                wq[i] = v / m.A[i + (int64_t)i * k];
            }
        }
        __syncthreads();
        for (int64_t e = tid; e < (int64_t)k * nwant; e += nt) {
            const int i = (int)(e % k), q = (int)(e / k);
            W[i + (int64_t)q * ldw] *= D[i];
        }
    } else {
        for (int64_t e = tid; e < (int64_t)k * nwant; e += nt) {
            const int i = (int)(e % k), q = (int)(e / k);
            const int src = sel[q];
            double v = 0.0;
            for (int p = 0; p < r; ++p) v += m.T[i + (int64_t)p * k] * m.V[p + (int64_t)src * r];
            W[i + (int64_t)q * ldw] = D[i] * v;
        }
    }
    if (tid == 0) { info[0] = k - r; info[1] = 0; }
}

}  // namespace

size_t rr_ws_bytes(int k) {
    const size_t kk = (size_t)k * k;
    return sizeof(double) * (4 * kk + 2 * (size_t)k + 2 * (size_t)(k / 2 + 1)) +
           sizeof(int) * (2 * (size_t)(k / 2 + 1) + (size_t)k + 4) + 256;
}

void launch_rayleigh_ritz(int k, int nwant, const double* HR, const double* SR, int64_t ldr,
                          double* gamma, double* W, int64_t ldw, int32_t* info, void* ws,
                          hipStream_t s) {
    if (k <= 0 || nwant <= 0) return;
    LABPSD_REQUIRE(k <= kRRMax, "Rayleigh-Ritz order exceeds the supported maximum");
    LABPSD_REQUIRE(nwant <= k, "more Ritz pairs requested than the search space holds");
    // LDS holds the scaled H_R / C and the eigenvectors when they fit
    const size_t kk = (size_t)k * k * sizeof(double);
    const size_t lds_cap = 160 * 1024 - 4096;
    int mask = 0;
    size_t lds = 0;
    if (3 * kk <= lds_cap) { mask = 1 | 2 | 4; lds = 3 * kk; }
    else if (2 * kk <= lds_cap) { mask = 2 | 4; lds = 2 * kk; }
    else if (kk <= lds_cap) { mask = 2; lds = kk; }
    if (lds > 0 &&
        hipFuncSetAttribute((const void*)k_rayleigh_ritz, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds) != hipSuccess) {
        (void)hipGetLastError();
        mask = 0;
        lds = 0;
    }
    hipLaunchKernelGGL(k_rayleigh_ritz, dim3(1), dim3(kRRThreads), lds, s, k, nwant, HR, SR, ldr,
                       gamma, W, ldw, info, (double*)ws, mask);
    LABPSD_HIP(hipGetLastError());
}

}  // namespace labpsd
