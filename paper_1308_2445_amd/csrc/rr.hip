// Rayleigh-Ritz step with S-orthonormalisation (outline step 9; the conclusions ask for a
// rank-revealing treatment when [Psi P] loses rank).
//
// One work-group solves the reduced pencil (H_R, S_R) of order k for its lowest nwant
// pairs:
//   1. diagonal scaling D = diag(S_R)^{-1/2}, so the scaled S_R has unit diagonal;
//   2. Cholesky L L^T of the scaled S_R (the S-orthonormalisation of the search space),
//      right-looking with one barrier per column;
//   3. C = L^{-1} (D H_R D) L^{-T} by two right-looking triangular solves;
//   4. the lowest nwant eigenpairs of C: Householder reduction to tridiagonal form,
//      eigenvalues by multisection on Sturm counts, eigenvectors by inverse iteration
//      with the tridiagonal LU (partial pivoting) and Gram-Schmidt inside clusters of
//      close eigenvalues, then the reflectors applied back;
//   5. W = D L^{-T} Z by back substitution.
// If a Cholesky pivot falls below 1e-14 the scaled S_R is instead diagonalised (cyclic
// Jacobi) and only its eigen-directions above 1e-14 of the largest eigenvalue are kept;
// C on that basis is diagonalised by cyclic Jacobi as well.
// Everything lives in LDS when it fits the per-block limit, otherwise in a global
// workspace.  Orders above 128 take the same steps on many work-groups (the "large
// orders" section below), with the one-work-group kernel as their fallback.
#include <type_traits>

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
        for (int i = tid; i < r; i += nt) f += M[i + j * r] * M[i + j * r];
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
                if (i != j) off += M[i + j * r] * M[i + j * r];
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
                    const double apq = M[p + q * r];
                    if (fabs(apq) > skip) {
                        const double app = M[p + p * r], aqq = M[q + q * r];
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
                double m00 = M[pa + pb * r];
                double m01 = vb ? M[pa + qb * r] : 0.0;
                double m10 = va ? M[qa + pb * r] : 0.0;
                double m11 = (va && vb) ? M[qa + qb * r] : 0.0;
                // columns: (p, q) <- (c p - s q, s p + c q); then the same on rows
                const double n00 = csb.x * m00 - csb.y * m01, n01 = csb.y * m00 + csb.x * m01;
                const double n10 = csb.x * m10 - csb.y * m11, n11 = csb.y * m10 + csb.x * m11;
                m00 = csa.x * n00 - csa.y * n10;
                m10 = csa.y * n00 + csa.x * n10;
                m01 = csa.x * n01 - csa.y * n11;
                m11 = csa.y * n01 + csa.x * n11;
                if (a == b) { m01 = 0.0; m10 = 0.0; }
                M[pa + pb * r] = m00;
                if (vb) M[pa + qb * r] = m01;
                if (va) M[qa + pb * r] = m10;
                if (va && vb) M[qa + qb * r] = m11;
            }
            // V' = V J
            for (int e = tid; e < nvec; e += nt) {
                const int a = (int)(((float)e + 0.5f) * inv_vr);
                const int i = e - a * vrows;
                const double2 cs = rcs[a];
                if (cs.y == 0.0) continue;
                const int2 pq = rpq[a];
                const double vp = V[i + pq.x * ldv], vq = V[i + pq.y * ldv];
                V[i + pq.x * ldv] = cs.x * vp - cs.y * vq;
                V[i + pq.y * ldv] = cs.y * vp + cs.x * vq;
            }
            __syncthreads();
        }
    }
}

// Y = X^T Z or X Z (k x k blocks, column-major, ld k; op selects the transpose of X)
__device__ void small_gemm(const double* X, bool xt, const double* Z, bool zt, double* Y, int rows,
                           int cols, int inner, int ldx, int ldz, int ldy) {
    for (int e = threadIdx.x; e < rows * cols; e += blockDim.x) {
        const int i = (int)(e % rows), j = (int)(e / rows);
        double acc = 0.0;
        for (int p = 0; p < inner; ++p) {
            const double x = xt ? X[p + i * ldx] : X[i + p * ldx];
            const double z = zt ? Z[j + p * ldz] : Z[p + j * ldz];
            acc = fma(x, z, acc);
        }
        Y[i + j * ldy] = acc;
    }
}

// 1 / x and 1 / sqrt(x) from the hardware approximations with two Newton steps
// (within an ulp or two, without the long IEEE division sequence)
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ double rsq_nr(double x) {
    double r = __builtin_amdgcn_rsq(x);
    r = r * fma(-0.5 * x * r, r, 1.5);
    return r * fma(-0.5 * x * r, r, 1.5);
}

typedef double rr_double4 __attribute__((ext_vector_type(4)));

// C = op(A) op(B) (m x n, inner kd) with the FP64 16x16x4 MFMA, one 16 x 16 tile per
// wavefront at a time; op(A)[i, p] = ta ? A[p + i lda] : A[i + p lda], op(B)[p, j] =
// tb ? B[j + p ldb] : B[p + j ldb]; store(i, j, v) receives every element.
template <typename Store>
__device__ void gemm_mfma(const double* A, int lda, bool ta, const double* B, int ldb, bool tb, int m,
                          int n, int kd, Store store) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
    const int tm = (m + 15) / 16, tn = (n + 15) / 16;
    for (int t = wave; t < tm * tn; t += nwave) {
        const int i0 = (t % tm) * 16, j0 = (t / tm) * 16;
        rr_double4 acc = {0.0, 0.0, 0.0, 0.0};
        const int ar = i0 + (lane & 15), bc = j0 + (lane & 15), kq = lane >> 4;
        for (int p0 = 0; p0 < kd; p0 += 4) {
            const int pk = p0 + kq;
            double a = 0.0, b = 0.0;
            if (ar < m && pk < kd) a = ta ? A[pk + ar * lda] : A[ar + pk * lda];
            if (bc < n && pk < kd) b = tb ? B[bc + pk * ldb] : B[pk + bc * ldb];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
        // accumulator layout: register q of lane l holds row 4q + l / 16, column l % 16
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = i0 + 4 * q + (lane >> 4), j = j0 + (lane & 15);
            if (i < m && j < n) store(i, j, acc[q]);
        }
    }
}

// Right-looking Cholesky of the r x r matrix A (lower triangle, column-major, ld r) in
// place, one barrier per column: step j updates the trailing matrix with the unscaled
// column j and scales column j - 1, which no thread of step j reads.  invd receives
// 1 / L[j, j].  Returns false (uniformly) at the first pivot not above kPivotTol.
__device__ bool cholesky_rl(double* A, int r, double* invd) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, nwave = nt >> 6;
    double il_prev = 0.0, l_prev = 0.0;
    for (int j = 0; j < r; ++j) {
        const double piv = A[j + j * r];
        if (!(piv > kPivotTol)) return false;
        const double il = rsq_nr(piv);
        const double ip = il * il;
        if (j > 0) {
            for (int i = j + tid; i < r; i += nt) A[i + (j - 1) * r] *= il_prev;
            if (tid == 0) {
                A[(j - 1) + (j - 1) * r] = l_prev;
                invd[j - 1] = il_prev;
            }
        }
        for (int c = j + 1 + wave; c < r; c += nwave) {
            const double acj = A[c + j * r] * ip;
            for (int i = c + lane; i < r; i += 64) A[i + c * r] -= A[i + j * r] * acj;
        }
        il_prev = il;
        l_prev = piv * il;
        __syncthreads();
    }
    if (tid == 0) {
        A[(r - 1) + (r - 1) * r] = l_prev;
        invd[r - 1] = il_prev;
    }
    return true;
}

// X = L^{-1} (lower triangular, column-major, ld r) by right-looking substitution on the
// identity, one barrier per row: step j eliminates row j (scaled by invd[j]) from the
// rows below and scales row j - 1.
__device__ void invert_lower_rl(const double* L, const double* invd, double* X, int r) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, nwave = nt >> 6;
    for (int e = tid; e < r * r; e += nt) {
        const int i = (int)(e % r), c = (int)(e / r);
        X[e] = (i == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int j = 0; j < r; ++j) {
        const double ij = invd[j];
        if (j > 0) {
            const double ip = invd[j - 1];
            for (int c = tid; c < j; c += nt) X[(j - 1) + c * r] *= ip;
        }
        for (int c = wave; c <= j; c += nwave) {
            const double xjc = X[j + c * r] * ij;
            for (int i = j + 1 + lane; i < r; i += 64) X[i + c * r] -= L[i + j * r] * xjc;
        }
        __syncthreads();
    }
    const double ip = invd[r - 1];
    for (int c = tid; c < r; c += nt) X[(r - 1) + c * r] *= ip;
}

// B <- (B + B^T) / 2 in place
__device__ void symmetrize(double* B, int r) {
    for (int e = threadIdx.x; e < r * r; e += blockDim.x) {
        const int i = (int)(e % r), j = (int)(e / r);
        if (i < j) {
            const double m = 0.5 * (B[i + j * r] + B[j + i * r]);
            B[i + j * r] = m;
            B[j + i * r] = m;
        }
    }
}

// Reflector that maps column j's tail B[j+1.., j] to (beta, 0, ...): H = I - tau v v^T,
// v = (1, v_{j+2}, ...), from alpha = B[j+1, j] and sigma = |B[j+2.., j]|^2.
__device__ __forceinline__ void reflector(double alpha, double sigma, double& tau, double& beta,
                                          double& scal) {
    tau = 0.0;
    beta = alpha;
    scal = 0.0;
    if (sigma != 0.0) {
        beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
        tau = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
    }
}

// The same reflector from one reciprocal square root and one reciprocal (Newton-refined
// hardware approximations): with nrm = |(alpha, x)|, beta = -sign(alpha) nrm,
// tau = 1 + |alpha| / nrm and scal = 1 / (alpha - beta) = sign(alpha) / (|alpha| + nrm).
// tau matches 2 / (v^T v) for v = (1, scal x) to a few ulps.
__device__ __forceinline__ void reflector_fast(double alpha, double sigma, double& tau, double& beta,
                                               double& scal) {
    tau = 0.0;
    beta = alpha;
    scal = 0.0;
    if (sigma != 0.0) {
        const double s2 = fma(alpha, alpha, sigma);
        const double rs = rsq_nr(s2);
        const double nrm = s2 * rs;
        const double aa = fabs(alpha);
        beta = -copysign(nrm, alpha);
        tau = fma(aa, rs, 1.0);
        scal = copysign(rcp_nr(aa + nrm), alpha);
    }
}

// Householder reduction of the symmetric r x r matrix B (both triangles stored) to
// tridiagonal form Q^T B Q = T (diagonal d, off-diagonal e), with Q = H_0 H_1 ... and
// H_j = I - tau_j v v^T on rows j+1..r-1, v = (1, v_{j+2}, ...).  The reflectors are
// accumulated on the right of M (r x r, row-major: M[i, c] at i r + c), M <- M H_j.
// Two barriers per reflector:
//   products  p = tau A22 v and M v, 8 lanes per row (A22 is symmetric, so row i is
//             read as column i), the terms of p . v stored per row;
//   updates   wavefront 0 updates column j + 1 of A22 and builds the next reflector from
//             it (vb double buffer of 2 r doubles; sc[2 s], sc[2 s + 1]: tau, beta); the
//             other wavefronts apply A22 -= v w^T + w v^T, w = p - (tau/2)(p . v) v, to
//             columns j + 2.. and M -= tau (M v) v^T, two columns or rows per batch with
//             every load issued before the stores.
// pA, pM, pv: r doubles each.
__device__ void tridiagonalize_acc(double* B, double* M, int r, double* d, double* e, double* vb,
                                   double* pA, double* pM, double* pv, double* sc) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, nwave = nt >> 6;
    if (r == 1) {
        if (tid == 0) d[0] = B[0];
        return;
    }
    if (r >= 3 && wave == 0) {
        double sg = 0.0, a1 = 0.0;
        for (int i = 1 + lane; i < r; i += 64) {
            const double x = B[i];
            if (i >= 2) sg += x * x;
            if (i == 1) a1 = x;
        }
        const double sigma = wave_allsum(sg), alpha = wave_allsum(a1);
        double t, beta, scal;
        reflector(alpha, sigma, t, beta, scal);
        for (int i = 1 + lane; i < r; i += 64) vb[i] = (i == 1) ? 1.0 : B[i] * scal;
        if (lane == 0) {
            sc[0] = t;
            sc[1] = beta;
        }
    }
    __syncthreads();
    const int g = tid >> 3, sub = tid & 7, ng = nt >> 3;
    const int w1 = wave - 1, nw1 = nwave - 1;   // the update wavefronts other than 0
    for (int j = 0; j + 2 < r; ++j) {
        const int s0 = j & 1, s1 = s0 ^ 1;
        const double t = sc[2 * s0], beta = sc[2 * s0 + 1];
        const bool refl = t != 0.0;   // uniform: every thread read the same tau
        const double* v = vb + s0 * r;
        if (refl) {
            // row tasks: A22 rows j+1..r-1, then M rows 0..r-1
            const int na = r - j - 1;
            for (int task = g; task < na + r; task += ng) {
                const bool isa = task < na;
                const int i = isa ? j + 1 + task : task - na;
                const double* src = isa ? B + i * r : M + i * r;
                double part = 0.0;
#pragma unroll 4
                for (int c = j + 1 + sub; c < r; c += 8) part = fma(src[c], v[c], part);
                part = row8_allsum(part);
                if (sub == 0) {
                    if (isa) {
                        const double pi = t * part;
                        pA[i] = pi;
                        pv[i] = pi * v[i];
                    } else {
                        pM[i] = part;
                    }
                }
            }
        }
        if (tid == 0) {
            d[j] = B[j + j * r];
            e[j] = beta;
        }
        __syncthreads();
        double K = 0.0;
        if (refl) {
            double part = 0.0;
            for (int i = j + 1 + lane; i < r; i += 64) part += pv[i];
            K = 0.5 * t * wave_allsum(part);
        }
        if (wave == 0) {
            // column j + 1, then the next reflector from it
            const int c = j + 1;
            const double vc = 1.0;
            const double wc = refl ? pA[c] - K * vc : 0.0;
            double* colc = B + c * r;
            double sg = 0.0, a1 = 0.0;
            for (int i = j + 1 + lane; i < r; i += 64) {
                double x = colc[i];
                if (refl) {
                    const double vi = v[i];
                    x -= vi * wc + (pA[i] - K * vi) * vc;
                    colc[i] = x;
                }
                if (i >= j + 3) sg += x * x;
                if (i == j + 2) a1 = x;
            }
            if (j + 3 < r) {
                const double sigma = wave_allsum(sg), alpha = wave_allsum(a1);
                double t2, beta2, scal2;
                reflector(alpha, sigma, t2, beta2, scal2);
                double* vn = vb + s1 * r;
                // each lane reads back only the rows it wrote above
                for (int i = j + 1 + lane; i < r; i += 64)
                    if (i >= j + 2) vn[i] = (i == j + 2) ? 1.0 : colc[i] * scal2;
                if (lane == 0) {
                    sc[2 * s1] = t2;
                    sc[2 * s1 + 1] = beta2;
                }
            }
        } else if (refl) {
            // A22 columns j+2..r-1: lanes over rows, two columns per batch
            for (int i0 = j + 1; i0 < r; i0 += 64) {
                const int i = i0 + lane;
                const bool okr = i < r;
                const double vi = okr ? v[i] : 0.0;
                const double wi = okr ? pA[i] - K * vi : 0.0;
                for (int c0 = j + 2 + 2 * w1; c0 < r; c0 += 2 * nw1) {
                    double x[2], vc[2], wc[2];
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const int c = c0 + q;
                        const bool okc = c < r;
                        vc[q] = okc ? v[c] : 0.0;
                        wc[q] = okc ? pA[c] - K * vc[q] : 0.0;
                        x[q] = (okr && okc) ? B[i + c * r] : 0.0;
                    }
#pragma unroll
                    for (int q = 0; q < 2; ++q)
                        if (okr && c0 + q < r) B[i + (c0 + q) * r] = x[q] - (vi * wc[q] + wi * vc[q]);
                }
            }
            // M rows 0..r-1, columns j+1..r-1: lanes over columns, two rows per batch
            for (int cb = j + 1; cb < r; cb += 64) {
                const int c = cb + lane;
                const bool okc = c < r;
                const double tv = okc ? t * v[c] : 0.0;
                for (int i0 = 2 * w1; i0 < r; i0 += 2 * nw1) {
                    double x[2], mi[2];
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const int i = i0 + q;
                        const bool oki = i < r;
                        mi[q] = oki ? pM[i] : 0.0;
                        x[q] = (oki && okc) ? M[i * r + c] : 0.0;
                    }
#pragma unroll
                    for (int q = 0; q < 2; ++q)
                        if (okc && i0 + q < r) M[(i0 + q) * r + c] = x[q] - mi[q] * tv;
                }
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        d[r - 2] = B[(r - 2) + (r - 2) * r];
        d[r - 1] = B[(r - 1) + (r - 1) * r];
        e[r - 2] = B[(r - 1) + (r - 2) * r];
    }
}

// ---------------------------------------------------------------- register-row routines
// For r <= 8 NT the dense phases keep the matrix rows in registers: the 8 lanes of group
// g = tid / 8 own row g, lane sub = tid % 8 the columns sub + 8 t (t < NT; zero at and
// beyond r).  Only the vectors one step hands to the next pass through memory, in
// buffers of P = 8 NT doubles whose entries at and beyond r stay zero, so that every
// lane reads and writes its columns at fixed offsets without bounds tests.

// Cholesky L L^T of D S_R D (read from S_R) fused with X = L^{-1}, right-looking: row j,
// once updated by steps 0..j-1, gives column j of L (by symmetry of the trailing matrix)
// and, scaled, the final row j of X; every later row then subtracts L[g, j] times both.
// One barrier per step.  X is written column-major (ld r).  buf: 4 P doubles; piv: 2.
// Entries of a row left of the current column are dead and take harmless updates.
// Returns false (uniformly) at the first pivot not above kPivotTol.
template <int NT>
__device__ __forceinline__ bool chol_inv_regs(const double* __restrict__ SR, int64_t ldr, const double* D, int r,
                              double* X, double* buf, double* piv) {
    constexpr int P = 8 * NT;
    const int tid = threadIdx.x, g = tid >> 3, sub = tid & 7;
    const bool row = g < r;
    double a[NT], x[NT];
    const double dg = row ? D[g] : 0.0;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int c = sub + 8 * t;
        const bool ok = row && c < r;
        a[t] = ok ? dg * SR[c + (int64_t)g * ldr] * D[c] : 0.0;
        x[t] = (ok && c == g) ? 1.0 : 0.0;
    }
    auto publish = [&](int j) {   // by the 8 lanes of group j
        double* lb = buf + (j & 1) * P + sub;       // column j of L
        double* xb = buf + (2 + (j & 1)) * P + sub; // row j of X
        // the pivot sits in column j: slot j / 8 of the lane with sub = j % 8
        double sel = a[0];
#pragma unroll
        for (int t = 1; t < NT; ++t)
            if (t == (j >> 3)) sel = a[t];
        const double p = readlane_d(sel, 8 * (j & 7) + (j & 7));
        const double il = p > kPivotTol ? rsq_nr(p) : 0.0;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            lb[8 * t] = sub + 8 * t >= j ? a[t] * il : 0.0;
            x[t] *= il;
            xb[8 * t] = x[t];
        }
        if (sub == 0) piv[j & 1] = p;
    };
    if (g == 0) publish(0);
    __syncthreads();
    for (int j = 0; j < r; ++j) {
        if (!(piv[j & 1] > kPivotTol)) return false;
        // the wavefront holding row j + 1 publishes the next step: it goes first
        const bool lead = __builtin_amdgcn_readfirstlane((tid >> 6) == ((j + 1) >> 3) ? 1 : 0) != 0;
        if (lead) __builtin_amdgcn_s_setprio(2);
        if (row && g > j) {
            const double* lb = buf + (j & 1) * P;
            const double* xb = buf + (2 + (j & 1)) * P + sub;
            const double lgj = lb[g];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                a[t] = fma(-lgj, lb[sub + 8 * t], a[t]);
                x[t] = fma(-lgj, xb[8 * t], x[t]);
            }
        }
        if (g == j + 1 && j + 1 < r) publish(j + 1);
        if (lead) __builtin_amdgcn_s_setprio(0);
        __syncthreads();
    }
    if (row) {
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int c = sub + 8 * t;
            if (c < r) X[g + c * r] = x[t];
        }
    }
    return true;
}

// Householder tridiagonalisation Q^T C Q = T with Q = H_0 H_1 ... accumulated onto
// M = X^T (M <- M H_j), rows of C and M in registers.  Per reflector j (support rows
// j+1..r-1, v = (1, v_{j+2}, ...)): each row forms its part of p = tau C v and of M v
// (8-lane sums) and updates its row of M at once; after one barrier every row applies
// C -= v w^T + w v^T, w = p - (tau/2)(p . v) v, and row j + 1 builds the next reflector;
// a second barrier publishes it.  C is read column-major and symmetrised on the way
// in; T holds X column-major on entry and M row-major on exit.  buf: 3 P doubles;
// sc: 4 (tau, beta of the two reflector buffers).
template <int NT>
__device__ __forceinline__ void tridiag_regs(const double* C, double* T, int r, double* d, double* e, double* buf,
                             double* sc) {
    constexpr int P = 8 * NT;
    const int tid = threadIdx.x, g = tid >> 3, sub = tid & 7, lane = tid & 63;
    const bool row = g < r;
    double a[NT], m[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int c = sub + 8 * t;
        const bool ok = row && c < r;
        a[t] = ok ? 0.5 * (C[c + g * r] + C[g + c * r]) : 0.0;
        m[t] = ok ? T[c + g * r] : 0.0;   // row g of M = X^T is column g of X
    }
    double* pb = buf + 2 * P;   // p; buf[0..2P): the two reflector buffers
    if (tid < P) pb[tid] = 0.0;
    // reflector j1 from row j1 (= column j1), by the 8 lanes of that group
    auto next_reflector = [&](int j1) {
        const int s = j1 & 1;
        double sg0 = 0.0, sg1 = 0.0, sel = a[0];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const double x = sub + 8 * t > j1 + 1 ? a[t] : 0.0;
            if (t & 1) sg1 = fma(x, x, sg1);
            else sg0 = fma(x, x, sg0);
            if (t > 0 && t == ((j1 + 1) >> 3)) sel = a[t];
        }
        const double sg = row8_allsum(sg0 + sg1);
        // alpha = C[j1, j1 + 1]: slot (j1 + 1) / 8 of the lane with sub = (j1 + 1) % 8
        const double a1 = readlane_d(sel, 8 * (j1 & 7) + ((j1 + 1) & 7));
        double tau, beta, scal;
        reflector_fast(a1, sg, tau, beta, scal);
        double* vn = buf + s * P + sub;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int c = sub + 8 * t;
            vn[8 * t] = c == j1 + 1 ? 1.0 : (c > j1 + 1 ? a[t] * scal : 0.0);
        }
        if (sub == 0) {
            sc[2 * s] = tau;
            sc[2 * s + 1] = beta;
        }
    };
    if (r >= 3 && g == 0) next_reflector(0);
    __syncthreads();
    for (int j = 0; j + 2 < r; ++j) {
        const int s0 = j & 1;
        const double tau = sc[2 * s0];
        const bool refl = tau != 0.0;   // uniform
        const double* v = buf + s0 * P;
        if (g == j) {
#pragma unroll
            for (int t = 0; t < NT; ++t)
                if (sub + 8 * t == j) d[j] = a[t];
            if (sub == 0) e[j] = sc[2 * s0 + 1];
        }
        double vt[NT];
        double pg = 0.0;
        // wavefronts without rows only take part in the barriers; rows up to j need only
        // their row of M
        if (refl && row) {
#pragma unroll
            for (int t = 0; t < NT; ++t) vt[t] = v[sub + 8 * t];
            double pm0 = 0.0, pm1 = 0.0, pa0 = 0.0, pa1 = 0.0;
#pragma unroll
            for (int t = 0; t < NT; t += 2) {
                pm0 = fma(m[t], vt[t], pm0);
                pa0 = fma(a[t], vt[t], pa0);
                if (t + 1 < NT) {
                    pm1 = fma(m[t + 1], vt[t + 1], pm1);
                    pa1 = fma(a[t + 1], vt[t + 1], pa1);
                }
            }
            const double pa = row8_allsum(pa0 + pa1), pm = row8_allsum(pm0 + pm1);
            if (g > j) pg = tau * pa;
            const double tm = tau * pm;
#pragma unroll
            for (int t = 0; t < NT; ++t) m[t] = fma(-tm, vt[t], m[t]);
            if (sub == 0) pb[g] = pg;
        }
        __syncthreads();
        // the wavefront holding row j + 1 builds the next reflector: it goes first
        const bool lead = __builtin_amdgcn_readfirstlane((tid >> 6) == ((j + 1) >> 3) ? 1 : 0) != 0;
        if (lead) __builtin_amdgcn_s_setprio(2);
        if (refl && 8 * (tid >> 6) < r) {
            double part = 0.0;
#pragma unroll
            for (int i = lane; i < P; i += 64) part = fma(pb[i], v[i], part);
            const double K = 0.5 * tau * wave_allsum(part);
            if (row && g > j) {
                // C -= v w^T + w v^T = (v p^T + p v^T) - 2 K v v^T
                const double vg = v[g];
                const double k2 = 2.0 * K * vg;
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const double u = fma(vg, pb[sub + 8 * t], pg * vt[t]);
                    a[t] = fma(k2, vt[t], a[t] - u);
                }
            }
        }
        if (j + 3 < r && g == j + 1) next_reflector(j + 1);
        if (lead) __builtin_amdgcn_s_setprio(0);
        __syncthreads();
    }
    // the trailing 2 x 2 (or 1 x 1) block
    if (row && g >= r - 2) {
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int c = sub + 8 * t;
            if (c == g) d[g] = a[t];
            if (g == r - 1 && c == r - 2) e[r - 2] = a[t];
        }
    }
    __syncthreads();
    if (row) {
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int c = sub + 8 * t;
            if (c < r) T[g * r + c] = m[t];
        }
    }
}

constexpr double kEps = 1.1102230246251565e-16;      // 2^-53
constexpr double kSafmin = 2.2250738585072014e-308;

// number of eigenvalues of T below x: sign changes of the Sturm sequence p_0 = 1,
// p_1 = d_0 - x, p_i = (d_{i-1} - x) p_{i-1} - e_{i-2}^2 p_{i-2} (the leading principal
// minors of T - x I; p_i / p_{i-1} is the i-th pivot of its LDL^T, so a sign change is a
// negative pivot).  The sequence is that of s T (s a power of two near 1 / ||T||, e2s
// holding (s e)^2), so every step changes the magnitude by a factor of order one.  One
// fused multiply-add per step is on the dependent chain, with no division; every fourth
// step p_{i-1}, p_{i-2} are rescaled by the same power of two (the larger to [0.5, 1)) to
// keep them in range.  An exact zero is replaced by a value of the opposite sign to its
// predecessor, tiny relative to it (the zero-pivot convention: it counts as negative).
__device__ int sturm_count(const double* d, const double* e2s, int r, double x, double s) {
    constexpr double kZeroRel = 0x1p-80;
    double p2 = 1.0, p1 = (d[0] - x) * s;
    if (p1 == 0.0) p1 = -kZeroRel;
    int cnt = p1 < 0.0 ? 1 : 0;
#pragma unroll 4
    for (int i = 1; i < r; ++i) {
        double p = fma((d[i] - x) * s, p1, -(e2s[i - 1] * p2));
        if (p == 0.0) p = -kZeroRel * p1;
        cnt += (__builtin_bit_cast(int64_t, p) ^ __builtin_bit_cast(int64_t, p1)) < 0 ? 1 : 0;
        p2 = p1;
        p1 = p;
        if ((i & 3) == 0) {
            // the larger of the two is brought to [0.5, 1)
            int ea, eb;
            (void)frexp(p1, &ea);
            (void)frexp(p2, &eb);
            const int ex = ea > eb ? ea : eb;
            p1 = ldexp(p1, -ex);
            p2 = ldexp(p2, -ex);
        }
    }
    return cnt;
}

// Lowest nw eigenvalues of T (ascending) by multisection: G lanes per eigenvalue (a
// power of two, at most 8, so a group never straddles a wavefront; more lanes make the
// work-group's vector units, not the dependent chain, the limit) evaluate the Sturm
// count at G interior points of the bracket, which shrinks G + 1 fold per step, down to
// the absolute width eps ||T|| (or 2 eps |lambda| when larger).  The bracket starts from
// the Gershgorin interval.  sc[3..7]: the Sturm scale, gl, gu, pivmin, ||T||; e2 receives
// the scaled squared off-diagonal.
__device__ void bisect_lowest(const double* d, const double* e, double* e2, int r, int nw,
                              double* theta, double* sc) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6;
    if (wave == 0) {
        double lo = 1.0 / 0.0, hi = -1.0 / 0.0, emax = 0.0;
        for (int i = lane; i < r; i += 64) {
            const double rad = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < r ? fabs(e[i]) : 0.0);
            lo = fmin(lo, d[i] - rad);
            hi = fmax(hi, d[i] + rad);
            if (i + 1 < r) emax = fmax(emax, e[i] * e[i]);
        }
        for (int o = 32; o > 0; o >>= 1) {
            lo = fmin(lo, __shfl_xor(lo, o, 64));
            hi = fmax(hi, __shfl_xor(hi, o, 64));
            emax = fmax(emax, __shfl_xor(emax, o, 64));
        }
        if (lane == 0) {
            const double tnorm = fmax(fabs(lo), fabs(hi));
            const double pivmin = kSafmin * fmax(1.0, emax);
            const double pad = 2.0 * kEps * tnorm * r + 2.0 * pivmin;
            sc[4] = lo - pad;
            sc[5] = hi + pad;
            sc[6] = pivmin;
            sc[7] = tnorm;
            int ex;
            (void)frexp(tnorm, &ex);
            sc[3] = ldexp(1.0, -ex);   // the Sturm counts' scale
        }
    }
    __syncthreads();
    const double ts = sc[3];
    for (int i = tid; i + 1 < r; i += nt) {
        const double es = e[i] * ts;
        e2[i] = es * es;
    }
    __syncthreads();
    const double gl = sc[4], gu = sc[5], pivmin = sc[6];
    const double atol = kEps * sc[7];
    int G = 1;
    while (G < 8 && 2 * G * nw <= nt) G *= 2;
    const int ng = nt / G;
    const int g = tid % G;
    const uint64_t gmask = (1ull << G) - 1;
    const int gbase = (lane / G) * G;
    const double inv_g1 = 1.0 / (double)(G + 1);
    for (int j0 = 0; j0 < nw; j0 += ng) {
        const int j = j0 + tid / G;
        const bool act = j < nw;
        double lo = gl, hi = gu;
        for (int it = 0; it < 100; ++it) {
            const bool done =
                !act || hi - lo <= fmax(atol, 2.0 * kEps * fmax(fabs(lo), fabs(hi))) + 2.0 * pivmin;
            if (__all(done)) break;
            const double w = hi - lo;
            const double x = lo + w * (double)(g + 1) * inv_g1;
            const int cnt = act ? sturm_count(d, e2, r, x, ts) : 0;
            const uint64_t bal = __ballot(cnt > j);
            const uint64_t gm = (bal >> gbase) & gmask;
            const int f = gm ? __builtin_ctzll(gm) : G;   // first point with lambda_j below it
            const double nlo = f > 0 ? lo + w * (double)f * inv_g1 : lo;
            const double nhi = f < G ? lo + w * (double)(f + 1) * inv_g1 : hi;
            if (!done) {
                lo = nlo;
                hi = nhi;
            }
        }
        if (act && g == 0) theta[j] = 0.5 * (lo + hi);
    }
}

// Row-swap flag and multiplier of elimination step i, kept in one double: the flag in the
// lowest mantissa bit (the multiplier moves by at most an ulp).
__device__ __forceinline__ double pack_step(double m, bool sw) {
    const uint64_t b = (__builtin_bit_cast(uint64_t, m) & ~1ull) | (sw ? 1ull : 0ull);
    return __builtin_bit_cast(double, b);
}
__device__ __forceinline__ double unpack_step(double v, bool& sw) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    sw = (b & 1ull) != 0;
    return __builtin_bit_cast(double, b & ~1ull);
}

// Back substitution with U (reciprocal diagonal in slot 0, first superdiagonal in slot 1;
// the second superdiagonal is e[i + 1] where step i swapped rows, else 0) from row r - 2
// up, x1 = x[r - 1] already in z.
__device__ __forceinline__ void tri_back(const double* e, int r, double* z, const double* u, int nwp,
                                         double x1) {
    if (r < 2) return;
    double x2 = 0.0;
    auto load = [&](int i, double& u0, double& u1, double& u2, double& zi) {
        const double* ui = u + 3 * i * nwp;
        bool sw;
        (void)unpack_step(ui[2 * nwp], sw);
        u0 = ui[0];
        u1 = ui[nwp];
        u2 = (sw && i + 2 < r) ? e[i + 1] : 0.0;
        zi = z[i * nwp];
    };
    double u0, u1, u2, zi;
    load(r - 2, u0, u1, u2, zi);
#pragma unroll 2
    for (int i = r - 2; i >= 0; --i) {
        double u0n = 0.0, u1n = 0.0, u2n = 0.0, zin = 0.0;
        if (i > 0) load(i - 1, u0n, u1n, u2n, zin);
        const double xi = (zi - u1 * x1 - u2 * x2) * u0;
        z[i * nwp] = xi;
        x2 = x1;
        x1 = xi;
        u0 = u0n;
        u1 = u1n;
        u2 = u2n;
        zi = zin;
    }
}

// One solve (T - lam I) x = z in place (z and the factor strided by nwp): LU with
// partial pivoting between neighbouring rows, U with two superdiagonals; the row
// operations are applied to z as they are made.  The factor u (3 r x nwp) keeps, per
// step, 1 / pivot, the first superdiagonal and the packed multiplier and swap flag (the
// second superdiagonal follows from the flag), and 1 / pivot of the last row, so that
// tri_resolve can repeat the solve.  The pivot choice is made with selects so lanes with
// different pivots do not diverge.  Zero pivots become eps ||T||.
__device__ void tri_solve(const double* d, const double* e, int r, double lam, double* z, double* u,
                          int nwp, double tiny) {
    // every value a step needs is loaded one step ahead, before the step's stores (the
    // compiler cannot move a load above a store to the same array)
    double cd = d[0] - lam, cs1 = r > 1 ? e[0] : 0.0;
    double yc = z[0];
    double nd = r > 1 ? e[0] : 0.0, dn = r > 1 ? d[1] : 0.0, en = r > 2 ? e[1] : 0.0;
    double yn = r > 1 ? z[nwp] : 0.0;
#pragma unroll 2
    for (int i = 0; i + 1 < r; ++i) {
        // current row (cd, cs1, 0 | yc), next row (nd, ns1, ns2 | yn)
        const double ns1 = dn - lam;
        const double ns2 = en;
        // the step after this one
        const double nd_n = en;
        const double dn_n = (i + 2 < r) ? d[i + 2] : 0.0;
        const double en_n = (i + 3 < r) ? e[i + 2] : 0.0;
        const double yn_n = (i + 2 < r) ? z[(i + 2) * nwp] : 0.0;
        const bool sw = fabs(cd) < fabs(nd);
        double pv = sw ? nd : cd;
        if (pv == 0.0) pv = tiny;
        const double ot = sw ? cd : nd;
        const double p1 = sw ? ns1 : cs1, p2 = sw ? ns2 : 0.0, py = sw ? yn : yc;
        const double o1 = sw ? cs1 : ns1, o2 = sw ? 0.0 : ns2, oy = sw ? yc : yn;
        const double ip = rcp_nr(pv);
        const double m = ot * ip;
        double* ui = u + 3 * i * nwp;
        ui[0] = ip;
        ui[nwp] = p1;
        ui[2 * nwp] = pack_step(m, sw);
        z[i * nwp] = py;
        cd = o1 - m * p1;
        cs1 = o2 - m * p2;
        yc = oy - m * py;
        nd = nd_n;
        dn = dn_n;
        en = en_n;
        yn = yn_n;
    }
    if (cd == 0.0) cd = tiny;
    const double il = rcp_nr(cd);
    u[3 * (r - 1) * nwp] = il;
    const double x1 = yc * il;
    z[(r - 1) * nwp] = x1;
    tri_back(e, r, z, u, nwp, x1);
}

// The solve of the last tri_solve with the same factor on a new z: the stored row
// swaps and multipliers, then the same back substitution.
__device__ void tri_resolve(const double* e, int r, double* z, const double* u, int nwp) {
    double yc = z[0];
    double yn = r > 1 ? z[nwp] : 0.0;
#pragma unroll 2
    for (int i = 0; i + 1 < r; ++i) {
        const double yn_n = (i + 2 < r) ? z[(i + 2) * nwp] : 0.0;
        bool sw;
        const double m = unpack_step(u[(3 * i + 2) * nwp], sw);
        const double py = sw ? yn : yc, oy = sw ? yc : yn;
        z[i * nwp] = py;
        yc = oy - m * py;
        yn = yn_n;
    }
    const double x1 = yc * u[3 * (r - 1) * nwp];
    z[(r - 1) * nwp] = x1;
    tri_back(e, r, z, u, nwp, x1);
}

// Eigenvectors of T for theta[0..nw) by two steps of inverse iteration (the second with
// the first step's factorisation), every vector in its own thread; eigenvalues closer
// than clrel ||T|| form a cluster whose vectors are orthonormalised by modified
// Gram-Schmidt (one wavefront per cluster) after every step, and whose equal shifts are
// separated by a few ulps.  Vectors of eigenvalues further apart are orthogonal to
// about eps / clrel without it.  Zt: r x nwp row-major (vector q in column q); U3:
// 3 r x nwp.
__device__ void inverse_iteration(const double* d, const double* e, int r, int nw, int nwp,
                                  const double* theta, double* sh, double* Zt, double* U3,
                                  int* cstart, int* csize, int* ncl, double tnorm, double clrel = 1e-3) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, nwave = nt >> 6;
    if (tid == 0) {
        const double ortol = clrel * tnorm;
        int c = -1;
        for (int j = 0; j < nw; ++j) {
            double s = theta[j];
            if (j == 0 || theta[j] - theta[j - 1] > ortol) {
                ++c;
                cstart[c] = j;
                csize[c] = 1;
            } else {
                ++csize[c];
                const double prev = sh[j - 1];
                if (s <= prev + 10.0 * kEps * fabs(prev)) s = prev + 10.0 * kEps * fmax(fabs(prev), 1e-3 * tnorm);
            }
            sh[j] = s;
        }
        *ncl = c + 1;
    }
    __syncthreads();
    const double tiny = kEps * tnorm > 0.0 ? kEps * tnorm : kSafmin;
    const int nc = *ncl;
    for (int it = 0; it < 2; ++it) {
        for (int q = tid; q < nw; q += nt) {
            double* z = Zt + q;
            if (it == 0) {
                // start vector: a fixed, non-degenerate pattern per column
                for (int i = 0; i < r; ++i) {
                    const uint32_t h = (uint32_t)(i + 1) * 2654435761u ^ (uint32_t)(q + 1) * 2246822519u;
                    z[i * nwp] = (double)((h >> 8) & 0xffff) * (1.0 / 65536.0) + 0.25;
                }
            }
            if (it == 0) tri_solve(d, e, r, sh[q], z, U3 + q, nwp, tiny);
            else tri_resolve(e, r, z, U3 + q, nwp);
            double s2 = 0.0;
#pragma unroll 4
            for (int i = 0; i < r; ++i) s2 = fma(z[i * nwp], z[i * nwp], s2);
            const double inv = rsq_nr(s2);
#pragma unroll 4
            for (int i = 0; i < r; ++i) z[i * nwp] *= inv;
        }
        __syncthreads();
        for (int c = wave; c < nc; c += nwave) {
            const int c0 = cstart[c], cn = csize[c];
            for (int m = 1; m < cn; ++m) {
                const int jj = c0 + m;
                for (int i0 = c0; i0 < jj; ++i0) {
                    double dot = 0.0;
                    for (int row = lane; row < r; row += 64)
                        dot = fma(Zt[row * nwp + i0], Zt[row * nwp + jj], dot);
                    dot = wave_allsum(dot);
                    for (int row = lane; row < r; row += 64)
                        Zt[row * nwp + jj] -= dot * Zt[row * nwp + i0];
                }
                double s2 = 0.0;
                for (int row = lane; row < r; row += 64)
                    s2 = fma(Zt[row * nwp + jj], Zt[row * nwp + jj], s2);
                const double inv = rsq_nr(wave_allsum(s2));
                for (int row = lane; row < r; row += 64) Zt[row * nwp + jj] *= inv;
            }
        }
        __syncthreads();
    }
}

// Workspace layout of the kernel, in doubles from a 16-byte-aligned base.  The main
// route and the rank-revealing route share D, the flags, A and B, and otherwise overlay.
// On the main route A holds L, then the product scratch, B holds D H_R D, then C, T
// holds L^{-1} = M^T, then M = L^{-T} Q; the inverse-iteration factors reuse A and B
// when they fit there.
// register-row width for order k (8 lanes per row, NT columns per lane); 0: LDS routines
__host__ __device__ inline int rr_nt(int k) { return k <= 40 ? 5 : k <= 72 ? 9 : k <= 128 ? 16 : 0; }

struct RRLayout {
    int64_t D, flags, A, B;
    int64_t T, Zt, U3, d, e, e2, invd, pA, pM, pv, vb, theta, sh, sc, icl, rb, main_end;   // main route
    int64_t V, fT, rot, ftheta, fsel, fb_end;                                      // rank-revealing
    int64_t total;
};

__host__ __device__ inline RRLayout rr_layout(int k, int nwp) {
    RRLayout L{};
    const int64_t kk = (int64_t)k * k;
    L.D = 0;
    L.flags = k + (k & 1);             // 8 ints
    L.A = L.flags + 4;
    L.B = L.A + kk;
    L.T = L.B + kk;
    L.Zt = L.T + kk;
    L.d = L.Zt + (int64_t)k * nwp;
    L.e = L.d + k;
    L.e2 = L.e + k;
    L.invd = L.e2 + k;
    L.pA = L.invd + k;
    L.pM = L.pA + k;
    L.pv = L.pM + k;
    L.vb = L.pv + k;                   // 2 k
    L.theta = L.vb + 2 * (int64_t)k;
    L.sh = L.theta + k;
    L.sc = L.sh + k;                   // 8 doubles
    L.icl = L.sc + 8;                  // 2 k + 2 ints
    L.rb = L.icl + k + 1;              // 4 P doubles for the register-row routines
    L.main_end = L.rb + 4 * 8 * (int64_t)rr_nt(k);
    if ((int64_t)3 * k * nwp <= 2 * kk) {
        L.U3 = L.A;
    } else {
        L.U3 = L.main_end;
        L.main_end += (int64_t)3 * k * nwp;
    }
    L.V = L.B + kk;
    L.fT = L.V + kk;
    L.rot = L.fT + kk;                 // (k/2 + 1) double2 then (k/2 + 1) int2
    if (L.rot & 1) L.rot += 1;
    L.ftheta = L.rot + 3 * (int64_t)(k / 2 + 1);
    L.fsel = L.ftheta + k;             // k ints
    L.fb_end = L.fsel + k / 2 + 1;
    L.total = L.main_end > L.fb_end ? L.main_end : L.fb_end;
    return L;
}

// ALL_LDS: the whole layout in LDS (pointers derived from the LDS base only, so the
// compiler emits LDS instructions); otherwise in the global workspace.  The global
// workspace always holds the k x k product scratch of the rank-revealing route.
// NT > 0: the dense phases on register rows (r <= 8 NT); NT = 0: the LDS routines.
template <bool ALL_LDS, int NT>
__global__ __launch_bounds__(kRRThreads) void k_rayleigh_ritz(int k, int nwant,
                                                              const double* __restrict__ HR,
                                                              const double* __restrict__ SR,
                                                              int64_t ldr, double* __restrict__ gamma,
                                                              double* __restrict__ W, int64_t ldw,
                                                              int32_t* __restrict__ info,
                                                              double* gws, double* gamma_host,
                                                              int32_t* info_host, const int32_t* run_if) {
    extern __shared__ double lds[];
    __shared__ double red[kRRThreads / 64];
    const int tid = threadIdx.x, nt = blockDim.x;
    if (run_if) {
        // the fallback of the many-work-group route: run only if it set its flag (read
        // by every thread before any store, since the flag lies in the workspace)
        const bool run = __hip_atomic_load(run_if, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
        __syncthreads();
        if (!run) return;
    }
    const int64_t kk = (int64_t)k * k;
    const int nwp = nwant | 1;
    const RRLayout Lo = rr_layout(k, nwp);
    double* galigned = gws + (((uintptr_t)gws & 15) ? 1 : 0);
    double* base = ALL_LDS ? lds : galigned;
    double* U = galigned + Lo.total;   // global scratch (rank-revealing route)
    double* D = base + Lo.D;
    int* flag = (int*)(base + Lo.flags);
    double* A = base + Lo.A;
    double* B = base + Lo.B;

    for (int i = tid; i < k; i += nt) {
        const double dd = SR[i + (int64_t)i * ldr];
        D[i] = dd > 0.0 ? 1.0 / sqrt(dd) : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < kk; e += nt) {
        const int i = (int)(e % k), j = (int)(e / k);
        if (NT == 0) A[e] = D[i] * SR[i + (int64_t)j * ldr] * D[j];
        B[e] = D[i] * HR[i + (int64_t)j * ldr] * D[j];
    }
    __syncthreads();
    double* invd = base + Lo.invd;
    double* T = base + Lo.T;
    double* sc = base + Lo.sc;
    bool spd;
    if constexpr (NT > 0) {
        // X = L^{-1} into T
        spd = chol_inv_regs<NT>(SR, ldr, D, k, T, base + Lo.rb, sc + 4);
    } else {
        spd = cholesky_rl(A, k, invd);
        if (spd) {
            __syncthreads();
            invert_lower_rl(A, invd, T, k);
        }
    }
    if (spd) {
        __syncthreads();
        double* Zt = base + Lo.Zt;
        double* U3 = base + Lo.U3;
        double* d = base + Lo.d;
        double* e = base + Lo.e;
        double* e2 = base + Lo.e2;
        double* theta = base + Lo.theta;
        double* sh = base + Lo.sh;
        int* cstart = (int*)(base + Lo.icl);
        int* csize = cstart + k;
        int* ncl = csize + k;
        // C = X B X^T via U = B X^T (into A, L is no longer needed)
        gemm_mfma(B, k, false, T, k, true, k, k, k,
                  [&](int i, int j, double v) { A[i + j * k] = v; });
        __syncthreads();
        gemm_mfma(T, k, false, A, k, false, k, k, k,
                  [&](int i, int j, double v) { B[i + j * k] = v; });
        __syncthreads();
        if constexpr (NT > 0) {
            // symmetrised on loading; M = X^T Q leaves row-major in T
            tridiag_regs<NT>(B, T, k, d, e, base + Lo.rb, sc);
        } else {
            symmetrize(B, k);
            __syncthreads();
            // T read row-major is X^T = L^{-T}: the reflectors accumulate onto it
            tridiagonalize_acc(B, T, k, d, e, base + Lo.vb, base + Lo.pA, base + Lo.pM, base + Lo.pv, sc);
        }
        __syncthreads();
        bisect_lowest(d, e, e2, k, nwant, theta, sc);
        __syncthreads();
        inverse_iteration(d, e, k, nwant, nwp, theta, sh, Zt, U3, cstart, csize, ncl, sc[7]);
        // W = D M Z (M row-major in T, Z row-major in Zt with ld nwp)
        gemm_mfma(T, k, true, Zt, nwp, true, k, nwant, k,
                  [&](int i, int q, double v) { W[i + (int64_t)q * ldw] = D[i] * v; });
        for (int q = tid; q < nwant; q += nt) {
            gamma[q] = theta[q];
            if (gamma_host) gamma_host[q] = theta[q];
        }
        if (tid == 0) {
            info[0] = 0;
            info[1] = 0;
            if (info_host) { info_host[0] = 0; info_host[1] = 0; }
        }
        return;
    }
    // ------------------------------------------------------------ rank-revealing route
    __syncthreads();
    double* V = base + Lo.V;
    double* fT = base + Lo.fT;
    double2* rcs = (double2*)(base + Lo.rot);
    int2* rpq = (int2*)(rcs + (k / 2 + 1));
    double* theta = base + Lo.ftheta;
    int* sel = (int*)(base + Lo.fsel);
    // eigen-decompose the scaled S_R (V accumulates its vectors)
    for (int e = tid; e < kk; e += nt) {
        const int i = (int)(e % k), j = (int)(e / k);
        A[e] = D[i] * SR[i + (int64_t)j * ldr] * D[j];
        V[e] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    jacobi(A, k, V, k, k, red, rcs, rpq);
    __syncthreads();
    double mx = 0.0;
    for (int i = 0; i < k; ++i) mx = fmax(mx, A[i + i * k]);
    if (tid == 0) {
        int c = 0;
        for (int i = 0; i < k; ++i)
            if (A[i + i * k] > kRankTol * mx) sel[c++] = i;
        flag[1] = c;
    }
    __syncthreads();
    const int r = flag[1];
    // T = Q_keep / sqrt(lambda_keep) (k x r, ld k)
    for (int e = tid; e < k * r; e += nt) {
        const int i = (int)(e % k), c = (int)(e / k);
        const int src = sel[c];
        fT[i + c * k] = V[i + src * k] / sqrt(A[src + src * k]);
    }
    __syncthreads();
    // C = T^T B T (r x r, ld r) into B, via U = B T (k x r)
    small_gemm(B, false, fT, false, U, k, r, k, k, k, k);
    __syncthreads();
    small_gemm(fT, true, U, false, B, r, r, k, k, k, r);
    __syncthreads();
    if (r < nwant) {
        if (tid == 0) {
            info[0] = k - r;
            info[1] = (int)LABPSD_ERANK;
            if (info_host) { info_host[0] = k - r; info_host[1] = (int)LABPSD_ERANK; }
        }
        return;
    }
    // symmetrise C (r x r, ld r), V = I
    for (int e = tid; e < r * r; e += nt) {
        const int i = (int)(e % r), j = (int)(e / r);
        if (i < j) {
            const double a = 0.5 * (B[i + j * r] + B[j + i * r]);
            B[i + j * r] = a;
            B[j + i * r] = a;
        }
        V[e] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    jacobi(B, r, V, r, r, red, rcs, rpq);
    __syncthreads();
    for (int i = tid; i < r; i += nt) theta[i] = B[i + i * r];
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
    for (int q = tid; q < nwant; q += nt) {
        gamma[q] = theta[sel[q]];
        if (gamma_host) gamma_host[q] = theta[sel[q]];
    }
    // W = D T V(:, sel)
    for (int e = tid; e < k * nwant; e += nt) {
        const int i = (int)(e % k), q = (int)(e / k);
        const int src = sel[q];
        double acc = 0.0;
        for (int p = 0; p < r; ++p) acc = fma(fT[i + p * k], V[p + src * r], acc);
        W[i + (int64_t)q * ldw] = D[i] * acc;
    }
    if (tid == 0) {
        info[0] = k - r;
        info[1] = 0;
        if (info_host) { info_host[0] = k - r; info_host[1] = 0; }
    }
}

// ---------------------------------------------------------------- large orders
// Above the register-row range the O(k^3) phases run on many work-groups, each phase
// its own launch (the launch boundary orders them), except the tridiagonal reduction:
//   prep      D, A = D S_R D and B = D H_R D, padded to kp = 16 ceil(k / 16) (A with
//             the identity, B with zeros, so the padding stays decoupled);
//   chol      blocked Cholesky A = L L^T, one launch per 16-column panel: every
//             work-group takes one 16 x 16 tile of the panel, forms it and the diagonal
//             tile from the finished panels with MFMA, factors the diagonal tile itself
//             (the same arithmetic in every work-group) and solves its tile; L^T's
//             tiles go to the unused upper blocks of A;
//   fwd (x2)  Y = L^{-1} B, then C = L^{-1} Y^T, one 16-column slice per work-group,
//             blocked forward substitution with MFMA; slices are kept row-major per
//             slice ((row, j) at row 16 + j) so the MFMA operands load contiguously;
//   sym       C <- (C + C^T) / 2, column-major;
//   tridiag   Householder reduction of C (order k) on G co-resident work-groups, column
//             c owned by work-group c mod G, one grid barrier per reflector (after the
//             products p = tau C v; every work-group then updates its columns and builds
//             the next reflector itself from the published next column); vectors shared
//             between work-groups are written and read with device-scope atomics;
//   bisect    the wanted eigenvalues by multisection, one wavefront (64 points per step)
//             per eigenvalue;
//   teig      eigenvectors by inverse iteration (one work-group, as in the one-work-group
//             kernel);
//   back      per 16-column slice of Z: X = Q Z (reflectors in reverse order), then
//             W = D L^{-T} X by blocked back substitution with MFMA.
// A pivot of the scaled S_R at or below 1e-14, or a barrier wait that runs out, sets a
// flag: the kernels after it return at once and the one-work-group kernel solves the
// pencil instead (rank-revealing route included).

constexpr int kRRLargeMin = 129;
constexpr int kLT = 16;
constexpr int kLThreads = 256;
constexpr int kRRSpinLimit = 1 << 20;

__host__ __device__ inline int rrl_kp(int k) { return (k + kLT - 1) / kLT * kLT; }

struct RRLLayout {
    int64_t ctl, D, A, L, B, Y, d, e, tau, theta, sh, vb, p, part, sc, icl, Zt, U3, wyt, total;
};

// blocks of kLT reflectors in the back-transformation (k - 2 reflectors)
__host__ __device__ inline int rrl_wy_blocks(int k) { return k > 2 ? (k - 2 + kLT - 1) / kLT : 1; }

// offsets in doubles; everything before Zt is independent of nwp
__host__ __device__ inline RRLLayout rrl_layout(int k, int nwp) {
    const int64_t kp = rrl_kp(k), kk = kp * kp;
    RRLLayout L{};
    L.ctl = 0;                 // 16 int32: [0] fallback flag, [1] barrier counter
    L.D = 8;
    L.A = L.D + kp;
    L.L = L.A + kk;
    L.B = L.L + kk;
    L.Y = L.B + kk;
    L.d = L.Y + kk;
    L.e = L.d + kp;
    L.tau = L.e + kp;
    L.theta = L.tau + kp;
    L.sh = L.theta + kp;
    L.vb = L.sh + kp;          // 2 kp
    L.p = L.vb + 2 * kp;       // 2 kp
    L.part = L.p + 2 * kp;     // 2 x 256
    L.sc = L.part + 512;       // 8
    L.icl = L.sc + 8;          // 2 kp + 4 int32
    L.Zt = L.icl + kp + 2;
    L.U3 = L.Zt + (int64_t)k * nwp;
    L.wyt = L.U3 + 3 * (int64_t)k * nwp;   // kLT x kLT per block of reflectors
    L.total = L.wyt + (int64_t)kLT * kLT * rrl_wy_blocks(k);
    return L;
}

__device__ __forceinline__ bool rrl_failed(const double* base) {
    return __hip_atomic_load((const int*)base, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// acc += sum over kc in [kb, ke) of X(i, kc) Y(kc, j) (16 x 16 tile, 4 columns of kc per
// MFMA step, the steps dealt round-robin to nwave wavefronts, loads issued 8 steps at a
// time); xa(i, kc) and yb(kc, j) return the operands.  ke - kb is a multiple of 4.
template <typename FA, typename FB>
__device__ __forceinline__ rr_double4 mfma_tile(FA xa, FB yb, int kb, int ke, int wave, int nwave,
                                                rr_double4 acc) {
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int nst = (ke - kb) >> 2;
    int s = wave;
    for (; s + 7 * nwave < nst; s += 8 * nwave) {
        double a[8], b[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int kc = kb + 4 * (s + u * nwave) + lk;
            a[u] = xa(li, kc);
            b[u] = yb(kc, li);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
    }
    for (; s < nst; s += nwave) {
        const int kc = kb + 4 * s + lk;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xa(li, kc), yb(kc, li), acc, 0, 0, 0);
    }
    return acc;
}

// the four wavefronts' accumulators into red[w][i * 16 + j] (accumulator register q of
// lane l holds row 4 q + l / 16, column l % 16)
__device__ __forceinline__ void tile_to_lds(const rr_double4& acc, double (*red)[256]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 4; ++q) red[wave][(4 * q + (lane >> 4)) * 16 + (lane & 15)] = acc[q];
}

__global__ __launch_bounds__(kLThreads) void k_rrl_prep(int k, const double* __restrict__ HR,
                                                        const double* __restrict__ SR, int64_t ldr,
                                                        double* __restrict__ base) {
    const RRLLayout Lo = rrl_layout(k, 1);
    const int64_t kp = rrl_kp(k), kk = kp * kp;
    double* D = base + Lo.D;
    double* A = base + Lo.A;
    double* B = base + Lo.B;
    const int64_t stride = (int64_t)gridDim.x * kLThreads;
    const int64_t t0 = (int64_t)blockIdx.x * kLThreads + threadIdx.x;
    if (t0 < 16) ((int*)(base + Lo.ctl))[t0] = 0;
    for (int64_t i = t0; i < kp; i += stride) {
        double di = 0.0;
        if (i < k) {
            const double sd = SR[i + i * ldr];
            di = sd > 0.0 ? 1.0 / sqrt(sd) : 0.0;
        }
        D[i] = di;
    }
    for (int64_t e = t0; e < kk; e += stride) {
        const int64_t i = e % kp, j = e / kp;
        double a = (i == j) ? 1.0 : 0.0, b = 0.0;
        if (i < k && j < k) {
            const double si = SR[i + i * ldr], sj = SR[j + j * ldr];
            const double di = si > 0.0 ? 1.0 / sqrt(si) : 0.0, dj = sj > 0.0 ? 1.0 / sqrt(sj) : 0.0;
            a = di * SR[i + j * ldr] * dj;
            b = di * HR[i + j * ldr] * dj;
        }
        A[e] = a;
        B[e] = b;
    }
}

// panel p of the blocked Cholesky; work-group b takes row tile r = p + b
__global__ __launch_bounds__(kLThreads) void k_rrl_chol(int k, int p, double* __restrict__ base) {
    if (rrl_failed(base)) return;
    const RRLLayout Lo = rrl_layout(k, 1);
    const int64_t kp = rrl_kp(k);
    double* A = base + Lo.A;
    double* L = base + Lo.L;
    const int tid = threadIdx.x, wave = tid >> 6;
    const int r = p + blockIdx.x, r0 = r * kLT, p0 = p * kLT;
    __shared__ double red[2][4][256];
    __shared__ double tD[16][17], tR[16][17];
    auto lr = [&](int i, int kc) { return L[(r0 + i) + (int64_t)kc * kp]; };
    auto lp = [&](int i, int kc) { return L[(p0 + i) + (int64_t)kc * kp]; };
    auto lpt = [&](int kc, int j) { return L[(p0 + j) + (int64_t)kc * kp]; };
    rr_double4 accR = {0.0, 0.0, 0.0, 0.0}, accD = {0.0, 0.0, 0.0, 0.0};
    accR = mfma_tile(lr, lpt, 0, p0, wave, 4, accR);
    if (r != p) accD = mfma_tile(lp, lpt, 0, p0, wave, 4, accD);
    tile_to_lds(accR, red[0]);
    tile_to_lds(accD, red[1]);
    __syncthreads();
    const int i = tid >> 4, j = tid & 15;
    {
        const double sR = red[0][0][tid] + red[0][1][tid] + red[0][2][tid] + red[0][3][tid];
        const double sD = r == p ? sR : red[1][0][tid] + red[1][1][tid] + red[1][2][tid] + red[1][3][tid];
        tR[i][j] = A[(r0 + i) + (int64_t)(p0 + j) * kp] - sR;
        tD[i][j] = A[(p0 + i) + (int64_t)(p0 + j) * kp] - sD;
    }
    __syncthreads();
    // the diagonal tile, one entry per thread (identical in every work-group)
    for (int c = 0; c < 16; ++c) {
        const double piv = tD[c][c];
        if (!(piv > kPivotTol)) {
            if (tid == 0) __hip_atomic_fetch_or((int*)base, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;   // uniform: every thread read the same pivot
        }
        const double lc = sqrt(piv);
        const double lic = i > c ? tD[i][c] / lc : 0.0;
        const double ljc = j > c ? tD[j][c] / lc : 0.0;
        __syncthreads();
        if (j == c) {
            if (i == c) tD[i][j] = lc;
            else if (i > c) tD[i][j] = lic;
        } else if (j > c && i >= j) {
            tD[i][j] -= lic * ljc;
        }
        __syncthreads();
    }
    if (r == p) {
        L[(p0 + i) + (int64_t)(p0 + j) * kp] = i >= j ? tD[i][j] : 0.0;
        return;
    }
    // L(r, p) = T_R L_pp^{-T}: row i of the tile by forward substitution
    if (tid < 16) {
        for (int c = 0; c < 16; ++c) {
            double v = tR[tid][c];
            for (int c2 = 0; c2 < c; ++c2) v -= tR[tid][c2] * tD[c][c2];
            tR[tid][c] = v / tD[c][c];
        }
    }
    __syncthreads();
    const double x = tR[i][j];
    L[(r0 + i) + (int64_t)(p0 + j) * kp] = x;
    A[(p0 + j) + (int64_t)(r0 + i) * kp] = x;   // L^T into the upper block (p, r) of A
}

// Y = L^{-1} X for the 16-column slice blockIdx.x; X(a, b) = xsr ? the slice-row-major
// matrix X at (row b, column a) : X[a + b kp]; Y slice-row-major.
__global__ __launch_bounds__(kLThreads) void k_rrl_fwd(int k, const double* X, int xsr, double* Ys,
                                                       double* __restrict__ base) {
    if (rrl_failed(base)) return;
    const RRLLayout Lo = rrl_layout(k, 1);
    const int64_t kp = rrl_kp(k);
    const int nrb = (int)(kp / kLT);
    const double* L = base + Lo.L;
    const int tid = threadIdx.x, wave = tid >> 6;
    const int c0 = blockIdx.x * kLT;
    double* Y = Ys + (int64_t)blockIdx.x * kp * kLT;
    __shared__ double red[4][256];
    __shared__ double t[16][17], lpp[16][17];
    const int i = tid >> 4, j = tid & 15;
    for (int p = 0; p < nrb; ++p) {
        const int p0 = p * kLT;
        rr_double4 acc = {0.0, 0.0, 0.0, 0.0};
        acc = mfma_tile([&](int a, int kc) { return L[(p0 + a) + (int64_t)kc * kp]; },
                        [&](int kc, int b) { return Y[(int64_t)kc * kLT + b]; }, 0, p0, wave, 4, acc);
        tile_to_lds(acc, red);
        const double xv = xsr ? X[(int64_t)p * kp * kLT + (int64_t)(c0 + j) * kLT + i]
                              : X[(p0 + i) + (int64_t)(c0 + j) * kp];
        lpp[i][j] = L[(p0 + i) + (int64_t)(p0 + j) * kp];
        __syncthreads();
        t[i][j] = xv - (red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid]);
        __syncthreads();
        if (tid < 16) {
            for (int a = 0; a < 16; ++a) {
                double v = t[a][tid];
                for (int b2 = 0; b2 < a; ++b2) v -= lpp[a][b2] * t[b2][tid];
                t[a][tid] = v / lpp[a][a];
            }
        }
        __syncthreads();
        Y[(int64_t)(p0 + i) * kLT + j] = t[i][j];
        __syncthreads();
    }
}

// C (slice-row-major in B) -> (C + C^T) / 2, column-major in Y
__global__ __launch_bounds__(kLThreads) void k_rrl_sym(int k, double* __restrict__ base) {
    if (rrl_failed(base)) return;
    const RRLLayout Lo = rrl_layout(k, 1);
    const int64_t kp = rrl_kp(k), kk = kp * kp;
    const double* Cs = base + Lo.B;
    double* C = base + Lo.Y;
    auto at = [&](int64_t a, int64_t b) { return Cs[(b >> 4) * kp * kLT + a * kLT + (b & 15)]; };
    const int64_t stride = (int64_t)gridDim.x * kLThreads;
    for (int64_t e = (int64_t)blockIdx.x * kLThreads + threadIdx.x; e < kk; e += stride) {
        const int64_t i = e % kp, j = e / kp;
        C[e] = (i < k && j < k) ? 0.5 * (at(i, j) + at(j, i)) : 0.0;
    }
}

// Householder tridiagonalisation of C (column-major, ld kp, order k) on gridDim.x
// co-resident work-groups: d, e, tau; reflector j = I - tau_j v v^T with v_{j+1} = 1 and
// v_i (i > j + 1) kept in C[i, j].  Column c belongs to work-group c mod G.  One grid
// barrier per reflector: before it, every work-group forms its part of p = tau C v and
// of p . v, and the owner of column j + 1 publishes that column; after it, every
// work-group applies the rank-2 update to its own columns and, redundantly and with the
// same arithmetic, to the published column, from which it builds the next reflector
// itself.  Vectors shared between work-groups (p, the partial sums, the published
// column; double-buffered by parity, so a work-group running one step ahead never
// overwrites what another still reads) go through device-scope atomics.  A work-group's
// own columns stay in LDS from the first reflector to the last (the dot products and the
// rank-2 updates read and write LDS, not L2) and go back to C at the end (OWN_LDS; orders
// whose columns do not fit keep them in C).
// Dynamic LDS: (4 + ceil(k / G)) kp doubles with OWN_LDS, else 4 kp.
template <bool OWN_LDS>
__global__ __launch_bounds__(kLThreads) void k_rrl_tridiag(int k, double* __restrict__ base) {
    if (rrl_failed(base)) return;
    const RRLLayout Lo = rrl_layout(k, 1);
    const int64_t kp = rrl_kp(k);
    int* fail = (int*)(base + Lo.ctl);
    int* bar = fail + 1;
    double* C = base + Lo.Y;
    double* d = base + Lo.d;
    double* e = base + Lo.e;
    double* tau = base + Lo.tau;
    double* colb = base + Lo.vb;     // 2 kp: the published column, by parity
    double* pg = base + Lo.p;        // 2 kp: p, by parity
    double* part = base + Lo.part;   // 2 x 256: the work-groups' parts of p . v, by parity
    extern __shared__ double sm[];
    double* sv = sm;                 // v_j
    double* svn = sm + kp;           // v_{j+1}
    double* sp = sm + 2 * kp;        // p_j
    double* sy = sm + 3 * kp;        // the published column, updated
    double* own = sm + 4 * kp;       // this work-group's columns g, g + G, g + 2 G, ...
    __shared__ double red[2][4];
    __shared__ int sok;
    const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // column c (owned here)
    auto ocol = [&](int c) -> double* {
        if constexpr (OWN_LDS) return own + (int64_t)((c - g) / G) * kp;
        else return C + (int64_t)c * kp;
    };
    int nbar = 0;
    // grid-wide barrier: this thread's stores and atomics have completed before the
    // work-group counts itself in; false once any work-group has given up
    auto gsync = [&]() -> bool {
        __builtin_amdgcn_s_waitcnt(0x0F70);
        __syncthreads();
        ++nbar;
        if (tid == 0) {
            __hip_atomic_fetch_add(bar, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int target = nbar * G;
            int ok = 1, spins = 0;
            while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                ++spins;
                if ((spins & 63) == 0 &&
                    (spins > kRRSpinLimit ||
                     __hip_atomic_load(fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
                    __hip_atomic_fetch_or(fail, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            sok = ok;
        }
        __syncthreads();
        return sok != 0;
    };
    // reflector of column c from y (LDS, rows c + 1.., final): v into vn, tau, beta; the
    // same result in every work-group (same data, same reduction order); keep: also store
    // v below the subdiagonal of C's column c.  The caller syncs before vn is read.
    auto make_reflector = [&](const double* y, int c, double* vn, double& t, double& beta, bool keep) {
        double sg = 0.0, a1 = 0.0;
        for (int i = c + 1 + tid; i < k; i += kLThreads) {
            const double x = y[i];
            if (i == c + 1) a1 = x;
            else sg = fma(x, x, sg);
        }
        sg = wave_allsum(sg);
        a1 = wave_allsum(a1);
        if (lane == 0) {
            red[0][wave] = sg;
            red[1][wave] = a1;
        }
        __syncthreads();
        const double sigma = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        const double alpha = red[1][0] + red[1][1] + red[1][2] + red[1][3];
        __syncthreads();
        double scal;
        reflector(alpha, sigma, t, beta, scal);
        double* col = keep ? ocol(c) : nullptr;
        for (int i = c + 1 + tid; i < k; i += kLThreads) {
            const double vi = (i == c + 1) ? 1.0 : y[i] * scal;
            vn[i] = vi;
            if (keep && i > c + 1) col[i] = vi;
        }
    };
    // the first column >= cmin owned by this wavefront (columns g + t G, t = wave mod 4)
    auto first_own = [&](int cmin) {
        int t = cmin > g ? (cmin - g + G - 1) / G : 0;
        t += ((wave - t) % 4 + 4) % 4;
        return g + t * G;
    };
    // this work-group's columns into LDS; reflector 0 from column 0, in every work-group
    if constexpr (OWN_LDS)
        for (int c = g; c < k; c += G) {
            double* oc = ocol(c);
            const double* src = C + (int64_t)c * kp;
            for (int64_t i = tid; i < kp; i += kLThreads) oc[i] = src[i];
        }
    for (int i = tid; i < k; i += kLThreads) sy[i] = C[i];
    __syncthreads();
    double tj, beta0;
    make_reflector(sy, 0, sv, tj, beta0, g == 0);
    if (g == 0 && tid == 0) {
        d[0] = sy[0];
        e[0] = beta0;
        tau[0] = tj;
    }
    __syncthreads();
    for (int j = 0; j + 2 < k; ++j) {
        const int par = j & 1;
        double* pgj = pg + par * kp;
        double* partj = part + par * 256;
        double* cbj = colb + ((j + 1) & 1) * kp;
        // the owner of column j + 1 publishes it (its updates up to reflector j - 1 are in)
        if (g == (j + 1) % G) {
            const double* col = ocol(j + 1);
            for (int i = j + 1 + tid; i < k; i += kLThreads)
                __hip_atomic_store(cbj + i, col[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        // p_c = tau (C v)_c for the owned columns, and this work-group's part of p . v
        double mp = 0.0;
        for (int c = first_own(j + 1); c < k; c += 4 * G) {
            const double* col = ocol(c);
            double dot = 0.0;
            for (int i = j + 1 + lane; i < k; i += 64) dot = fma(col[i], sv[i], dot);
            dot = tj * wave_allsum(dot);
            if (lane == 0) __hip_atomic_store(pgj + c, dot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            mp = fma(dot, sv[c], mp);
        }
        if (lane == 0) red[0][wave] = mp;
        __syncthreads();
        if (tid == 0)
            __hip_atomic_store(partj + g, red[0][0] + red[0][1] + red[0][2] + red[0][3], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        if (!gsync()) return;
        // C <- C - v w^T - w v^T with w = p - K v, K = tau (p . v) / 2
        for (int i = j + 1 + tid; i < k; i += kLThreads) {
            sp[i] = __hip_atomic_load(pgj + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            sy[i] = __hip_atomic_load(cbj + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        double ps = 0.0;
        for (int q = lane; q < G; q += 64) ps += __hip_atomic_load(partj + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const double K = 0.5 * tj * wave_allsum(ps);
        __syncthreads();
        for (int c = first_own(j + 2); c < k; c += 4 * G) {
            double* col = ocol(c);
            const double vc = sv[c], wc = sp[c] - K * vc;
            for (int i = j + 1 + lane; i < k; i += 64) {
                const double vi = sv[i];
                col[i] -= vi * wc + (sp[i] - K * vi) * vc;
            }
            if (c == k - 1 && j + 3 == k && lane == 0) d[k - 1] = col[k - 1];
        }
        {
            // column j + 1, from its published copy
            const int c = j + 1;
            const double vc = sv[c], wc = sp[c] - K * vc;
            for (int i = j + 1 + tid; i < k; i += kLThreads) {
                const double vi = sv[i];
                sy[i] -= vi * wc + (sp[i] - K * vi) * vc;
            }
        }
        __syncthreads();
        if (j + 3 < k) {
            double tn, bn;
            make_reflector(sy, j + 1, svn, tn, bn, g == (j + 1) % G);
            if (g == 0 && tid == 0) {
                d[j + 1] = sy[j + 1];
                e[j + 1] = bn;
                tau[j + 1] = tn;
            }
            tj = tn;
            double* tsw = sv;
            sv = svn;
            svn = tsw;
            __syncthreads();
        } else if (g == 0 && tid == 0) {   // j + 1 = k - 2: the last off-diagonal
            d[k - 2] = sy[k - 2];
            e[k - 2] = sy[k - 1];
        }
    }
    // the columns (reflectors below the subdiagonal) back to C
    if constexpr (OWN_LDS) {
        __syncthreads();
        for (int c = g; c < k; c += G) {
            const double* oc = ocol(c);
            double* dst = C + (int64_t)c * kp;
            for (int64_t i = tid; i < kp; i += kLThreads) dst[i] = oc[i];
        }
    }
}

// The wanted eigenvalues of T by multisection, one wavefront per eigenvalue: the 64
// lanes evaluate the Sturm count at 64 interior points of the bracket, which shrinks
// 65-fold per step (about nine steps from the Gershgorin interval to the width eps ||T||).
// Every work-group forms the bounds, the Sturm scale and the scaled e^2 itself (d and
// e^2 in LDS, 2 kp doubles); work-group 0 also stores sc[3..7] for the inverse iteration.
__global__ __launch_bounds__(kLThreads) void k_rrl_bisect(int k, int nwant, double* __restrict__ base) {
    if (rrl_failed(base)) return;
    const RRLLayout Lo = rrl_layout(k, 1);
    const int64_t kp = rrl_kp(k);
    const double* dg = base + Lo.d;
    const double* eg = base + Lo.e;
    double* theta = base + Lo.theta;
    double* sc = base + Lo.sc;
    extern __shared__ double bl[];
    double* d = bl;
    double* e2 = bl + kp;
    __shared__ double red[3][4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double lo = 1.0 / 0.0, hi = -1.0 / 0.0, emax = 0.0;
    for (int i = tid; i < k; i += kLThreads) {
        const double di = dg[i];
        d[i] = di;
        const double em = i > 0 ? eg[i - 1] : 0.0, ei = i + 1 < k ? eg[i] : 0.0;
        const double rad = fabs(em) + fabs(ei);
        lo = fmin(lo, di - rad);
        hi = fmax(hi, di + rad);
        if (i + 1 < k) emax = fmax(emax, ei * ei);
    }
    for (int o = 32; o > 0; o >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, o, 64));
        hi = fmax(hi, __shfl_xor(hi, o, 64));
        emax = fmax(emax, __shfl_xor(emax, o, 64));
    }
    if (lane == 0) {
        red[0][wave] = lo;
        red[1][wave] = hi;
        red[2][wave] = emax;
    }
    __syncthreads();
    lo = fmin(fmin(red[0][0], red[0][1]), fmin(red[0][2], red[0][3]));
    hi = fmax(fmax(red[1][0], red[1][1]), fmax(red[1][2], red[1][3]));
    emax = fmax(fmax(red[2][0], red[2][1]), fmax(red[2][2], red[2][3]));
    const double tnorm = fmax(fabs(lo), fabs(hi));
    const double pivmin = kSafmin * fmax(1.0, emax);
    const double pad = 2.0 * kEps * tnorm * k + 2.0 * pivmin;
    const double gl = lo - pad, gu = hi + pad;
    int ex;
    (void)frexp(tnorm, &ex);
    const double ts = ldexp(1.0, -ex);   // the Sturm counts' scale
    if (blockIdx.x == 0 && tid == 0) {
        sc[3] = ts;
        sc[4] = gl;
        sc[5] = gu;
        sc[6] = pivmin;
        sc[7] = tnorm;
    }
    for (int i = tid; i + 1 < k; i += kLThreads) {
        const double es = eg[i] * ts;
        e2[i] = es * es;
    }
    __syncthreads();
    const int j = blockIdx.x * (kLThreads / 64) + wave;
    if (j >= nwant) return;
    const double atol = kEps * tnorm;
    double a = gl, b = gu;
    for (int it = 0; it < 40; ++it) {
        if (b - a <= fmax(atol, 2.0 * kEps * fmax(fabs(a), fabs(b))) + 2.0 * pivmin) break;   // uniform
        const double w = b - a;
        const double x = a + w * (double)(lane + 1) * (1.0 / 65.0);
        const int cnt = sturm_count(d, e2, k, x, ts);
        const uint64_t bal = __ballot(cnt > j);
        const int f = bal ? __builtin_ctzll(bal) : 64;   // first point with lambda_j below it
        const double na = f > 0 ? a + w * (double)f * (1.0 / 65.0) : a;
        const double nb = f < 64 ? a + w * (double)(f + 1) * (1.0 / 65.0) : b;
        a = na;
        b = nb;
    }
    if (lane == 0) theta[j] = 0.5 * (a + b);
}

// eigenvectors of the tridiagonal matrix for the eigenvalues k_rrl_bisect found (one
// work-group of kRRThreads)
__global__ __launch_bounds__(kRRThreads) void k_rrl_teig(int k, int nwant, double* __restrict__ base,
                                                         double* __restrict__ gamma, int32_t* __restrict__ info,
                                                         double* gamma_host, int32_t* info_host) {
    if (rrl_failed(base)) return;
    const int nwp = nwant | 1;
    const RRLLayout Lo = rrl_layout(k, nwp);
    double* d = base + Lo.d;
    double* e = base + Lo.e;
    double* theta = base + Lo.theta;
    double* sc = base + Lo.sc;
    int* cstart = (int*)(base + Lo.icl);
    int* csize = cstart + k;
    int* ncl = csize + k;
    // theta and sc[3..7] come from k_rrl_bisect
    // LABPSD's wanted Ritz values lie dense in a narrow band: clusters at 1e-3 ||T|| chain
    // into hundreds of vectors, at 1e-5 ||T|| (vectors orthogonal to ~1e-11 outside
    // them) they stay a few wide
    inverse_iteration(d, e, k, nwant, nwp, theta, base + Lo.sh, base + Lo.Zt, base + Lo.U3, cstart, csize, ncl,
                      sc[7], 1e-5);
    const int tid = threadIdx.x;
    for (int q = tid; q < nwant; q += blockDim.x) {
        gamma[q] = theta[q];
        if (gamma_host) gamma_host[q] = theta[q];
    }
    if (tid == 0) {
        info[0] = 0;
        info[1] = 0;
        if (info_host) { info_host[0] = 0; info_host[1] = 0; }
    }
}

// The compact-WY factor T of every block of kLT reflectors (one work-group per block):
// T upper triangular from tau and V^T V, wyt[kLT kLT b + kLT r + c] = T(r, c) for block b
// (reflectors kLT b .. kLT b + kLT - 1).  Every 16-column slice of the back-transformation
// applies the same blocks, so T is formed once here rather than in each of them.
__global__ __launch_bounds__(kLThreads) void k_rrl_wyt(int k, int nwant, double* __restrict__ base) {
    if (rrl_failed(base)) return;
    const int nwp = nwant | 1;
    const RRLLayout Lo = rrl_layout(k, nwp);
    const int64_t kp = rrl_kp(k);
    const double* C = base + Lo.Y;
    const double* tau = base + Lo.tau;
    double* wyt = base + Lo.wyt;
    const int tid = threadIdx.x, wave = tid >> 6;
    __shared__ double red[4][256];
    __shared__ double lpp[16][17], tm[16][17];
    const int i = tid >> 4, j = tid & 15;
    const int nref = k - 2;
    const int j0 = (int)blockIdx.x * kLT;
    const int nb = min(kLT, nref - j0);
    // V(row, c): 0 above row j0 + c + 1, 1 there, the stored entries below
    auto vv = [&](int row, int c) -> double {
        const int top = j0 + c + 1;
        if (c >= nb || row < top || row >= k) return 0.0;
        return row == top ? 1.0 : C[row + (int64_t)(j0 + c) * kp];
    };
    rr_double4 accG = {0.0, 0.0, 0.0, 0.0};
    accG = mfma_tile([&](int c, int row) { return vv(row, c); },
                     [&](int row, int b) { return vv(row, b); }, j0, (int)kp, wave, 4, accG);
    tile_to_lds(accG, red);
    __syncthreads();
    lpp[i][j] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];   // V^T V
    __syncthreads();
    // T: column c from columns < c
    if (tid < 16) {
        const int r = tid;
        for (int c = 0; c < 16; ++c) {
            double v = 0.0;
            if (c < nb && r <= c) {
                const double tc = tau[j0 + c];
                if (r == c) {
                    v = tc;
                } else {
                    double acc = 0.0;
                    for (int m = r; m < c; ++m) acc = fma(tm[r][m], lpp[m][c], acc);
                    v = -tc * acc;
                }
            }
            tm[r][c] = v;
        }
    }
    __syncthreads();
    wyt[(int64_t)blockIdx.x * (kLT * kLT) + tid] = tm[i][j];
}

// W(:, slice) = D L^{-T} Q Z(:, slice) for the 16-column slice blockIdx.x.  XLDS: the
// slice (kp x 16) lives in dynamic LDS for the whole kernel, else in the workspace.
template <bool XLDS>
__global__ __launch_bounds__(kLThreads) void k_rrl_back(int k, int nwant, double* __restrict__ base,
                                                        double* __restrict__ W, int64_t ldw) {
    if (rrl_failed(base)) return;
    const int nwp = nwant | 1;
    const RRLLayout Lo = rrl_layout(k, nwp);
    const int64_t kp = rrl_kp(k);
    const int nrb = (int)(kp / kLT);
    const double* C = base + Lo.Y;
    const double* Zt = base + Lo.Zt;
    const double* L = base + Lo.L;
    const double* At = base + Lo.A;
    const double* D = base + Lo.D;
    const double* wyt = base + Lo.wyt;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int q0 = blockIdx.x * kLT;
    extern __shared__ double xdyn[];
    double* X = XLDS ? xdyn : base + Lo.B + (int64_t)blockIdx.x * kp * kLT;
    __shared__ double red[4][256];
    __shared__ double t[16][17], lpp[16][17], tm[16][17], w2[16][17];
    for (int64_t el = tid; el < kp * kLT; el += kLThreads) {
        const int64_t row = el >> 4;
        const int q = q0 + (int)(el & 15);
        X[el] = (row < k && q < nwant) ? Zt[row * nwp + q] : 0.0;
    }
    __syncthreads();
    // X <- H_j0 ... H_j0+15 X for the blocks of 16 reflectors from the last one down, in
    // compact WY form I - V T V^T (V: the block's reflectors, rows j0.. kp; T from
    // k_rrl_wyt): X -= V (T (V^T X))
    const int i = tid >> 4, j = tid & 15;
    const int nref = k - 2;
    for (int j0 = (nref - 1) / kLT * kLT; j0 >= 0; j0 -= kLT) {
        const int nb = min(kLT, nref - j0);
        // V(row, c): 0 above row j0 + c + 1, 1 there, the stored entries below
        auto vv = [&](int row, int c) -> double {
            const int top = j0 + c + 1;
            if (c >= nb || row < top || row >= k) return 0.0;
            return row == top ? 1.0 : C[row + (int64_t)(j0 + c) * kp];
        };
        const double tij = wyt[(int64_t)(j0 / kLT) * (kLT * kLT) + tid];
        rr_double4 accW = {0.0, 0.0, 0.0, 0.0};
        accW = mfma_tile([&](int c, int row) { return vv(row, c); },
                         [&](int row, int b) { return X[(int64_t)row * kLT + b]; }, j0, (int)kp, wave, 4, accW);
        tile_to_lds(accW, red);
        tm[i][j] = tij;
        __syncthreads();
        t[i][j] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];   // V^T X
        __syncthreads();
        // W2 = T (V^T X)
        {
            double acc = 0.0;
#pragma unroll
            for (int m = 0; m < 16; ++m) acc = fma(tm[i][m], t[m][j], acc);
            w2[i][j] = acc;
        }
        __syncthreads();
        // X(rows, :) -= V(rows, :) W2, one 16-row tile per wavefront at a time
        for (int rt = j0 / kLT + wave; rt < (int)(kp / kLT); rt += 4) {
            const int row0 = rt * kLT;
            rr_double4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                const int c = 4 * s4 + (lane >> 4);
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(vv(row0 + (lane & 15), c), w2[c][lane & 15], acc, 0, 0, 0);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t el = (int64_t)(row0 + 4 * q + (lane >> 4)) * kLT + (lane & 15);
                X[el] -= acc[q];
            }
        }
        __syncthreads();
    }
    // L^T Y = X, row tiles from the bottom; Y overwrites X
    for (int p = nrb - 1; p >= 0; --p) {
        const int p0 = p * kLT;
        rr_double4 acc = {0.0, 0.0, 0.0, 0.0};
        acc = mfma_tile([&](int a, int kc) { return At[(p0 + a) + (int64_t)kc * kp]; },
                        [&](int kc, int b) { return X[(int64_t)kc * kLT + b]; }, p0 + kLT, (int)kp, wave, 4, acc);
        tile_to_lds(acc, red);
        const double xv = X[(int64_t)(p0 + i) * kLT + j];
        lpp[i][j] = L[(p0 + i) + (int64_t)(p0 + j) * kp];
        __syncthreads();
        t[i][j] = xv - (red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid]);
        __syncthreads();
        if (tid < 16) {
            for (int a = 15; a >= 0; --a) {
                double v = t[a][tid];
                for (int b2 = a + 1; b2 < 16; ++b2) v -= lpp[b2][a] * t[b2][tid];
                t[a][tid] = v / lpp[a][a];
            }
        }
        __syncthreads();
        const double y = t[i][j];
        X[(int64_t)(p0 + i) * kLT + j] = y;
        if (p0 + i < k && q0 + j < nwant) W[(p0 + i) + (int64_t)(q0 + j) * ldw] = D[p0 + i] * y;
        __syncthreads();
    }
}

}  // namespace

size_t rr_ws_bytes(int k) {
    // the layout at the widest nwant (= k) plus the k x k product scratch and alignment;
    // large orders also run the many-work-group route in the same workspace
    const RRLayout L = rr_layout(k, k | 1);
    size_t n = (size_t)L.total + (size_t)k * k + 4;
    if (k >= kRRLargeMin) n = std::max(n, (size_t)rrl_layout(k, k | 1).total + 4);
    return sizeof(double) * n;
}

namespace {

// the device's LDS per work-group (initialised once, thread-safely: slot threads of the
// server launch Rayleigh-Ritz steps concurrently)
static int device_lds_per_block() {
    static const int v = [] {
        int dev = 0, x = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&x, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            x = 64 * 1024;
        (void)hipGetLastError();
        return x;
    }();
    return v;
}

// the many-work-group route for k >= kRRLargeMin; the one-work-group kernel follows it
// and runs only if the route gave up (or runs in its place if the cooperative launch
// is refused)
void launch_rr_large(int k, int nwant, const double* HR, const double* SR, int64_t ldr, double* gamma,
                     double* W, int64_t ldw, int32_t* info, void* ws, hipStream_t s, double* gamma_host,
                     int32_t* info_host) {
    double* gws = (double*)ws;
    double* base = gws + (((uintptr_t)gws & 15) ? 1 : 0);
    const int kp = rrl_kp(k), nrb = kp / kLT;
    const int64_t kk = (int64_t)kp * kp;
    const int prep_blocks = (int)std::min<int64_t>(2048, (kk + kLThreads - 1) / kLThreads);
    hipLaunchKernelGGL(k_rrl_prep, dim3(prep_blocks), dim3(kLThreads), 0, s, k, HR, SR, ldr, base);
    for (int p = 0; p < nrb; ++p)
        hipLaunchKernelGGL(k_rrl_chol, dim3(nrb - p), dim3(kLThreads), 0, s, k, p, base);
    const RRLLayout Lo = rrl_layout(k, 1);
    hipLaunchKernelGGL(k_rrl_fwd, dim3(nrb), dim3(kLThreads), 0, s, k, (const double*)(base + Lo.B), 0,
                       base + Lo.Y, base);
    hipLaunchKernelGGL(k_rrl_fwd, dim3(nrb), dim3(kLThreads), 0, s, k, (const double*)(base + Lo.Y), 1,
                       base + Lo.B, base);
    hipLaunchKernelGGL(k_rrl_sym, dim3(prep_blocks), dim3(kLThreads), 0, s, k, base);
    LABPSD_HIP(hipGetLastError());
    // about eight columns per work-group, kept in LDS when they fit
    const int G = std::min(128, std::max(8, (k + 7) / 8));
    const size_t lds_own = (4 + (size_t)((k + G - 1) / G)) * (size_t)kp * sizeof(double);
    const bool own_lds = lds_own + 1024 <= (size_t)device_lds_per_block();
    const size_t lds = own_lds ? lds_own : 4 * (size_t)kp * sizeof(double);
    const void* tridiag = own_lds ? (const void*)k_rrl_tridiag<true> : (const void*)k_rrl_tridiag<false>;
    if (lds + 1024 > 64 * 1024) allow_dynamic_lds(tridiag);
    int kk_arg = k;
    double* base_arg = base;
    void* targs[] = {(void*)&kk_arg, (void*)&base_arg};
    const int32_t* run_if = (const int32_t*)base;
    if (hipLaunchCooperativeKernel(tridiag, dim3(G), dim3(kLThreads), targs,
                                   (unsigned)lds, s) == hipSuccess &&
        hipGetLastError() == hipSuccess) {
        const size_t bl = 2 * (size_t)kp * sizeof(double);
        if (bl + 1024 > 64 * 1024) allow_dynamic_lds((const void*)k_rrl_bisect);
        hipLaunchKernelGGL(k_rrl_bisect, dim3((nwant + 3) / 4), dim3(kLThreads), bl, s, k, nwant, base);
        hipLaunchKernelGGL(k_rrl_teig, dim3(1), dim3(kRRThreads), 0, s, k, nwant, base, gamma, info, gamma_host,
                           info_host);
        hipLaunchKernelGGL(k_rrl_wyt, dim3((unsigned)rrl_wy_blocks(k)), dim3(kLThreads), 0, s, k, nwant, base);
        // the 16-column slice in LDS when it fits beside the kernel's static LDS (about 18 KB)
        const size_t xl = (size_t)kp * kLT * sizeof(double);
        const bool xlds = xl + 20 * 1024 <= (size_t)device_lds_per_block();
        const void* back = xlds ? (const void*)k_rrl_back<true> : (const void*)k_rrl_back<false>;
        if (xlds && xl > 32 * 1024) allow_dynamic_lds(back);
        void* bargs[] = {(void*)&k, (void*)&nwant, (void*)&base, (void*)&W, (void*)&ldw};
        LABPSD_HIP(hipLaunchKernel(back, dim3((nwant + kLT - 1) / kLT), dim3(kLThreads), bargs, xlds ? xl : 0, s));
        LABPSD_HIP(hipGetLastError());
    } else {
        (void)hipGetLastError();
        run_if = nullptr;   // nothing ran: the one-work-group kernel solves the pencil
    }
    void* args[] = {(void*)&k,    (void*)&nwant, (void*)&HR, (void*)&SR, (void*)&ldr,
                    (void*)&gamma, (void*)&W,    (void*)&ldw, (void*)&info, (void*)&ws,
                    (void*)&gamma_host, (void*)&info_host, (void*)&run_if};
    LABPSD_HIP(hipLaunchKernel((const void*)k_rayleigh_ritz<false, 0>, dim3(1), dim3(kRRThreads), args, 0, s));
    LABPSD_HIP(hipGetLastError());
}

}  // namespace

void launch_rayleigh_ritz(int k, int nwant, const double* HR, const double* SR, int64_t ldr,
                          double* gamma, double* W, int64_t ldw, int32_t* info, void* ws,
                          hipStream_t s, double* gamma_host, int32_t* info_host) {
    if (k <= 0 || nwant <= 0) return;
    LABPSD_REQUIRE(k <= kRRMax, "Rayleigh-Ritz order exceeds the supported maximum");
    LABPSD_REQUIRE(nwant <= k, "more Ritz pairs requested than the search space holds");
    if (k >= kRRLargeMin) {
        launch_rr_large(k, nwant, HR, SR, ldr, gamma, W, ldw, info, ws, s, gamma_host, info_host);
        return;
    }
    const int lds_limit = device_lds_per_block();
    const RRLayout L = rr_layout(k, nwant | 1);
    const size_t bytes = (size_t)L.total * sizeof(double);
    // register-row width: 8 lanes per row, NT columns per lane
    const int nt = rr_nt(k);
    // the static LDS of the kernel (the reduction array) stays below 1 KiB
    const bool all_lds = lds_limit > 2048 && bytes <= (size_t)lds_limit - 1024;
    auto pick = [&](auto lds_tag) -> const void* {
        constexpr bool L_ = decltype(lds_tag)::value;
        switch (nt) {
            case 5: return (const void*)k_rayleigh_ritz<L_, 5>;
            case 9: return (const void*)k_rayleigh_ritz<L_, 9>;
            case 16: return (const void*)k_rayleigh_ritz<L_, 16>;
            default: return (const void*)k_rayleigh_ritz<L_, 0>;
        }
    };
    const int32_t* run_if = nullptr;
    void* args[] = {(void*)&k,    (void*)&nwant, (void*)&HR, (void*)&SR, (void*)&ldr,
                    (void*)&gamma, (void*)&W,    (void*)&ldw, (void*)&info, (void*)&ws,
                    (void*)&gamma_host, (void*)&info_host, (void*)&run_if};
    if (all_lds) {
        const void* f = pick(std::true_type{});
        if (bytes > 64 * 1024) allow_dynamic_lds(f);
        if (hipLaunchKernel(f, dim3(1), dim3(kRRThreads), args, bytes, s) == hipSuccess &&
            hipGetLastError() == hipSuccess)
            return;
        // the launch was refused (nothing ran): use the global-memory variant
    }
    LABPSD_HIP(hipLaunchKernel(pick(std::false_type{}), dim3(1), dim3(kRRThreads), args, 0, s));
    LABPSD_HIP(hipGetLastError());
}

}  // namespace labpsd
