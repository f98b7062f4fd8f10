// Tall-skinny dense steps of one LABPSD iteration:
//   residual block and Res (outline step 4, eq. (res1)),
//   Gram matrices H_R = Z^T (HZ), S_R = Z^T (SZ) (step 8) on FP64 matrix cores,
//   block update [Psi P] W for Psi, Psi_H, Psi_S (steps 10-11) on FP64 matrix cores,
//   and the gathers / precision casts between the FP64 blocks and the preconditioner.
#include "common.h"

namespace labpsd {

namespace {

typedef double double4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// ------------------------------------------------------------------ residual

constexpr int kResRows = 4096;   // rows per residual work-group

// grid (nblk, m): column j of R = PsiH_j - E_j PsiS_j; partial sums of ||r||^2 and
// ||PsiH_j - sigma0 PsiS_j||^2 per work-group
__global__ __launch_bounds__(256) void k_residual(int64_t n, const double* __restrict__ PsiH,
                                                  const double* __restrict__ PsiS, int64_t ld,
                                                  const double* __restrict__ E, double sigma0,
                                                  double* __restrict__ R, int64_t ldr,
                                                  double* __restrict__ partial) {
    const int j = blockIdx.y;
    const double e = E[j];
    const double* h = PsiH + (int64_t)j * ld;
    const double* s = PsiS + (int64_t)j * ld;
    double* r = R + (int64_t)j * ldr;
    const int64_t r0 = (int64_t)blockIdx.x * kResRows;
    const int64_t r1 = min(n, r0 + kResRows);
    double num = 0.0, den = 0.0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) {
        const double hi = h[i], si = s[i];
        const double ri = hi - e * si;
        r[i] = ri;
        num = fma(ri, ri, num);
        const double di = hi - sigma0 * si;
        den = fma(di, di, den);
    }
    __shared__ double sh[2][4];
    num = wave_sum(num);
    den = wave_sum(den);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { sh[0][wv] = num; sh[1][wv] = den; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int k = 0; k < 4; ++k) { a += sh[0][k]; b += sh[1][k]; }
        partial[((int64_t)j * gridDim.x + blockIdx.x) * 2 + 0] = a;
        partial[((int64_t)j * gridDim.x + blockIdx.x) * 2 + 1] = b;
    }
}

__global__ void k_residual_finish(int m, const double* __restrict__ partial, int nblk,
                                  double* __restrict__ res, double* __restrict__ rnorm,
                                  double* __restrict__ host, const int32_t* __restrict__ flag_src,
                                  int32_t* __restrict__ flag_dst) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (flag_dst && j == 0)   // an error word of earlier work, carried to the host with Res
        flag_dst[0] = flag_src ? __hip_atomic_load(flag_src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
    if (j >= m) return;
    double a = 0.0, b = 0.0;
    for (int k = 0; k < nblk; ++k) {
        a += partial[((int64_t)j * nblk + k) * 2 + 0];
        b += partial[((int64_t)j * nblk + k) * 2 + 1];
    }
    const double rn = sqrt(a), r = b > 0.0 ? sqrt(a / b) : (a > 0.0 ? INFINITY : 0.0);
    rnorm[j] = rn;
    res[j] = r;
    if (host) {   // pinned host memory, device-mapped: [Res | norms]
        host[j] = r;
        host[m + j] = rn;
    }
}

// ------------------------------------------------------------------ seeded start block

// splitmix64 output function (Steele, Lea and Flood, OOPSLA 2014) applied to a
// counter: the k-th output of the generator started at `seed`.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// X(i, j) = Box-Muller normal from outputs 2c and 2c + 1, c = i + n j
__global__ __launch_bounds__(256) void k_random_block(int64_t n, int64_t total, uint64_t seed,
                                                      double* __restrict__ X, int64_t ldx) {
    for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < total; c += (int64_t)gridDim.x * 256) {
        const uint64_t a = splitmix64_at(seed, 2 * (uint64_t)c), b = splitmix64_at(seed, 2 * (uint64_t)c + 1);
        const double u1 = (double)((a >> 11) + 1) * 0x1.0p-53;   // (0, 1]
        const double u2 = (double)(b >> 11) * 0x1.0p-53;         // [0, 1)
        const double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
        const int64_t i = c % n, j = c / n;
        X[i + j * ldx] = z;
    }
}

// ------------------------------------------------------------------ complex embedding

// dst = J src (transpose = false) or J^T src for interleaved complex columns, J the real
// form of multiplication by i: (J v)_{2k} = -v_{2k+1}, (J v)_{2k+1} = v_{2k}
__global__ __launch_bounds__(256) void k_apply_j(int64_t nc, const double* __restrict__ src, int64_t lds,
                                                 double* __restrict__ dst, int64_t ldd, int transpose) {
    const int j = blockIdx.y;
    const double* a = src + (int64_t)j * lds;
    double* d = dst + (int64_t)j * ldd;
    const double sg = transpose ? -1.0 : 1.0;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < nc; k += (int64_t)gridDim.x * 256) {
        const double re = a[2 * k], im = a[2 * k + 1];
        d[2 * k] = -sg * im;
        d[2 * k + 1] = sg * re;
    }
}

// ------------------------------------------------------------------ gather / cast

template <typename TS, typename TD>
__global__ __launch_bounds__(256) void k_gather_cast(int64_t n, const TS* __restrict__ src,
                                                     int64_t lds, const int32_t* __restrict__ cols,
                                                     double scale, TD* __restrict__ dst,
                                                     int64_t ldd) {
    const int j = blockIdx.y;
    const int64_t sc = cols ? cols[j] : j;
    const TS* a = src + sc * lds;
    TD* b = dst + (int64_t)j * ldd;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        b[i] = (TD)((double)a[i] * scale);
}

template <typename TS, typename TD>
__global__ __launch_bounds__(256) void k_scatter_cast(int64_t n, const TS* __restrict__ src,
                                                      int64_t lds, const int32_t* __restrict__ cols,
                                                      double scale, TD* __restrict__ dst,
                                                      int64_t ldd) {
    const int j = blockIdx.y;
    const TS* a = src + (int64_t)j * lds;
    TD* b = dst + (int64_t)cols[j] * ldd;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        b[i] = (TD)((double)a[i] * scale);
}

// Column-major <-> row-major casts through a 64-row x 32-column LDS tile, so both the
// column-major side (rows contiguous) and the row-major side (the ncols values of a
// row contiguous) are read and written in whole cache lines.
// to_rm:   dst[i * ncols + j] = (TD) src[i + cols[j] * lds] * scale  (cols may be null)
// to_cm:   dst[i + j * ldd]   = (TD) src[i * ncols + j] * scale
template <typename TS, typename TD, bool TO_RM>
__global__ __launch_bounds__(256) void k_transpose_cast(int64_t n, int ncols, const TS* __restrict__ src,
                                                        int64_t lds, const int32_t* __restrict__ cols,
                                                        double scale, TD* __restrict__ dst, int64_t ldd) {
    __shared__ double tile[32][65];
    const int t = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int j0 = blockIdx.y * 32;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        int ii, jj;
        if (TO_RM) { ii = t % 64; jj = t / 64 + 4 * k; }    // column-major read
        else { jj = t % 32; ii = t / 32 + 8 * k; }          // row-major read
        const int64_t i = i0 + ii;
        const int j = j0 + jj;
        double v = 0.0;
        if (i < n && j < ncols) {
            if (TO_RM) v = (double)src[i + (int64_t)(cols ? cols[j] : j) * lds];
            else v = (double)src[i * ncols + j];
        }
        tile[jj][ii] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        int ii, jj;
        if (TO_RM) { jj = t % 32; ii = t / 32 + 8 * k; }    // row-major write
        else { ii = t % 64; jj = t / 64 + 4 * k; }          // column-major write
        const int64_t i = i0 + ii;
        const int j = j0 + jj;
        if (i < n && j < ncols) {
            const TD v = (TD)(tile[jj][ii] * scale);
            if (TO_RM) dst[i * ncols + j] = v;
            else dst[i + (int64_t)j * ldd] = v;
        }
    }
}

// partial sums of squares of the columns cols[j] (or j) per block of rows
template <typename T>
__global__ __launch_bounds__(256) void k_colnorm_partial(int64_t n, const T* __restrict__ src,
                                                         int64_t ld, const int32_t* __restrict__ cols,
                                                         double* __restrict__ partial) {
    const int j = blockIdx.y;
    const T* a = src + (int64_t)(cols ? cols[j] : j) * ld;
    const int64_t r0 = (int64_t)blockIdx.x * kResRows, r1 = min(n, r0 + kResRows);
    double acc = 0.0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) {
        const double v = (double)a[i];
        acc = fma(v, v, acc);
    }
    __shared__ double sh[4];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[(int64_t)j * gridDim.x + blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ void k_colnorm_finish(int q, const double* __restrict__ partial, int nblk,
                                 double* __restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= q) return;
    double a = 0.0;
    for (int k = 0; k < nblk; ++k) a += partial[(int64_t)j * nblk + k];
    out[j] = sqrt(a);
}

// ------------------------------------------------------------------ Gram on MFMA

// Output tile GT x GT per work-group (GT = 32 or 64): four wavefronts in a 2 x 2 grid,
// each one (GT/2) x (GT/2) block of both H_R and S_R as (GT/32)^2 MFMA tiles of 16 x 16.
// Rows of Z are staged in LDS GR at a time, transposed so that each lane's MFMA operand
// (row k, column i) is a conflict-free LDS read.  The 64 x 64 tile doubles the products
// per staged byte; it is used from k = 192 up (below, its padding of k costs more).
template <int GT, int GR>
__global__ __launch_bounds__(256) void k_gram(int64_t n, int k, const double* __restrict__ Z,
                                              const double* __restrict__ ZH,
                                              const double* __restrict__ ZS, int64_t ld, int nb,
                                              int64_t rows_per_chunk, double* __restrict__ part,
                                              int kp) {
    constexpr int TW = GT / 32;   // MFMA tiles per wavefront and direction
    int p = blockIdx.x, bi = 0;
    while (p >= nb - bi) { p -= nb - bi; ++bi; }
    const int bj = bi + p;
    const int i0 = bi * GT, j0 = bj * GT;
    __shared__ double sZ[GT][GR + 1];
    __shared__ double sH[GT][GR + 1];
    __shared__ double sS[GT][GR + 1];
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    const int ti = wave >> 1, tj = wave & 1;
    double4_t aH[TW][TW], aS[TW][TW];
#pragma unroll
    for (int u = 0; u < TW; ++u)
#pragma unroll
        for (int v = 0; v < TW; ++v) {
            aH[u][v] = double4_t{0.0, 0.0, 0.0, 0.0};
            aS[u][v] = double4_t{0.0, 0.0, 0.0, 0.0};
        }
    const int64_t rb = (int64_t)blockIdx.y * rows_per_chunk;
    const int64_t re = min(n, rb + rows_per_chunk);
    // a stage's loads are all issued before any is used (out-of-range elements read a
    // valid one and are zeroed), and the next stage is fetched into registers while the
    // current one is multiplied
    constexpr int NQ = (GT * GR) / 256;
    double vz[NQ], vh[NQ], vs[NQ];
    auto load_stage = [&](int64_t r0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int e = t + 256 * q;
            const int rr = e & (GR - 1), cc = e / GR;
            const int64_t row = r0 + rr;
            const bool okr = row < re, okz = okr && i0 + cc < k, okc = okr && j0 + cc < k;
            const int64_t rowc = okr ? row : rb;
            const double z = Z[rowc + (int64_t)(i0 + cc < k ? i0 + cc : 0) * ld];
            const int64_t hcol = (int64_t)(j0 + cc < k ? j0 + cc : 0) * ld;
            const double h = ZH[rowc + hcol], sv = ZS[rowc + hcol];
            vz[q] = okz ? z : 0.0;
            vh[q] = okc ? h : 0.0;
            vs[q] = okc ? sv : 0.0;
        }
    };
    if (rb < re) load_stage(rb);
    for (int64_t r0 = rb; r0 < re; r0 += GR) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int e = t + 256 * q;
            const int rr = e & (GR - 1), cc = e / GR;
            sZ[cc][rr] = vz[q];
            sH[cc][rr] = vh[q];
            sS[cc][rr] = vs[q];
        }
        __syncthreads();
        if (r0 + GR < re) load_stage(r0 + GR);
#pragma unroll 2
        for (int kk = 0; kk < GR; kk += 4) {
            const int kr = kk + (lane >> 4);
            double a[TW], h[TW], sv[TW];
#pragma unroll
            for (int u = 0; u < TW; ++u) {
                a[u] = sZ[ti * (GT / 2) + 16 * u + (lane & 15)][kr];
                h[u] = sH[tj * (GT / 2) + 16 * u + (lane & 15)][kr];
                sv[u] = sS[tj * (GT / 2) + 16 * u + (lane & 15)][kr];
            }
#pragma unroll
            for (int u = 0; u < TW; ++u)
#pragma unroll
                for (int v = 0; v < TW; ++v) {
                    aH[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], h[v], aH[u][v], 0, 0, 0);
                    aS[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], sv[v], aS[u][v], 0, 0, 0);
                }
        }
        __syncthreads();
    }
    double* ph = part + (int64_t)blockIdx.y * 2 * kp * kp;
    double* ps = ph + (int64_t)kp * kp;
    // accumulator layout of the f64 16x16x4 MFMA on gfx950 (measured): register q of
    // lane l holds row 4q + l / 16 and column l % 16 of the 16 x 16 tile
#pragma unroll
    for (int u = 0; u < TW; ++u)
#pragma unroll
        for (int v = 0; v < TW; ++v)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int ii = i0 + ti * (GT / 2) + 16 * u + 4 * q + (lane >> 4);
                const int jj = j0 + tj * (GT / 2) + 16 * v + (lane & 15);
                ph[ii + (int64_t)jj * kp] = aH[u][v][q];
                ps[ii + (int64_t)jj * kp] = aS[u][v][q];
            }
}

// sum the chunk partials of the upper triangle (i <= j) and mirror it: eight lanes per
// element, lane u summing chunks u, u + 8, ..., then a fixed-order 8-lane sum (the same
// result on every run)
__global__ __launch_bounds__(256) void k_gram_reduce(int k, int kp, int nchunk,
                                                     const double* __restrict__ part,
                                                     double* __restrict__ HR,
                                                     double* __restrict__ SR, int64_t ldr) {
    const int64_t idx = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 3;
    const int u = threadIdx.x & 7;
    const bool in = idx < (int64_t)k * k;
    const int i = in ? (int)(idx % k) : 0, j = in ? (int)(idx / k) : 0;
    const bool act = in && i <= j;
    const int64_t stride = (int64_t)kp * kp, off = i + (int64_t)j * kp;
    double h = 0.0, s = 0.0;
    if (act)
        for (int c = u; c < nchunk; c += 8) {
            h += part[((int64_t)c * 2 + 0) * stride + off];
            s += part[((int64_t)c * 2 + 1) * stride + off];
        }
    // the 8 lanes of an element share a DPP half-row; every lane takes part
    h = row8_allsum(h);
    s = row8_allsum(s);
    if (act && u == 0) {
        HR[i + (int64_t)j * ldr] = h;
        HR[j + (int64_t)i * ldr] = h;
        SR[i + (int64_t)j * ldr] = s;
        SR[j + (int64_t)i * ldr] = s;
    }
}

// ------------------------------------------------------------------ block update on MFMA

// out = Zm W for the three (Zm, out) pairs (grid.z).  Work-group tile: 64 rows x 32
// columns; wavefront w owns rows [16w, 16w+16) and both 16-column halves.
__global__ __launch_bounds__(256) void k_block_update(int64_t n, int k, int b,
                                                      const double* __restrict__ Z0,
                                                      const double* __restrict__ Z1,
                                                      const double* __restrict__ Z2, int64_t ldz,
                                                      const double* __restrict__ W, int64_t ldw,
                                                      double* __restrict__ O0,
                                                      double* __restrict__ O1,
                                                      double* __restrict__ O2, int64_t ldo) {
    const double* Zm = blockIdx.z == 0 ? Z0 : (blockIdx.z == 1 ? Z1 : Z2);
    double* O = blockIdx.z == 0 ? O0 : (blockIdx.z == 1 ? O1 : O2);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t r0 = (int64_t)blockIdx.x * 64 + wave * 16;
    const int c0 = blockIdx.y * 32;
    const int64_t arow = r0 + (lane & 15);
    const int kq = lane >> 4;
    const int bc0 = c0 + (lane & 15), bc1 = bc0 + 16;
    double4_t acc0 = {0.0, 0.0, 0.0, 0.0};
    double4_t acc1 = {0.0, 0.0, 0.0, 0.0};
    for (int kk = 0; kk < k; kk += 4) {
        const int kr = kk + kq;
        const bool kin = kr < k;
        const double a = (kin && arow < n) ? Zm[arow + (int64_t)kr * ldz] : 0.0;
        const double w0 = (kin && bc0 < b) ? W[kr + (int64_t)bc0 * ldw] : 0.0;
        const double w1 = (kin && bc1 < b) ? W[kr + (int64_t)bc1 * ldw] : 0.0;
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, w0, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, w1, acc1, 0, 0, 0);
    }
    // accumulator layout (see k_gram): register q of lane l is row 4q + l / 16, column l % 16
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t row = r0 + 4 * q + (lane >> 4);
        if (row < n) {
            if (bc0 < b) O[row + (int64_t)bc0 * ldo] = acc0[q];
            if (bc1 < b) O[row + (int64_t)bc1 * ldo] = acc1[q];
        }
    }
}

// The same product for wide blocks (large k or b): each wavefront accumulates 16 rows x
// 16 CT columns (CT MFMA tiles), so Z is re-read b / (16 CT) times instead of b / 32; W
// passes through LDS in 16-row chunks (double-buffered, shared by the four wavefronts,
// rows padded by one element against bank conflicts) and the next chunk's Z operands and
// W entries are loaded while the current chunk's MFMAs run.  CT (6, 8 or 9) is chosen
// per launch to pad b the least.
template <int CT>
__global__ __launch_bounds__(256) void k_block_update_wide(int64_t n, int k, int b,
                                                           const double* __restrict__ Z0,
                                                           const double* __restrict__ Z1,
                                                           const double* __restrict__ Z2, int64_t ldz,
                                                           const double* __restrict__ W, int64_t ldw,
                                                           double* __restrict__ O0,
                                                           double* __restrict__ O1,
                                                           double* __restrict__ O2, int64_t ldo) {
    constexpr int NC = 16 * CT;               // columns per work-group
    constexpr int WL = 16 * NC / 256;         // W entries per thread per chunk
    __shared__ double Wl[2][16][NC + 1];   // + 1: the four k-rows a wavefront reads fall in different banks
    const double* Zm = blockIdx.z == 0 ? Z0 : (blockIdx.z == 1 ? Z1 : Z2);
    double* O = blockIdx.z == 0 ? O0 : (blockIdx.z == 1 ? O1 : O2);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t r0 = (int64_t)blockIdx.x * 64 + wave * 16;
    const int c0 = blockIdx.y * NC;
    const int64_t arow = r0 + (lane & 15);
    const bool rin = arow < n;
    const int kq = lane >> 4;
    const int nchunk = (k + 15) / 16;
    double an[4], wn[WL];
    auto load = [&](int ch) {
        const int kb = ch * 16;
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const int kr = kb + 4 * s4 + kq;
            an[s4] = (rin && kr < k) ? Zm[arow + (int64_t)kr * ldz] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < WL; ++u) {
            const int r = tid & 15, c = (tid >> 4) + 16 * u;
            const int kr = kb + r;
            wn[u] = (kr < k && c0 + c < b) ? W[kr + (int64_t)(c0 + c) * ldw] : 0.0;
        }
    };
    auto stage = [&](int buf) {
#pragma unroll
        for (int u = 0; u < WL; ++u) Wl[buf][tid & 15][(tid >> 4) + 16 * u] = wn[u];
    };
    double4_t acc[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[ct] = double4_t{0.0, 0.0, 0.0, 0.0};
    load(0);
    stage(0);
    __syncthreads();
    for (int ch = 0; ch < nchunk; ++ch) {
        double a[4];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) a[s4] = an[s4];
        const bool more = ch + 1 < nchunk;
        if (more) load(ch + 1);
        const int buf = ch & 1;
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
                acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s4], Wl[buf][4 * s4 + kq][16 * ct + (lane & 15)],
                                                               acc[ct], 0, 0, 0);
        }
        if (more) stage(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
        const int col = c0 + 16 * ct + (lane & 15);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t row = r0 + 4 * q + (lane >> 4);
            if (row < n && col < b) O[row + (int64_t)col * ldo] = acc[ct][q];
        }
    }
}

// max |SR - I| over the b x b matrix SR (ld ld), one work-group; a NaN counts as infinite
__global__ __launch_bounds__(256) void k_orth_deviation(int b, const double* __restrict__ SR, int64_t ld,
                                                        double* __restrict__ out) {
    __shared__ double red[4];
    double mx = 0.0;
    for (int64_t e = threadIdx.x; e < (int64_t)b * b; e += 256) {
        const int64_t i = e % b, j = e / b;
        const double dv = fabs(SR[i + j * ld] - (i == j ? 1.0 : 0.0));
        mx = (dv == dv) ? fmax(mx, dv) : INFINITY;
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) *out = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

}  // namespace

void launch_random_block(int64_t n, int b, uint64_t seed, double* X, int64_t ldx, hipStream_t s) {
    const int64_t total = n * (int64_t)b;
    if (total <= 0) return;
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_random_block, dim3((unsigned)blocks), dim3(256), 0, s, n, total, seed, X, ldx);
    LABPSD_HIP(hipGetLastError());
}

void launch_apply_j(int64_t nc, int ncols, const double* src, int64_t lds, double* dst, int64_t ldd, bool transpose,
                    hipStream_t s) {
    if (nc <= 0 || ncols <= 0) return;
    const unsigned bx = (unsigned)std::min<int64_t>((nc + 255) / 256, 1024);
    hipLaunchKernelGGL(k_apply_j, dim3(bx, ncols), dim3(256), 0, s, nc, src, lds, dst, ldd, transpose ? 1 : 0);
    LABPSD_HIP(hipGetLastError());
}

int residual_blocks(int64_t n) { return (int)std::max<int64_t>(1, (n + kResRows - 1) / kResRows); }

void launch_residual(int64_t n, int m, const double* PsiH, const double* PsiS, int64_t ld,
                     const double* E, double sigma0, double* R, int64_t ldr, double* partial,
                     int nblk, hipStream_t s) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_residual, dim3(nblk, m), dim3(256), 0, s, n, PsiH, PsiS, ld, E, sigma0, R,
                       ldr, partial);
    LABPSD_HIP(hipGetLastError());
}

void launch_residual_finish(int m, const double* partial, int nblk, double* res, double* rnorm,
                            hipStream_t s, double* host, const int32_t* flag_src, int32_t* flag_dst) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_residual_finish, dim3((m + 255) / 256), dim3(256), 0, s, m, partial, nblk,
                       res, rnorm, host, flag_src, flag_dst);
    LABPSD_HIP(hipGetLastError());
}

template <typename TS, typename TD>
void launch_gather_cast(int64_t n, int ncols, const TS* src, int64_t lds, const int32_t* cols,
                        double scale, TD* dst, int64_t ldd, hipStream_t s) {
    if (ncols <= 0 || n <= 0) return;
    const int64_t bx = std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL((k_gather_cast<TS, TD>), dim3((unsigned)bx, ncols), dim3(256), 0, s, n, src,
                       lds, cols, scale, dst, ldd);
    LABPSD_HIP(hipGetLastError());
}

template void launch_gather_cast<double, double>(int64_t, int, const double*, int64_t,
                                                 const int32_t*, double, double*, int64_t,
                                                 hipStream_t);
template void launch_gather_cast<double, float>(int64_t, int, const double*, int64_t,
                                                const int32_t*, double, float*, int64_t,
                                                hipStream_t);
template void launch_gather_cast<float, double>(int64_t, int, const float*, int64_t,
                                                const int32_t*, double, double*, int64_t,
                                                hipStream_t);
template void launch_gather_cast<float, float>(int64_t, int, const float*, int64_t,
                                               const int32_t*, double, float*, int64_t,
                                               hipStream_t);

template <typename TS, typename TD>
void launch_cast_to_rm(int64_t n, int ncols, const TS* src, int64_t lds, const int32_t* cols,
                       double scale, TD* dst, hipStream_t s) {
    if (ncols <= 0 || n <= 0) return;
    const dim3 g((unsigned)((n + 63) / 64), (unsigned)((ncols + 31) / 32));
    hipLaunchKernelGGL((k_transpose_cast<TS, TD, true>), g, dim3(256), 0, s, n, ncols, src, lds, cols,
                       scale, dst, (int64_t)0);
    LABPSD_HIP(hipGetLastError());
}

template <typename TS, typename TD>
void launch_cast_from_rm(int64_t n, int ncols, const TS* src, double scale, TD* dst, int64_t ldd,
                         hipStream_t s) {
    if (ncols <= 0 || n <= 0) return;
    const dim3 g((unsigned)((n + 63) / 64), (unsigned)((ncols + 31) / 32));
    hipLaunchKernelGGL((k_transpose_cast<TS, TD, false>), g, dim3(256), 0, s, n, ncols, src, (int64_t)0,
                       (const int32_t*)nullptr, scale, dst, ldd);
    LABPSD_HIP(hipGetLastError());
}

template void launch_cast_to_rm<double, double>(int64_t, int, const double*, int64_t, const int32_t*,
                                                double, double*, hipStream_t);
template void launch_cast_to_rm<double, float>(int64_t, int, const double*, int64_t, const int32_t*,
                                               double, float*, hipStream_t);
template void launch_cast_from_rm<double, double>(int64_t, int, const double*, double, double*, int64_t,
                                                  hipStream_t);
template void launch_cast_from_rm<float, float>(int64_t, int, const float*, double, float*, int64_t,
                                                hipStream_t);
template void launch_cast_from_rm<float, double>(int64_t, int, const float*, double, double*, int64_t,
                                                 hipStream_t);

template <typename TS, typename TD>
void launch_scatter_cast(int64_t n, int ncols, const TS* src, int64_t lds, const int32_t* cols,
                         double scale, TD* dst, int64_t ldd, hipStream_t s) {
    if (ncols <= 0 || n <= 0) return;
    const int64_t bx = std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL((k_scatter_cast<TS, TD>), dim3((unsigned)bx, ncols), dim3(256), 0, s, n, src,
                       lds, cols, scale, dst, ldd);
    LABPSD_HIP(hipGetLastError());
}

template void launch_scatter_cast<double, double>(int64_t, int, const double*, int64_t,
                                                  const int32_t*, double, double*, int64_t,
                                                  hipStream_t);
template void launch_scatter_cast<float, double>(int64_t, int, const float*, int64_t,
                                                 const int32_t*, double, double*, int64_t,
                                                 hipStream_t);
template void launch_scatter_cast<double, float>(int64_t, int, const double*, int64_t,
                                                 const int32_t*, double, float*, int64_t,
                                                 hipStream_t);
template void launch_scatter_cast<float, float>(int64_t, int, const float*, int64_t,
                                                const int32_t*, double, float*, int64_t,
                                                hipStream_t);

template <typename T>
void launch_colnorms(int64_t n, int q, const T* src, int64_t ld, const int32_t* cols,
                     double* partial, double* out, hipStream_t s) {
    if (q <= 0) return;
    const int nblk = residual_blocks(n);
    hipLaunchKernelGGL((k_colnorm_partial<T>), dim3(nblk, q), dim3(256), 0, s, n, src, ld, cols,
                       partial);
    LABPSD_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_colnorm_finish, dim3((q + 255) / 256), dim3(256), 0, s, q, partial, nblk,
                       out);
    LABPSD_HIP(hipGetLastError());
}

template void launch_colnorms<double>(int64_t, int, const double*, int64_t, const int32_t*, double*,
                                      double*, hipStream_t);
template void launch_colnorms<float>(int64_t, int, const float*, int64_t, const int32_t*, double*,
                                     double*, hipStream_t);

// tile of the Gram kernel for k columns: 64 x 64 (32-row stages) from k = 192, else
// 32 x 32 (64-row stages)
static int gram_tile(int k) { return k >= 192 ? 64 : 32; }

static void gram_shape(int64_t n, int k, int cu_count, int& nb, int& kp, int& nchunk,
                       int64_t& rows) {
    const int gt = gram_tile(k), gr = gt == 64 ? 32 : 64;
    nb = (k + gt - 1) / gt;
    kp = nb * gt;
    const int pairs = nb * (nb + 1) / 2;
    // enough work-groups to cover the chip's resident slots several times over (the
    // products of a tile pair over a row chunk are short), chunks of at least 256 rows
    int64_t want = std::max<int64_t>(1, (8LL * cu_count + pairs - 1) / pairs);
    int64_t maxc = std::max<int64_t>(1, (n + 255) / 256);
    nchunk = (int)std::min<int64_t>(want, maxc);
    rows = (n + nchunk - 1) / nchunk;
    rows = ((rows + gr - 1) / gr) * gr;
    nchunk = (int)std::max<int64_t>(1, (n + rows - 1) / rows);
}

size_t gram_ws_doubles(int64_t n, int k, int cu_count) {
    int nb, kp, nchunk;
    int64_t rows;
    gram_shape(n, k, cu_count, nb, kp, nchunk, rows);
    return (size_t)nchunk * 2 * kp * kp;
}

void launch_gram(int64_t n, int k, const double* Z, const double* ZH, const double* ZS, int64_t ldz,
                 double* HR, double* SR, int64_t ldr, double* ws, int cu_count, hipStream_t s) {
    if (k <= 0) return;
    int nb, kp, nchunk;
    int64_t rows;
    gram_shape(n, k, cu_count, nb, kp, nchunk, rows);
    const int pairs = nb * (nb + 1) / 2;
    if (gram_tile(k) == 64)
        hipLaunchKernelGGL((k_gram<64, 32>), dim3(pairs, nchunk), dim3(256), 0, s, n, k, Z, ZH, ZS, ldz, nb, rows,
                           ws, kp);
    else
        hipLaunchKernelGGL((k_gram<32, 64>), dim3(pairs, nchunk), dim3(256), 0, s, n, k, Z, ZH, ZS, ldz, nb, rows,
                           ws, kp);
    LABPSD_HIP(hipGetLastError());
    const int64_t tot = (int64_t)k * k;
    hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((8 * tot + 255) / 256)), dim3(256), 0, s, k, kp,
                       nchunk, ws, HR, SR, ldr);
    LABPSD_HIP(hipGetLastError());
}

// MFMA tiles per wavefront of the wide block update: the width 16 CT that pads b the
// least, then the fewest column groups (each group re-reads Z)
int block_update_ct(int b) {
    int best_ct = 8;
    int64_t best_cost = INT64_MAX;
    for (int ct : {9, 8, 6}) {
        const int64_t g = (b + 16 * ct - 1) / (16 * ct);
        const int64_t cost = (g * 16 * ct - b) * 4 + g;
        if (cost < best_cost) {
            best_cost = cost;
            best_ct = ct;
        }
    }
    return best_ct;
}

void launch_block_update(int64_t n, int k, int b, const double* Z, const double* ZH,
                         const double* ZS, int64_t ldz, const double* W, int64_t ldw, double* Psi,
                         double* PsiH, double* PsiS, int64_t ldo, hipStream_t s) {
    if (n <= 0 || b <= 0) return;
    dim3 grid((unsigned)((n + 63) / 64), (unsigned)((b + 31) / 32), 3);
    if (k >= 128 || b >= 96) {
        // wide blocks: 128 columns per work-group
        const int ct = block_update_ct(b);
        const dim3 gw((unsigned)((n + 63) / 64), (unsigned)((b + 16 * ct - 1) / (16 * ct)), 3);
        if (ct == 9)
            hipLaunchKernelGGL(k_block_update_wide<9>, gw, dim3(256), 0, s, n, k, b, Z, ZH, ZS, ldz, W, ldw, Psi,
                               PsiH, PsiS, ldo);
        else if (ct == 6)
            hipLaunchKernelGGL(k_block_update_wide<6>, gw, dim3(256), 0, s, n, k, b, Z, ZH, ZS, ldz, W, ldw, Psi,
                               PsiH, PsiS, ldo);
        else
            hipLaunchKernelGGL(k_block_update_wide<8>, gw, dim3(256), 0, s, n, k, b, Z, ZH, ZS, ldz, W, ldw, Psi,
                               PsiH, PsiS, ldo);
        LABPSD_HIP(hipGetLastError());
        return;
    }
    hipLaunchKernelGGL(k_block_update, grid, dim3(256), 0, s, n, k, b, Z, ZH, ZS, ldz, W, ldw, Psi,
                       PsiH, PsiS, ldo);
    LABPSD_HIP(hipGetLastError());
}

void launch_orth_deviation(int b, const double* SR, int64_t ld, double* out, hipStream_t s) {
    if (b <= 0) return;
    hipLaunchKernelGGL(k_orth_deviation, dim3(1), dim3(256), 0, s, b, SR, ld, out);
    LABPSD_HIP(hipGetLastError());
}

}  // namespace labpsd
