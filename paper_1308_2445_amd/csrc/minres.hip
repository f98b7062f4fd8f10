// Locally accelerated refinement (outline step 6(b), Section 4): for every localised
// pair j, MINRES on (H - eps_j S) dp = -dr_j with dr_j = (H - eps_j S) p_j + r_j, from
// dp = 0, until the recurred residual norm ||dr_j + (H - eps_j S) dp|| is at most
// eta ||r_j|| (eq. (approxp)) or the iteration cap; then p_j += dp.
//
// MINRES (Paige and Saunders): Lanczos on A = H - eps_j S builds an orthonormal Krylov
// basis with A V_k = V_{k+1} T_k; the least-squares problem with T_k is solved by one
// Givens rotation per step, whose running product gives the residual norm for free.
// All localised columns advance together, three kernels per iteration:
//   spmv    u = A v - beta_k v_prev, per-slice FP64 partial sums of v.u, u.u and v.v
//           (one pattern pass)
//   colsums the three sums of every live column from its slices' partials (with at most
//           kMinresOwnSums slices the update kernels sum them themselves instead)
//   update  alpha_k = v.u; w = u - alpha_k v, whose norm follows from the sums without
//           another pass: ||w||^2 = u.u - 2 alpha_k v.u + alpha_k^2 v.v; beta_{k+1} = ||w||,
//           the new rotation, tau_k and |phibar_k|;
//           d = (v - delta_k d1 - eps_k d2) / gamma_k, x += tau_k d, v_next = w / beta_{k+1}
// Every block recomputes the column's scalars from the column sums (identical values);
// block 0 of the column stores the new scalar state into the other half of a double
// buffer, so no block reads a state that another block of the same kernel writes.
// The one-step variant (the conclusions' first-order method) shares the SpMV and the
// host loop; see k_onestep_update.
// The host checks the columns' done flags every few iterations (the update kernel writes
// them straight into pinned host memory on those iterations).  T = double (FP64)
// or float (mixed: FP32 vectors and products; the per-slice sums are FP64 in both).
#include "common.h"

namespace labpsd {

namespace {

// slices up to which the update kernels sum the MINRES partials themselves
constexpr int64_t kMinresOwnSums = 1024;

struct MinresScal {
    double beta;        // beta_k: coupling of v_k to v_{k-1}
    double cprev, sprev, cpp, spp;   // rotations k-1 and k-2
    double phibar;      // rotated right-hand side, |phibar| = residual norm
    double stop;        // eta * ||r_j||
    int its, done, pad0, pad1;
};

template <typename T>
__device__ __forceinline__ T wave_sum_t(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// One slice per work-group (the sliced-ELL walk of the products: pattern staged in LDS,
// wavefronts on different columns); a wavefront covers all 64 rows of the slice for its
// CW columns, so each column's per-slice sums are one wavefront reduction, stored as the
// slice's partial: partial[(w q + j) npart + slice], npart = nslices, the slices of one
// sum and column contiguous for k_minres_colsums.  Columns that have all converged skip the products
// (every barrier stays uniform: only the segment staging has barriers).
template <typename T, int MODE, int CW>
__global__ __launch_bounds__(64 * kSellWaves) void k_minres_spmv(
    const int64_t* __restrict__ off, const int32_t* __restrict__ col, const T* __restrict__ hv,
    const T* __restrict__ sv, int64_t n, int64_t nslices, const T* __restrict__ X, int64_t ldx,
    const int32_t* __restrict__ xcols, const T* __restrict__ aux, int64_t ldaux,
    const int32_t* __restrict__ auxcols, const double* __restrict__ shift,
    const MinresScal* __restrict__ sc, T* __restrict__ out, double* __restrict__ partial,
    int64_t npart, int q, int cpb, int lseg, NlEpi<T, T> nl) {
    constexpr int NS = MODE == 0 ? 1 : 3;   // partial sums per column
    extern __shared__ double sell_dyn[];
    const SliceLds<T> L = slice_lds<T>(sell_dyn, lseg);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t slice = xcd_block(blockIdx.x, nslices);
    const int64_t e0 = off[slice];
    const int nsl = (int)((off[slice + 1] - e0) / kSlice);
    const int nseg = (nsl + lseg - 1) / lseg;
    const int64_t row = slice * kSlice + lane;
    const int jb = (int)blockIdx.y * cpb, je = min(q, jb + cpb);
    if (nseg == 1) {
        sell_stage<T>(col, hv, sv, e0, 0, nsl, L);
        __syncthreads();
    }
    for (int r = jb; r < je; r += kSellWaves * CW) {
        const int j0 = r + wave * CW;
        bool act[CW];
        const T* xc[CW];
        T ah[CW], as[CW];
        bool any = false;
#pragma unroll
        for (int j = 0; j < CW; ++j) {
            const int jj = j0 + j;
            act[j] = jj < je && (MODE == 0 || !sc[jj].done);
            any = any || act[j];
            xc[j] = act[j] ? X + (int64_t)(MODE == 0 ? xcols[jj] : jj) * ldx : X;
            ah[j] = T(0);
            as[j] = T(0);
        }
        const T* xp[CW];
#pragma unroll
        for (int j = 0; j < CW; ++j) xp[j] = xc[j];
        for (int sg = 0; sg < nseg; ++sg) {
            const int s0 = sg * lseg, ns = min(lseg, nsl - s0);
            if (nseg > 1) {
                __syncthreads();
                sell_stage<T>(col, hv, sv, e0, s0, ns, L);
                __syncthreads();
            }
            if (any) sell_lds_accumulate<T, CW>(L, ns, xp, ah, as);
        }
        if (!any) continue;   // wavefront-uniform; no barrier follows in this round
#pragma unroll
        for (int j = 0; j < CW; ++j) {
            const int jj = j0 + j;
            if (jj >= je) break;
            double c[NS];
#pragma unroll
            for (int w = 0; w < NS; ++w) c[w] = 0.0;
            if (act[j] && row < n) {
                // the nonlocal term belongs to H: (H_loc + F G F^T - shift S) x
                const T hx = nl.rp ? ah[j] + nl_row_term(nl, row, jj) : ah[j];
                const T y = hx - (T)shift[jj] * as[j];
                T v;
                if constexpr (MODE == 0) {
                    v = -(y + aux[row + (int64_t)auxcols[jj] * ldaux]);
                    c[0] = (double)v * (double)v;
                } else {
                    v = y - (T)sc[jj].beta * aux[row + (int64_t)jj * ldaux];
                    const double xv = (double)xc[j][row];
                    c[0] = xv * (double)v;
                    c[1] = (double)v * (double)v;
                    c[2] = xv * xv;
                }
                out[row + (int64_t)jj * n] = v;
            }
#pragma unroll
            for (int w = 0; w < NS; ++w) {
                const double t = wave_allsum(c[w]);
                if (lane == 0) partial[((int64_t)w * q + jj) * npart + slice] = act[j] ? t : 0.0;
            }
        }
    }
}

// sums[t] = the sum over the npart slices of partial set t = w q + j (w < nsets), one
// wavefront per set and column in a fixed order (so the values are reproducible); columns
// already done (sc != nullptr) are skipped, their sums are not read
__global__ __launch_bounds__(256) void k_minres_colsums(const double* __restrict__ partial, int64_t npart, int q,
                                                        int nsets, const MinresScal* __restrict__ sc,
                                                        double* __restrict__ sums) {
    const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= nsets * q) return;
    if (sc && sc[t % q].done) return;
    const double* p = partial + (int64_t)t * npart;
    double v = 0.0;
    for (int64_t i = threadIdx.x & 63; i < npart; i += 64) v += p[i];
    v = wave_sum_t(v);
    if ((threadIdx.x & 63) == 0) sums[t] = v;
}

// The three sums (v.u, u.u, v.v or their one-step analogues) of column j straight from
// its slices' partials, for a whole work-group: wavefronts 0, 1 and 2 each sum one set
// (contiguous, fixed order) and LDS hands them to all.  Used instead of k_minres_colsums
// when there are few slices (the launch would cost more than the sums).
__device__ void block_column_sums3(const double* __restrict__ part, int64_t npart, int q, int j,
                                   double out[3]) {
    __shared__ double bc[3];
    const int w = threadIdx.x >> 6;
    if (w < 3) {
        const double* p = part + ((int64_t)w * q + j) * npart;
        double v = 0.0;
        for (int64_t i = threadIdx.x & 63; i < npart; i += 64) v += p[i];
        v = wave_sum_t(v);
        if ((threadIdx.x & 63) == 0) bc[w] = v;
    }
    __syncthreads();
    out[0] = bc[0];
    out[1] = bc[1];
    out[2] = bc[2];
}

// sum over the work-group, valid in thread 0
template <typename T>
__device__ T block_sum(T v) {
    __shared__ T w[4];
    v = wave_sum_t(v);
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = v;
    __syncthreads();
    return w[0] + w[1] + w[2] + w[3];
}

__global__ __launch_bounds__(256) void k_minres_init_finish(const double* __restrict__ sums, int q,
                                                            const double* __restrict__ rnorm,
                                                            double eta, int max_inner,
                                                            MinresScal* __restrict__ sc) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= q) return;
    const double b2 = sums[j];
    const double beta1 = sqrt(b2);
    MinresScal s{};
    s.beta = beta1;
    s.cprev = 1.0; s.sprev = 0.0; s.cpp = 1.0; s.spp = 0.0;
    s.phibar = beta1;
    s.stop = eta * rnorm[j];
    s.done = (beta1 == 0.0 || beta1 <= s.stop || max_inner <= 0) ? 1 : 0;
    s.its = 0;
    sc[j] = s;
}

// v = b / beta1, zero the other vectors
template <typename T>
__global__ __launch_bounds__(256) void k_minres_init_vectors(int64_t n, int q,
                                                             const MinresScal* __restrict__ sc,
                                                             T* __restrict__ V, T* __restrict__ VP,
                                                             T* __restrict__ D1, T* __restrict__ D2,
                                                             T* __restrict__ Xs) {
    const int j = blockIdx.y;
    const bool live = !sc[j].done;
    const T inv = live ? (T)(1.0 / sc[j].beta) : T(0);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int64_t o = i + (int64_t)j * n;
        V[o] = live ? V[o] * inv : T(0);
        VP[o] = T(0);
        D1[o] = T(0);
        D2[o] = T(0);
        Xs[o] = T(0);
    }
}

// Scalar recurrences of the tridiagonal QR, computed identically by every work-group of
// the column, then the vector updates of its rows.  Work-group 0 of the column stores
// the new state in sc_out (the host swaps sc_in and sc_out between iterations).
template <typename T>
__global__ __launch_bounds__(256) void k_minres_update(int64_t n, int q, int max_inner,
                                                       const MinresScal* __restrict__ sc_in,
                                                       MinresScal* __restrict__ sc_out,
                                                       const double* __restrict__ part, int64_t npa,
                                                       const double* __restrict__ csum,
                                                       const T* __restrict__ V, T* __restrict__ Wb,
                                                       const T* __restrict__ D1, T* __restrict__ D2,
                                                       T* __restrict__ Xs, int32_t* __restrict__ done_out) {
    const int j = blockIdx.y;
    const MinresScal s = sc_in[j];
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (s.done) {
        if (lead) {
            sc_out[j] = s;
            if (done_out) done_out[j] = 1;
        }
        return;
    }
    // v.u, u.u, v.v: from the column-sum kernel, or summed here when there are few slices
    double sums[3];
    if (csum) {
        sums[0] = csum[j];
        sums[1] = csum[q + j];
        sums[2] = csum[2 * q + j];
    } else {
        block_column_sums3(part, npa, q, j, sums);
    }
    const double al = sums[0];
    const double bnext = sqrt(fmax(sums[1] - al * (2.0 * sums[0] - al * sums[2]), 0.0));
    const int k = s.its + 1;
    // rotation k-2 maps (0, beta_k) to (eps_k, t1); column 1 has no entry above the diagonal
    const double epsk = k > 1 ? s.spp * s.beta : 0.0;
    const double t1 = k > 1 ? s.cpp * s.beta : 0.0;
    // rotation k-1 maps (t1, alpha_k) to (delta_k, gammabar_k)
    const double delta = s.cprev * t1 + s.sprev * al;
    const double gbar = -s.sprev * t1 + s.cprev * al;
    const double gamma = sqrt(gbar * gbar + bnext * bnext);
    if (gamma == 0.0) {
        if (lead) {
            MinresScal t = s;
            t.done = 1;
            sc_out[j] = t;
        }
        return;
    }
    // rotation k maps (gammabar_k, beta_{k+1}) to (gamma_k, 0)
    const double c = gbar / gamma, sn = bnext / gamma;
    const double tau = c * s.phibar;
    const double phibar = -sn * s.phibar;
    const T ig = (T)(1.0 / gamma), de = (T)delta, ep = (T)epsk, ta = (T)tau;
    const T ib = bnext > 0.0 ? (T)(1.0 / bnext) : T(0);
    const T tal = (T)al;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int64_t o = i + (int64_t)j * n;
        const T v = V[o];
        const T d = (v - de * D1[o] - ep * D2[o]) * ig;
        D2[o] = d;
        Xs[o] += ta * d;
        Wb[o] = (Wb[o] - tal * v) * ib;
    }
    if (lead) {
        MinresScal t = s;
        t.its = k;
        t.phibar = phibar;
        t.cpp = s.cprev;
        t.spp = s.sprev;
        t.cprev = c;
        t.sprev = sn;
        t.beta = bnext;
        t.done = (fabs(phibar) <= s.stop || bnext == 0.0 || k >= max_inner) ? 1 : 0;
        sc_out[j] = t;
        if (done_out) done_out[j] = t.done;
    }
}

// ---- the conclusions' first-order one-step refinement: g = -rho, rho = (H - eps S) p + r;
// each step u = A g (the SpMV above with beta = 0 gives u and the sums g.u, u.u, g.g),
// alpha = g.u / u.u minimises ||g - alpha u||, p += alpha g (accumulated in Xs),
// g -= alpha u, ||g||^2 = g.g - (g.u)^2 / u.u.  The scalar state reuses MinresScal:
// beta = 0 always, phibar = ||g||.

__global__ __launch_bounds__(256) void k_onestep_init_finish(const double* __restrict__ sums, int q,
                                                             const double* __restrict__ rnorm,
                                                             double eta, int max_inner,
                                                             MinresScal* __restrict__ sc) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= q) return;
    const double g2 = sums[j];
    MinresScal s{};
    s.beta = 0.0;
    s.cprev = 1.0; s.sprev = 0.0; s.cpp = 1.0; s.spp = 0.0;
    s.phibar = sqrt(g2);
    s.stop = eta * rnorm[j];
    s.done = (s.phibar == 0.0 || s.phibar <= s.stop || max_inner <= 0) ? 1 : 0;
    s.its = 0;
    sc[j] = s;
}

template <typename T>
__global__ __launch_bounds__(256) void k_zero_cols(int64_t n, T* __restrict__ Xs) {
    const int j = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        Xs[i + (int64_t)j * n] = T(0);
}

template <typename T>
__global__ __launch_bounds__(256) void k_onestep_update(int64_t n, int q, int max_inner,
                                                        const MinresScal* __restrict__ sc_in,
                                                        MinresScal* __restrict__ sc_out,
                                                        const double* __restrict__ part, int64_t npa,
                                                        const double* __restrict__ csum,
                                                        T* __restrict__ G, const T* __restrict__ U,
                                                        T* __restrict__ Xs, int32_t* __restrict__ done_out) {
    const int j = blockIdx.y;
    const MinresScal s = sc_in[j];
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (s.done) {
        if (lead) {
            sc_out[j] = s;
            if (done_out) done_out[j] = 1;
        }
        return;
    }
    // g.u, u.u, g.g (as in k_minres_update)
    double sums[3];
    if (csum) {
        sums[0] = csum[j];
        sums[1] = csum[q + j];
        sums[2] = csum[2 * q + j];
    } else {
        block_column_sums3(part, npa, q, j, sums);
    }
    if (!(sums[1] > 0.0)) {   // A g = 0: no step reduces the residual
        if (lead) {
            MinresScal t = s;
            t.done = 1;
            sc_out[j] = t;
            if (done_out) done_out[j] = 1;
        }
        return;
    }
    const double alpha = sums[0] / sums[1];
    const double g2 = fmax(sums[2] - sums[0] * alpha, 0.0);
    const T a = (T)alpha;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int64_t o = i + (int64_t)j * n;
        const T g = G[o];
        Xs[o] += a * g;
        G[o] = g - a * U[o];
    }
    if (lead) {
        MinresScal t = s;
        t.its = s.its + 1;
        t.phibar = sqrt(g2);
        t.done = (t.phibar <= s.stop || t.its >= max_inner) ? 1 : 0;
        sc_out[j] = t;
        if (done_out) done_out[j] = t.done;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_minres_final(int64_t n, int q, const int32_t* __restrict__ cols,
                                                      const MinresScal* __restrict__ sc,
                                                      const T* __restrict__ Xs, T* __restrict__ P,
                                                      int64_t ldp, int32_t* __restrict__ its,
                                                      unsigned long long* __restrict__ its_total) {
    const int j = blockIdx.y;
    T* p = P + (int64_t)cols[j] * ldp;
    const T* x = Xs + (int64_t)j * n;
    if (sc[j].its > 0)
        for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
            p[i] += x[i];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (its) its[j] = sc[j].its;
        if (its_total) atomicAdd(its_total, (unsigned long long)sc[j].its);
    }
}

template <typename T, int MODE, int CW>
int64_t launch_spmv_s(const Sell& A, SellShape sh, const T* hv, const T* sv, const T* X, int64_t ldx,
                      const int32_t* xcols, const T* aux, int64_t ldaux, const int32_t* auxcols,
                      const double* shift, const MinresScal* sc, T* out, double* partial, int q,
                      hipStream_t s, NlEpi<T, T> nl) {
    allow_dynamic_lds((const void*)k_minres_spmv<T, MODE, CW>);
    const int cpb = (q + sh.bands - 1) / sh.bands;
    const dim3 g((unsigned)A.nslices, (unsigned)sh.bands);
    hipLaunchKernelGGL((k_minres_spmv<T, MODE, CW>), g, dim3(64 * kSellWaves), sh.lds_bytes, s, A.slice_off.p,
                       A.col.p, hv, sv, A.n, A.nslices, X, ldx, xcols, aux, ldaux, auxcols, shift, sc, out,
                       partial, A.nslices, q, cpb, sh.lseg, nl);
    return A.nslices;
}

// (H - eps_j S) products of the MINRES columns in the launch shape sell_shape picks;
// returns the number of partials per column (one per slice)
template <typename T, int MODE>
int64_t launch_spmv(const Sell& A, SellShape sh, const T* hv, const T* sv, const T* X, int64_t ldx,
                    const int32_t* xcols, const T* aux, int64_t ldaux, const int32_t* auxcols,
                    const double* shift, const MinresScal* sc, T* out, double* partial, int q,
                    hipStream_t s, const NonLocal* nlp) {
    // the nonlocal term: G F^T x of the product's columns first, then the epilogue
    const NlEpi<T, T> nl = nlp ? nl_prepare<T>(*nlp, X, ldx, xcols, q, s) : NlEpi<T, T>{};
    if (sh.cw >= 4)
        return launch_spmv_s<T, MODE, 4>(A, sh, hv, sv, X, ldx, xcols, aux, ldaux, auxcols, shift, sc, out, partial,
                                         q, s, nl);
    if (sh.cw == 2)
        return launch_spmv_s<T, MODE, 2>(A, sh, hv, sv, X, ldx, xcols, aux, ldaux, auxcols, shift, sc, out, partial,
                                         q, s, nl);
    return launch_spmv_s<T, MODE, 1>(A, sh, hv, sv, X, ldx, xcols, aux, ldaux, auxcols, shift, sc, out, partial, q,
                                     s, nl);
}

}  // namespace

size_t minres_ws_elems(int64_t n, int q) {
    // six vectors, then 3 FP64 partial sums per slice and column and the 3 q column sums
    // (as T elements: 6 (nslices + 1) q of them hold 3 (nslices + 1) q doubles even for float)
    return (size_t)6 * n * q + 3 * (8 / sizeof(float)) * (size_t)((n + 63) / 64 + 1) * q;
}

size_t minres_scal_doubles(int q) {
    static_assert(sizeof(MinresScal) % 8 == 0, "scalar state must be a whole number of doubles");
    return 2 * (sizeof(MinresScal) / 8) * (size_t)q + (size_t)q + 2;
}

// Work-groups per column of the row-wise kernels: enough to cover the rows at one
// element per thread up to 128, beyond that each thread takes several rows (this also
// bounds the partials every work-group of the next kernel re-sums).
static unsigned rowwise_groups(int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, 128); }

template <typename T>
void run_minres(const Sell& A, T* P, int64_t ldp, const T* R, int64_t ldr, int q,
                const int32_t* cols_dev, const double* shift_dev, const double* rnorm_dev,
                double eta, int max_inner, int32_t* its_dev, T* ws, double* scal_ws,
                int32_t* flag_host_pinned, hipStream_t s, int64_t* launches, hipEvent_t ev0,
                hipEvent_t ev1, unsigned long long* its_total, int method, const NonLocal* nlt) {
    if (q <= 0 || A.n == 0) return;
    if (nlt && nlt->k == 0) nlt = nullptr;
    const bool onestep = method == LABPSD_REFINE_ONESTEP;
    const int64_t n = A.n;
    T* V = ws;
    T* VP = V + n * q;
    T* Wb = VP + n * q;
    T* D1 = Wb + n * q;
    T* D2 = D1 + n * q;
    T* Xs = D2 + n * q;
    const SellShape sh = sell_shape(A, q, sizeof(T));
    const unsigned G = rowwise_groups(n);
    // spmv partials: 3 sets of at most nslices per column, FP64 (6 n q T elements precede,
    // an even count, so the address is 8-byte aligned)
    double* pa = (double*)(Xs + n * q);
    // scalar state double buffer (the rest of the scalar workspace is spare)
    constexpr size_t kScalDoubles = sizeof(MinresScal) / 8;
    MinresScal* sa = (MinresScal*)scal_ws;
    MinresScal* sb = (MinresScal*)(scal_ws + kScalDoubles * q);
    // the done flags of a check iteration are written by the device into pinned host
    // memory: two slots of q flags (flag_host_pinned holds 2 q ints)
    int32_t* flag_dev = nullptr;
    LABPSD_HIP(hipHostGetDevicePointer((void**)&flag_dev, flag_host_pinned, 0));
    auto all_done = [&](int sl) {
        const volatile int32_t* f = flag_host_pinned + (size_t)sl * q;
        for (int j = 0; j < q; ++j)
            if (f[j] == 0) return false;
        return true;
    };
    const T* hv;
    const T* sv;
    if constexpr (sizeof(T) == 8) { hv = A.hv.p; sv = A.sv.p; }
    else { hv = A.hv32.p; sv = A.sv32.p; }
    const unsigned bx = (unsigned)std::min<int64_t>((n + 255) / 256, 512);
    const dim3 gel(bx, q);
    const dim3 grow(G, q);
    int64_t nl = 0;
    // b = -((H - eps S) p + r); beta1 = ||b||
    // spmv partials: one per slice and column
    const int64_t npa = launch_spmv<T, 0>(A, sh, hv, sv, P, ldp, cols_dev, R, ldr, cols_dev, shift_dev, sa, V,
                                          pa, q, s, nlt);
    // the column sums of the partials (3 q doubles after the 3 nslices q partials); with few
    // slices the update kernels sum the partials themselves (one launch fewer per iteration)
    double* csum = pa + 3 * A.nslices * (int64_t)q;
    const bool own_sums = A.nslices <= kMinresOwnSums;
    double* ucsum = own_sums ? nullptr : csum;
    const dim3 gsum1((unsigned)((q + 3) / 4)), gsum3((unsigned)((3 * q + 3) / 4)), gq((unsigned)((q + 255) / 256));
    hipLaunchKernelGGL(k_minres_colsums, gsum1, dim3(256), 0, s, (const double*)pa, npa, q, 1,
                       (const MinresScal*)nullptr, csum);
    if (onestep) {
        hipLaunchKernelGGL(k_onestep_init_finish, gq, dim3(256), 0, s, (const double*)csum, q, rnorm_dev,
                           eta, max_inner, sa);
        hipLaunchKernelGGL((k_zero_cols<T>), gel, dim3(256), 0, s, n, Xs);
    } else {
        hipLaunchKernelGGL(k_minres_init_finish, gq, dim3(256), 0, s, (const double*)csum, q, rnorm_dev,
                           eta, max_inner, sa);
        hipLaunchKernelGGL((k_minres_init_vectors<T>), gel, dim3(256), 0, s, n, q, (const MinresScal*)sa, V,
                           VP, D1, D2, Xs);
    }
    LABPSD_HIP(hipGetLastError());
    nl += 4;
    MinresScal* cur = sa;
    MinresScal* nxt = sb;
    // The host reads the active count every kCheckEvery iterations; iterations issued
    // after the last column finished find every column done and exit at once.  With two
    // events (and two flag slots) the read is pipelined: after issuing a check the host
    // waits for the previous one, so the iterations in between keep the device busy.
    const bool piped = ev0 != nullptr && ev1 != nullptr;
    const int kCheckEvery = piped ? 2 : 3;
    hipEvent_t evs[2] = {ev0, ev1};
    int slot = 0;
    bool pending = false;
    for (int it = 0; it < max_inner; ++it) {
        // on a check iteration the done flags go to host slot `slot`
        const bool check = it + 1 < max_inner && (it + 1) % kCheckEvery == 0;
        if (onestep) {
            // u = A g (beta is 0 in the one-step state), then the step
            launch_spmv<T, 1>(A, sh, hv, sv, V, n, nullptr, V, n, nullptr, shift_dev, cur, Wb, pa, q, s, nlt);
            if (!own_sums)
                hipLaunchKernelGGL(k_minres_colsums, gsum3, dim3(256), 0, s, (const double*)pa, npa, q, 3,
                                   (const MinresScal*)cur, csum);
            hipLaunchKernelGGL((k_onestep_update<T>), grow, dim3(256), 0, s, n, q, max_inner,
                               (const MinresScal*)cur, nxt, (const double*)pa, npa, (const double*)ucsum, V,
                               (const T*)Wb, Xs,
                               check ? flag_dev + (size_t)slot * q : nullptr);
            LABPSD_HIP(hipGetLastError());
            nl += own_sums ? 2 : 3;
            MinresScal* t2 = cur; cur = nxt; nxt = t2;
        } else {
        launch_spmv<T, 1>(A, sh, hv, sv, V, n, nullptr, VP, n, nullptr, shift_dev, cur, Wb, pa, q, s, nlt);
        if (!own_sums)
            hipLaunchKernelGGL(k_minres_colsums, gsum3, dim3(256), 0, s, (const double*)pa, npa, q, 3,
                               (const MinresScal*)cur, csum);
        hipLaunchKernelGGL((k_minres_update<T>), grow, dim3(256), 0, s, n, q, max_inner,
                           (const MinresScal*)cur, nxt, (const double*)pa, npa, (const double*)ucsum,
                           (const T*)V, Wb,
                           (const T*)D1, D2, Xs, check ? flag_dev + (size_t)slot * q : nullptr);
        LABPSD_HIP(hipGetLastError());
        nl += own_sums ? 2 : 3;
        // rotate: v_prev <- v, v <- w (now scaled), w <- old v_prev; d1 <- new d, d2 <- old d1
        T* t0 = VP; VP = V; V = Wb; Wb = t0;
        T* t1 = D1; D1 = D2; D2 = t1;
        MinresScal* t2 = cur; cur = nxt; nxt = t2;
        }
        if (it + 1 == max_inner) break;
        if (check) {
            if (!piped) {
                LABPSD_HIP(hipStreamSynchronize(s));
                if (all_done(slot)) break;
                continue;
            }
            LABPSD_HIP(hipEventRecord(evs[slot], s));
            if (pending) {
                spin_event(evs[slot ^ 1]);
                if (all_done(slot ^ 1)) break;
            }
            pending = true;
            slot ^= 1;
        }
    }
    hipLaunchKernelGGL((k_minres_final<T>), gel, dim3(256), 0, s, n, q, cols_dev, (const MinresScal*)cur,
                       Xs, P, ldp, its_dev, its_total);
    LABPSD_HIP(hipGetLastError());
    nl += 1;
    if (launches) *launches += nl;
}

template void run_minres<double>(const Sell&, double*, int64_t, const double*, int64_t, int,
                                 const int32_t*, const double*, const double*, double, int, int32_t*,
                                 double*, double*, int32_t*, hipStream_t, int64_t*, hipEvent_t, hipEvent_t,
                                 unsigned long long*, int, const NonLocal*);
template void run_minres<float>(const Sell&, float*, int64_t, const float*, int64_t, int,
                                const int32_t*, const double*, const double*, double, int, int32_t*,
                                float*, double*, int32_t*, hipStream_t, int64_t*, hipEvent_t, hipEvent_t,
                                unsigned long long*, int, const NonLocal*);

}  // namespace labpsd
