// Locally accelerated refinement (outline step 6(b), Section 4): for every localised
// pair j, MINRES on (H - eps_j S) dp = -dr_j with dr_j = (H - eps_j S) p_j + r_j, from
// dp = 0, until the recurred residual norm ||dr_j + (H - eps_j S) dp|| is at most
// eta ||r_j|| (eq. (approxp)) or the iteration cap; then p_j += dp.
//
// All localised columns advance together, one MINRES iteration per sweep of kernels:
//   spmv    w = (H - eps_j S) v - beta_j v_prev, partial v.w   (one pass over the pattern)
//   alpha   alpha_j = v.w
//   axpy    w -= alpha_j v, partial ||w||^2
//   scalar  beta_{k+1}, the Givens rotation of the tridiagonal QR, step tau, |phibar|
//   update  d = (v - delta d1 - eps d2) / gamma, x += tau d, v_next = w / beta_{k+1}
// A converged column stops changing; the host rotates the vector buffers between
// sweeps and stops once every column is done.  T = double (FP64) or float (mixed:
// FP32 vectors, FP32 products and FP32 per-slice sums).
#include "common.h"

namespace labpsd {

namespace {

struct MinresScal {
    double beta, cprev, sprev, cpp, spp, phibar, stop;
    double alpha, gamma, delta, eps, tau, betanext;
    int apply, done, its, pad;
};

template <typename T>
__device__ __forceinline__ T wave_sum_t(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

constexpr int kWaves = 4;
constexpr int kCW = 4;

template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_minres_spmv(
    const int64_t* __restrict__ off, const int32_t* __restrict__ col, const T* __restrict__ hv,
    const T* __restrict__ sv, int64_t n, int64_t nslices, const T* __restrict__ X, int64_t ldx,
    const int32_t* __restrict__ xcols, const T* __restrict__ aux, int64_t ldaux,
    const int32_t* __restrict__ auxcols, const double* __restrict__ shift,
    const MinresScal* __restrict__ sc, T* __restrict__ out, T* __restrict__ partial, int q) {
    const int lane = threadIdx.x & 63;
    const int64_t slice = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (slice >= nslices) return;
    const int j0 = blockIdx.y * kCW;
    const int64_t row = slice * kSlice + lane;
    const int64_t e0 = off[slice], e1 = off[slice + 1];
    bool act[kCW];
    const T* xc[kCW];
    T ah[kCW], as[kCW];
#pragma unroll
    for (int j = 0; j < kCW; ++j) {
        const int jj = j0 + j;
        act[j] = jj < q && (MODE == 0 || !sc[jj].done);
        xc[j] = act[j] ? X + (int64_t)(MODE == 0 ? xcols[jj] : jj) * ldx : X;
        ah[j] = T(0);
        as[j] = T(0);
    }
    for (int64_t e = e0 + lane; e < e1; e += kSlice) {
        const int64_t c = col[e];
        const T h = hv[e], s = sv[e];
#pragma unroll
        for (int j = 0; j < kCW; ++j) {
            if (act[j]) {
                const T x = xc[j][c];
                ah[j] = fma(h, x, ah[j]);
                as[j] = fma(s, x, as[j]);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kCW; ++j) {
        const int jj = j0 + j;
        T contrib = T(0);
        if (act[j] && row < n) {
            const T y = ah[j] - (T)shift[jj] * as[j];
            T v;
            if (MODE == 0) {
                v = -(y + aux[row + (int64_t)auxcols[jj] * ldaux]);
                contrib = v * v;
            } else {
                v = y - (T)sc[jj].beta * aux[row + (int64_t)jj * ldaux];
                contrib = xc[j][row] * v;
            }
            out[row + (int64_t)jj * n] = v;
        }
        if (jj < q) {
            contrib = wave_sum_t(contrib);
            if (lane == 0) partial[slice * q + jj] = act[j] ? contrib : T(0);
        }
    }
}

// sum of the per-slice partials of column j (one wavefront per column)
template <typename T>
__device__ double column_sum(const T* partial, int64_t nslices, int q, int j) {
    double s = 0.0;
    for (int64_t i = threadIdx.x & 63; i < nslices; i += 64) s += (double)partial[i * q + j];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    return __shfl(s, 0, 64);
}

template <typename T>
__global__ __launch_bounds__(256) void k_minres_init_finish(const T* __restrict__ partial,
                                                            int64_t nslices, int q,
                                                            const double* __restrict__ rnorm,
                                                            double eta, int max_inner,
                                                            MinresScal* __restrict__ sc) {
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= q) return;
    const double b2 = column_sum(partial, nslices, q, j);
    if ((threadIdx.x & 63) != 0) return;
    const double beta1 = sqrt(b2);
    MinresScal s{};
    s.beta = beta1;
    s.cprev = 1.0; s.sprev = 0.0; s.cpp = 1.0; s.spp = 0.0;
    s.phibar = beta1;
    s.stop = eta * rnorm[j];
    s.done = (beta1 == 0.0 || beta1 <= s.stop || max_inner <= 0) ? 1 : 0;
    s.apply = 0;
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

template <typename T>
__global__ __launch_bounds__(256) void k_minres_alpha(const T* __restrict__ partial, int64_t nslices,
                                                      int q, MinresScal* __restrict__ sc,
                                                      int32_t* __restrict__ active_count) {
    // the scalar kernel of this sweep counts the columns still active
    if (blockIdx.x == 0 && threadIdx.x == 0) *active_count = 0;
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= q) return;
    const double a = column_sum(partial, nslices, q, j);
    if ((threadIdx.x & 63) == 0 && !sc[j].done) sc[j].alpha = a;
}

// w -= alpha v; partial ||w||^2 per slice-sized chunk of rows
template <typename T>
__global__ __launch_bounds__(256) void k_minres_axpy(int64_t n, int q, int64_t nslices,
                                                     const MinresScal* __restrict__ sc,
                                                     const T* __restrict__ V, T* __restrict__ Wb,
                                                     T* __restrict__ partial) {
    const int j = blockIdx.y;
    const int64_t slice = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (slice >= nslices) return;
    const int lane = threadIdx.x & 63;
    const int64_t row = slice * kSlice + lane;
    T c = T(0);
    const bool live = !sc[j].done;
    if (live && row < n) {
        const int64_t o = row + (int64_t)j * n;
        const T w = Wb[o] - (T)sc[j].alpha * V[o];
        Wb[o] = w;
        c = w * w;
    }
    c = wave_sum_t(c);
    if (lane == 0) partial[slice * q + j] = c;
}

// scalar recurrences of the tridiagonal QR (one wavefront per column)
template <typename T>
__global__ __launch_bounds__(256) void k_minres_scalar(const T* __restrict__ partial,
                                                       int64_t nslices, int q, int max_inner,
                                                       MinresScal* __restrict__ sc,
                                                       int32_t* __restrict__ active_count) {
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= q) return;
    const double w2 = column_sum(partial, nslices, q, j);
    if ((threadIdx.x & 63) != 0) return;
    MinresScal s = sc[j];
    if (s.done) {
        s.apply = 0;
        sc[j] = s;
        return;
    }
    const double bnext = sqrt(w2);
    const int k = s.its + 1;
    // rotation k-2 maps (0, beta_k) to (eps_k, t1); column 1 has no entry above the diagonal
    const double epsk = k > 1 ? s.spp * s.beta : 0.0;
    const double t1 = k > 1 ? s.cpp * s.beta : 0.0;
    // rotation k-1 maps (t1, alpha_k) to (delta_k, gammabar_k)
    const double delta = s.cprev * t1 + s.sprev * s.alpha;
    const double gbar = -s.sprev * t1 + s.cprev * s.alpha;
    const double gamma = sqrt(gbar * gbar + bnext * bnext);
    if (gamma == 0.0) {
        s.apply = 0;
        s.done = 1;
        sc[j] = s;
        return;
    }
    const double c = gbar / gamma, sn = bnext / gamma;
    s.tau = c * s.phibar;
    s.phibar = -sn * s.phibar;
    s.gamma = gamma;
    s.delta = delta;
    s.eps = epsk;
    s.betanext = bnext;
    s.apply = 1;
    s.its = k;
    s.cpp = s.cprev; s.spp = s.sprev;
    s.cprev = c; s.sprev = sn;
    s.beta = bnext;
    if (fabs(s.phibar) <= s.stop || bnext == 0.0 || k >= max_inner) s.done = 1;
    sc[j] = s;
    if (!s.done) atomicAdd(active_count, 1);
}

// d2 <- (v - delta d1 - eps d2) / gamma ; x += tau d2 ; w <- w / beta_{k+1}
template <typename T>
__global__ __launch_bounds__(256) void k_minres_update(int64_t n, const MinresScal* __restrict__ sc,
                                                       const T* __restrict__ V,
                                                       T* __restrict__ Wb, const T* __restrict__ D1,
                                                       T* __restrict__ D2, T* __restrict__ Xs) {
    const int j = blockIdx.y;
    const MinresScal& s = sc[j];
    if (!s.apply) return;
    const T ig = (T)(1.0 / s.gamma), de = (T)s.delta, ep = (T)s.eps, ta = (T)s.tau;
    const T ib = s.betanext > 0.0 ? (T)(1.0 / s.betanext) : T(0);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int64_t o = i + (int64_t)j * n;
        const T d = (V[o] - de * D1[o] - ep * D2[o]) * ig;
        D2[o] = d;
        Xs[o] += ta * d;
        Wb[o] *= ib;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_minres_final(int64_t n, int q, const int32_t* __restrict__ cols,
                                                      const MinresScal* __restrict__ sc,
                                                      const T* __restrict__ Xs, T* __restrict__ P,
                                                      int64_t ldp, int32_t* __restrict__ its) {
    const int j = blockIdx.y;
    T* p = P + (int64_t)cols[j] * ldp;
    const T* x = Xs + (int64_t)j * n;
    if (sc[j].its > 0)
        for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
            p[i] += x[i];
    if (blockIdx.x == 0 && threadIdx.x == 0 && its) its[j] = sc[j].its;
}

}  // namespace

size_t minres_ws_elems(int64_t n, int q) { return (size_t)6 * n * q + (size_t)((n + 63) / 64 + 1) * q; }

template <typename T>
void run_minres(const Sell& A, T* P, int64_t ldp, const T* R, int64_t ldr, int q,
                const int32_t* cols_dev, const double* shift_dev, const double* rnorm_dev,
                double eta, int max_inner, int32_t* its_dev, T* ws, double* scal_ws,
                int32_t* flag_host_pinned, hipStream_t s, int64_t* launches) {
    if (q <= 0) return;
    const int64_t n = A.n;
    T* V = ws;
    T* VP = V + n * q;
    T* Wb = VP + n * q;
    T* D1 = Wb + n * q;
    T* D2 = D1 + n * q;
    T* Xs = D2 + n * q;
    T* partial = Xs + n * q;
    MinresScal* sc = (MinresScal*)scal_ws;
    int32_t* counter = (int32_t*)(sc + q);
    const T* hv;
    const T* sv;
    if constexpr (sizeof(T) == 8) { hv = A.hv.p; sv = A.sv.p; }
    else { hv = A.hv32.p; sv = A.sv32.p; }
    const dim3 gsp((unsigned)((A.nslices + kWaves - 1) / kWaves), (unsigned)((q + kCW - 1) / kCW));
    const dim3 gcol((unsigned)((q + 3) / 4));
    const unsigned bx = (unsigned)std::min<int64_t>((n + 255) / 256, 512);
    const dim3 gel(bx, q);
    const dim3 gsl((unsigned)((A.nslices + kWaves - 1) / kWaves), q);
    int64_t nl = 0;
    // b = -((H - eps S) p + r); beta1 = ||b||
    hipLaunchKernelGGL((k_minres_spmv<T, 0>), gsp, dim3(256), 0, s, A.slice_off.p, A.col.p, hv, sv, n,
                       A.nslices, P, ldp, cols_dev, R, ldr, cols_dev, shift_dev,
                       (const MinresScal*)sc, V, partial, q);
    hipLaunchKernelGGL((k_minres_init_finish<T>), gcol, dim3(256), 0, s, partial, A.nslices, q,
                       rnorm_dev, eta, max_inner, sc);
    hipLaunchKernelGGL((k_minres_init_vectors<T>), gel, dim3(256), 0, s, n, q, (const MinresScal*)sc, V,
                       VP, D1, D2, Xs);
    LABPSD_HIP(hipGetLastError());
    nl += 3;
    for (int it = 0; it < max_inner; ++it) {
        hipLaunchKernelGGL((k_minres_spmv<T, 1>), gsp, dim3(256), 0, s, A.slice_off.p, A.col.p, hv, sv,
                           n, A.nslices, V, n, nullptr, VP, n, nullptr, shift_dev,
                           (const MinresScal*)sc, Wb, partial, q);
        hipLaunchKernelGGL((k_minres_alpha<T>), gcol, dim3(256), 0, s, partial, A.nslices, q, sc,
                           counter);
        hipLaunchKernelGGL((k_minres_axpy<T>), gsl, dim3(256), 0, s, n, q, A.nslices,
                           (const MinresScal*)sc, V, Wb, partial);
        hipLaunchKernelGGL((k_minres_scalar<T>), gcol, dim3(256), 0, s, partial, A.nslices, q,
                           max_inner, sc, counter);
        hipLaunchKernelGGL((k_minres_update<T>), gel, dim3(256), 0, s, n, (const MinresScal*)sc, V, Wb,
                           D1, D2, Xs);
        LABPSD_HIP(hipGetLastError());
        nl += 5;
        // rotate: v_prev <- v, v <- w (now scaled), w <- old v_prev; d1 <- d2 (new d), d2 <- old d1
        T* t0 = VP; VP = V; V = Wb; Wb = t0;
        T* t1 = D1; D1 = D2; D2 = t1;
        LABPSD_HIP(hipMemcpyAsync(flag_host_pinned, counter, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        LABPSD_HIP(hipStreamSynchronize(s));
        if (*flag_host_pinned == 0) break;
    }
    hipLaunchKernelGGL((k_minres_final<T>), gel, dim3(256), 0, s, n, q, cols_dev, (const MinresScal*)sc,
                       Xs, P, ldp, its_dev);
    LABPSD_HIP(hipGetLastError());
    nl += 1;
    if (launches) *launches += nl;
}

template void run_minres<double>(const Sell&, double*, int64_t, const double*, int64_t, int,
                                 const int32_t*, const double*, const double*, double, int, int32_t*,
                                 double*, double*, int32_t*, hipStream_t, int64_t*);
template void run_minres<float>(const Sell&, float*, int64_t, const float*, int64_t, int,
                                const int32_t*, const double*, const double*, double, int, int32_t*,
                                float*, double*, int32_t*, hipStream_t, int64_t*);

}  // namespace labpsd
