// Sparse products with the shared pattern of H and S (outline steps 3 and 7, and the
// shifted products (H - sigma S) v of the refinement; Section 5 notes the PUFE code
// forms (H - sigma S) v for any shift).
//
// Layout: sliced ELL with 64-row slices (one row per lane), each slice padded to its
// longest row and stored slot-major, so a wavefront's loads of column indices and
// values are contiguous.  A slice's slots go to one wavefront, or round-robin to four
// whose sums meet in LDS when the launch would otherwise have too few wavefronts.  H and S values sit on the same
// pattern, so one pass over the pattern and one gather of X serve both products.
// Work-groups map slices XCD-locally: consecutive slices land on the same XCD so the
// neighbouring rows' gathers of X hit the same L2.
#include "common.h"

namespace labpsd {

namespace {

// One work-group of 256 threads covers 4 / WPS slices; wavefront `wave` serves slice
// sb * (4 / WPS) + wave / WPS and takes every WPS-th slot of it.  The work-group walks a
// contiguous band of column chunks (grid.y bands of about 32 columns): after the band's
// first chunk the slices' column indices and values come from L1/L2, so the pattern is
// fetched from HBM once per band rather than once per chunk, while the work-groups in
// flight share one band of X (~32 columns), which stays in the last-level cache for the
// neighbouring rows' gathers.
template <int CW, int WPS>
__global__ __launch_bounds__(256) void k_spmm_hs(const int64_t* __restrict__ off,
                                                 const int32_t* __restrict__ col,
                                                 const double* __restrict__ hv,
                                                 const double* __restrict__ sv, int64_t n,
                                                 int64_t nslices, const double* __restrict__ X,
                                                 int64_t ldx, int w, double* __restrict__ YH,
                                                 double* __restrict__ YS, int64_t ldy,
                                                 NlEpi<double, double> nl) {
    constexpr int SPB = 4 / WPS;
    __shared__ double red[WPS > 1 ? 256 * 2 * CW : 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t nblk = (nslices + SPB - 1) / SPB;
    const int64_t sb = xcd_block(blockIdx.x, nblk);
    const int64_t slice = sb * SPB + wave / WPS;
    const int sw = wave % WPS;
    const bool valid = slice < nslices;
    const int64_t row = slice * kSlice + lane;
    const int64_t e0 = valid ? off[slice] : 0, e1 = valid ? off[slice + 1] : 0;
    const int nch = (w + CW - 1) / CW, cpg = (nch + (int)gridDim.y - 1) / (int)gridDim.y;
    const int jb = (int)blockIdx.y * cpg * CW, je = min(w, jb + cpg * CW);
    for (int j0 = jb; j0 < je; j0 += CW) {
        const int nc = min(CW, w - j0);
        double ah[CW], as[CW];
#pragma unroll
        for (int j = 0; j < CW; ++j) { ah[j] = 0.0; as[j] = 0.0; }
        const double* Xj = X + (int64_t)j0 * ldx;
        const double* xp[CW];
#pragma unroll
        for (int j = 0; j < CW; ++j) xp[j] = Xj + (j < nc ? (int64_t)j * ldx : 0);
        sell_accumulate<double, CW>(col, hv, sv, e0 + sw * kSlice + lane, e1, (int64_t)kSlice * WPS, xp, ah, as);
        slice_reduce<double, CW, WPS>(ah, as, red);
        if (valid && sw == 0 && row < n) {
#pragma unroll
            for (int j = 0; j < CW; ++j) {
                if (j < nc) {
                    const double yh = nl.rp ? ah[j] + nl_row_term(nl, row, j0 + j) : ah[j];
                    YH[row + (int64_t)(j0 + j) * ldy] = yh;
                    YS[row + (int64_t)(j0 + j) * ldy] = as[j];
                }
            }
        }
        if constexpr (WPS > 1) __syncthreads();   // red is rewritten by the next chunk
    }
}

// Y[:, j] = H X[:, j] - shift[j] S X[:, j]
template <typename T, int CW, int WPS>
__global__ __launch_bounds__(256) void k_spmm_shift(const int64_t* __restrict__ off,
                                                    const int32_t* __restrict__ col,
                                                    const T* __restrict__ hv,
                                                    const T* __restrict__ sv, int64_t n,
                                                    int64_t nslices, const T* __restrict__ X,
                                                    int64_t ldx, int w,
                                                    const double* __restrict__ shift,
                                                    T* __restrict__ Y, int64_t ldy, NlEpi<T, T> nl) {
    constexpr int SPB = 4 / WPS;
    __shared__ T red[WPS > 1 ? 256 * 2 * CW : 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t nblk = (nslices + SPB - 1) / SPB;
    const int64_t sb = xcd_block(blockIdx.x, nblk);
    const int64_t slice = sb * SPB + wave / WPS;
    const int sw = wave % WPS;
    const bool valid = slice < nslices;
    const int64_t row = slice * kSlice + lane;
    const int64_t e0 = valid ? off[slice] : 0, e1 = valid ? off[slice + 1] : 0;
    const int nch = (w + CW - 1) / CW, cpg = (nch + (int)gridDim.y - 1) / (int)gridDim.y;
    const int jb = (int)blockIdx.y * cpg * CW, je = min(w, jb + cpg * CW);
    for (int j0 = jb; j0 < je; j0 += CW) {
        const int nc = min(CW, w - j0);
        T ah[CW], as[CW];
#pragma unroll
        for (int j = 0; j < CW; ++j) { ah[j] = T(0); as[j] = T(0); }
        const T* Xj = X + (int64_t)j0 * ldx;
        const T* xp[CW];
#pragma unroll
        for (int j = 0; j < CW; ++j) xp[j] = Xj + (j < nc ? (int64_t)j * ldx : 0);
        sell_accumulate<T, CW>(col, hv, sv, e0 + sw * kSlice + lane, e1, (int64_t)kSlice * WPS, xp, ah, as);
        slice_reduce<T, CW, WPS>(ah, as, red);
        if (valid && sw == 0 && row < n) {
#pragma unroll
            for (int j = 0; j < CW; ++j) {
                if (j < nc) {
                    const T sh = (T)shift[j0 + j];
                    const T h = nl.rp ? ah[j] + nl_row_term(nl, row, j0 + j) : ah[j];
                    Y[row + (int64_t)(j0 + j) * ldy] = h - sh * as[j];
                }
            }
        }
        if constexpr (WPS > 1) __syncthreads();
    }
}

}  // namespace

void build_sell(Sell& S, const HostCSR& A, const double* hv, const double* sv, hipStream_t s) {
    const int64_t n = A.n;
    S.n = n;
    S.nslices = (n + kSlice - 1) / kSlice;
    S.h_slice_off.assign(S.nslices + 1, 0);
    for (int64_t sl = 0; sl < S.nslices; ++sl) {
        int64_t mx = 0;
        for (int64_t r = sl * kSlice; r < std::min(n, (sl + 1) * kSlice); ++r)
            mx = std::max<int64_t>(mx, A.rowptr[r + 1] - A.rowptr[r]);
        S.h_slice_off[sl + 1] = S.h_slice_off[sl] + mx * kSlice;
    }
    S.stored = S.h_slice_off[S.nslices];
    std::vector<int32_t> col(S.stored);
    std::vector<double> h(S.stored, 0.0), sv_(S.stored, 0.0);
    std::vector<float> h32(S.stored, 0.0f), s32(S.stored, 0.0f);
    S.h_map.assign(S.stored, -1);
    for (int64_t sl = 0; sl < S.nslices; ++sl) {
        const int64_t base = S.h_slice_off[sl];
        const int64_t len = (S.h_slice_off[sl + 1] - base) / kSlice;
        for (int lane = 0; lane < kSlice; ++lane) {
            const int64_t r = sl * kSlice + lane;
            const int64_t b = r < n ? A.rowptr[r] : 0;
            const int64_t cnt = r < n ? A.rowptr[r + 1] - b : 0;
            for (int64_t k = 0; k < len; ++k) {
                const int64_t e = base + k * kSlice + lane;
                if (k < cnt) {
                    col[e] = A.col[b + k];
                    h[e] = hv[b + k];
                    sv_[e] = sv[b + k];
                    h32[e] = (float)hv[b + k];
                    s32[e] = (float)sv[b + k];
                    S.h_map[e] = b + k;
                } else {
                    col[e] = (int32_t)(r < n ? r : 0);   // padding: own row, value 0
                }
            }
        }
    }
    S.slice_off.upload(S.h_slice_off.data(), S.h_slice_off.size(), s);
    S.col.upload(col.data(), col.size(), s);
    S.hv.upload(h.data(), h.size(), s);
    S.sv.upload(sv_.data(), sv_.size(), s);
    S.hv32.upload(h32.data(), h32.size(), s);
    S.sv32.upload(s32.data(), s32.size(), s);
    LABPSD_HIP(hipStreamSynchronize(s));
}

void refresh_sell_h(Sell& S, const double* hv, hipStream_t s) {
    std::vector<double> h(S.stored, 0.0);
    std::vector<float> h32(S.stored, 0.0f);
    for (int64_t e = 0; e < S.stored; ++e)
        if (S.h_map[e] >= 0) {
            h[e] = hv[S.h_map[e]];
            h32[e] = (float)h[e];
        }
    S.hv.upload(h.data(), h.size(), s);
    S.hv32.upload(h32.data(), h32.size(), s);
    LABPSD_HIP(hipStreamSynchronize(s));
}

// Launch shape: the widest column chunk (fewest passes over the pattern) that, with one
// or four wavefronts per slice, gives want_waves wavefronts; bands of about 32 columns
// (grid.y = their number, more if the wavefront target needs it); when even one chunk
// per band falls short, the shape with the most wavefronts.
SellShape sell_shape(int64_t nslices, int w, int max_cw, int64_t want_waves) {
    constexpr int kBandCols = 32;
    SellShape best{1, 4, 1};
    int64_t best_waves = -1;
    for (int cw : {8, 4, 2, 1}) {
        if (cw > max_cw) continue;
        const int64_t nch = (w + cw - 1) / cw;
        for (int wps : {1, 4}) {
            const int64_t per_group = nslices * wps;
            if (per_group * nch >= want_waves) {
                const int64_t band = std::max(1, kBandCols / cw);
                const int64_t g = std::max<int64_t>((nch + band - 1) / band,
                                                    (want_waves + per_group - 1) / per_group);
                return SellShape{cw, wps, (int)std::max<int64_t>(1, std::min<int64_t>(nch, g))};
            }
            if (per_group * nch > best_waves) {
                best_waves = per_group * nch;
                best = SellShape{cw, wps, (int)std::max<int64_t>(1, nch)};
            }
        }
    }
    return best;
}

template <int CW, int WPS>
static void spmm_hs_cw(const Sell& A, const double* X, int64_t ldx, int w, double* YH, double* YS,
                       int64_t ldy, hipStream_t s, NlEpi<double, double> nl, int groups) {
    constexpr int SPB = 4 / WPS;
    dim3 grid((unsigned)((A.nslices + SPB - 1) / SPB), (unsigned)groups);
    hipLaunchKernelGGL((k_spmm_hs<CW, WPS>), grid, dim3(256), 0, s, A.slice_off.p, A.col.p, A.hv.p,
                       A.sv.p, A.n, A.nslices, X, ldx, w, YH, YS, ldy, nl);
    LABPSD_HIP(hipGetLastError());
}

template <int CW>
static void spmm_hs_w(const Sell& A, SellShape sh, const double* X, int64_t ldx, int w, double* YH,
                      double* YS, int64_t ldy, hipStream_t s, NlEpi<double, double> nl) {
    if (sh.wps == 4) spmm_hs_cw<CW, 4>(A, X, ldx, w, YH, YS, ldy, s, nl, sh.groups);
    else spmm_hs_cw<CW, 1>(A, X, ldx, w, YH, YS, ldy, s, nl, sh.groups);
}

void launch_spmm_hs(const Sell& A, const double* X, int64_t ldx, int w, double* YH, double* YS,
                    int64_t ldy, hipStream_t s, const NonLocal* nlp) {
    if (w <= 0 || A.n == 0) return;
    const NlEpi<double, double> nl =
        nlp ? nl_prepare<double>(*nlp, X, ldx, nullptr, w, s) : NlEpi<double, double>{};
    const SellShape sh = sell_shape(A.nslices, w, 8, 2048);
    switch (sh.cw) {
        case 8: spmm_hs_w<8>(A, sh, X, ldx, w, YH, YS, ldy, s, nl); break;
        case 4: spmm_hs_w<4>(A, sh, X, ldx, w, YH, YS, ldy, s, nl); break;
        case 2: spmm_hs_w<2>(A, sh, X, ldx, w, YH, YS, ldy, s, nl); break;
        default: spmm_hs_w<1>(A, sh, X, ldx, w, YH, YS, ldy, s, nl); break;
    }
}

template <typename T, int CW, int WPS>
static void spmm_shift_cw(const Sell& A, const T* X, int64_t ldx, int w, const double* shift, T* Y,
                          int64_t ldy, hipStream_t s, NlEpi<T, T> nl, int groups) {
    constexpr int SPB = 4 / WPS;
    dim3 grid((unsigned)((A.nslices + SPB - 1) / SPB), (unsigned)groups);
    const T* hv;
    const T* sv;
    if constexpr (sizeof(T) == 8) {
        hv = A.hv.p;
        sv = A.sv.p;
    } else {
        hv = A.hv32.p;
        sv = A.sv32.p;
    }
    hipLaunchKernelGGL((k_spmm_shift<T, CW, WPS>), grid, dim3(256), 0, s, A.slice_off.p, A.col.p, hv, sv,
                       A.n, A.nslices, X, ldx, w, shift, Y, ldy, nl);
    LABPSD_HIP(hipGetLastError());
}

template <typename T, int CW>
static void spmm_shift_w(const Sell& A, SellShape sh, const T* X, int64_t ldx, int w, const double* shift,
                         T* Y, int64_t ldy, hipStream_t s, NlEpi<T, T> nl) {
    if (sh.wps == 4) spmm_shift_cw<T, CW, 4>(A, X, ldx, w, shift, Y, ldy, s, nl, sh.groups);
    else spmm_shift_cw<T, CW, 1>(A, X, ldx, w, shift, Y, ldy, s, nl, sh.groups);
}

template <typename T>
void launch_spmm_shift(const Sell& A, const T* X, int64_t ldx, int w, const double* shift, T* Y,
                       int64_t ldy, hipStream_t s, const NonLocal* nlp) {
    if (w <= 0 || A.n == 0) return;
    const NlEpi<T, T> nl = nlp ? nl_prepare<T>(*nlp, X, ldx, nullptr, w, s) : NlEpi<T, T>{};
    const SellShape sh = sell_shape(A.nslices, w, 8, 2048);
    switch (sh.cw) {
        case 8: spmm_shift_w<T, 8>(A, sh, X, ldx, w, shift, Y, ldy, s, nl); break;
        case 4: spmm_shift_w<T, 4>(A, sh, X, ldx, w, shift, Y, ldy, s, nl); break;
        case 2: spmm_shift_w<T, 2>(A, sh, X, ldx, w, shift, Y, ldy, s, nl); break;
        default: spmm_shift_w<T, 1>(A, sh, X, ldx, w, shift, Y, ldy, s, nl); break;
    }
}

template void launch_spmm_shift<double>(const Sell&, const double*, int64_t, int, const double*,
                                        double*, int64_t, hipStream_t, const NonLocal*);
template void launch_spmm_shift<float>(const Sell&, const float*, int64_t, int, const double*,
                                       float*, int64_t, hipStream_t, const NonLocal*);

}  // namespace labpsd
