// Sparse products with the shared pattern of H and S (outline steps 3 and 7, and the
// shifted products (H - sigma S) v of the refinement; Section 5 notes the PUFE code
// forms (H - sigma S) v for any shift).
//
// Layout: sliced ELL with 64-row slices (one row per lane), each slice padded to its
// longest row and stored slot-major, so the loads of a slot's column indices and values
// are contiguous.  H and S values sit on the same pattern, so one pass over the pattern
// and one gather of X serve both products.
// A work-group of kSellWaves wavefronts owns one slice: it stages the slice's pattern in
// LDS (once when the slice fits one segment) and its wavefronts walk the band's columns
// CW at a time, gathering X straight from global memory.  Work-groups map slices
// XCD-locally: consecutive slices land on the same XCD, so neighbouring rows' gathers of
// X hit the same L2.
#include "common.h"

#include <mutex>
#include <set>
#include <utility>

namespace labpsd {

namespace {

template <int CW>
__global__ __launch_bounds__(64 * kSellWaves) void k_spmm_hs(const int64_t* __restrict__ off,
                                                            const int32_t* __restrict__ col,
                                                            const double* __restrict__ hv,
                                                            const double* __restrict__ sv, int64_t n,
                                                            int64_t nslices, const double* __restrict__ X,
                                                            int64_t ldx, int w, int cpb, int lseg,
                                                            double* __restrict__ YH, double* __restrict__ YS,
                                                            int64_t ldy, NlEpi<double, double> nl) {
    extern __shared__ double sell_dyn[];
    const SliceLds<double> L = slice_lds<double>(sell_dyn, lseg);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t slice = xcd_block(blockIdx.x, nslices);
    const int64_t e0 = off[slice];
    const int nsl = (int)((off[slice + 1] - e0) / kSlice);
    const int nseg = (nsl + lseg - 1) / lseg;
    const int64_t row = slice * kSlice + lane;
    const int jb = (int)blockIdx.y * cpb, je = min(w, jb + cpb);
    if (nseg == 1) {
        sell_stage<double>(col, hv, sv, e0, 0, nsl, L);
        __syncthreads();
    }
    for (int r = jb; r < je; r += kSellWaves * CW) {
        const int j0 = r + wave * CW;
        const bool act = j0 < je;
        double ah[CW], as[CW];
        const double* xp[CW];
#pragma unroll
        for (int j = 0; j < CW; ++j) {
            ah[j] = 0.0;
            as[j] = 0.0;
            xp[j] = X + (int64_t)(j0 + j < je ? j0 + j : jb) * ldx;   // unused columns read a valid one
        }
        for (int sg = 0; sg < nseg; ++sg) {
            const int s0 = sg * lseg, ns = min(lseg, nsl - s0);
            if (nseg > 1) {   // uniform over the work-group
                __syncthreads();
                sell_stage<double>(col, hv, sv, e0, s0, ns, L);
                __syncthreads();
            }
            if (act) sell_lds_accumulate<double, CW>(L, ns, xp, ah, as);
        }
        if (act && row < n) {
#pragma unroll
            for (int j = 0; j < CW; ++j) {
                if (j0 + j < je) {
                    const double yh = nl.rp ? ah[j] + nl_row_term(nl, row, j0 + j) : ah[j];
                    YH[row + (int64_t)(j0 + j) * ldy] = yh;
                    YS[row + (int64_t)(j0 + j) * ldy] = as[j];
                }
            }
        }
    }
}

// Y[:, j] = H X[:, j] - shift[j] S X[:, j]
template <typename T, int CW>
__global__ __launch_bounds__(64 * kSellWaves) void k_spmm_shift(const int64_t* __restrict__ off,
                                                               const int32_t* __restrict__ col,
                                                               const T* __restrict__ hv,
                                                               const T* __restrict__ sv, int64_t n,
                                                               int64_t nslices, const T* __restrict__ X,
                                                               int64_t ldx, int w, int cpb, int lseg,
                                                               const double* __restrict__ shift,
                                                               T* __restrict__ Y, int64_t ldy, NlEpi<T, T> nl) {
    extern __shared__ double sell_dyn[];
    const SliceLds<T> L = slice_lds<T>(sell_dyn, lseg);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t slice = xcd_block(blockIdx.x, nslices);
    const int64_t e0 = off[slice];
    const int nsl = (int)((off[slice + 1] - e0) / kSlice);
    const int nseg = (nsl + lseg - 1) / lseg;
    const int64_t row = slice * kSlice + lane;
    const int jb = (int)blockIdx.y * cpb, je = min(w, jb + cpb);
    if (nseg == 1) {
        sell_stage<T>(col, hv, sv, e0, 0, nsl, L);
        __syncthreads();
    }
    for (int r = jb; r < je; r += kSellWaves * CW) {
        const int j0 = r + wave * CW;
        const bool act = j0 < je;
        T ah[CW], as[CW];
        const T* xp[CW];
#pragma unroll
        for (int j = 0; j < CW; ++j) {
            ah[j] = T(0);
            as[j] = T(0);
            xp[j] = X + (int64_t)(j0 + j < je ? j0 + j : jb) * ldx;
        }
        for (int sg = 0; sg < nseg; ++sg) {
            const int s0 = sg * lseg, ns = min(lseg, nsl - s0);
            if (nseg > 1) {
                __syncthreads();
                sell_stage<T>(col, hv, sv, e0, s0, ns, L);
                __syncthreads();
            }
            if (act) sell_lds_accumulate<T, CW>(L, ns, xp, ah, as);
        }
        if (act && row < n) {
#pragma unroll
            for (int j = 0; j < CW; ++j) {
                if (j0 + j < je) {
                    const T sh = (T)shift[j0 + j];
                    const T h = nl.rp ? ah[j] + nl_row_term(nl, row, j0 + j) : ah[j];
                    Y[row + (int64_t)(j0 + j) * ldy] = h - sh * as[j];
                }
            }
        }
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
    S.max_slots = 0;
    for (int64_t sl = 0; sl < S.nslices; ++sl)
        S.max_slots = std::max<int>(S.max_slots, (int)((S.h_slice_off[sl + 1] - S.h_slice_off[sl]) / kSlice));
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

// Launch shape: 4 columns per wavefront from 32 columns up (2 from 16, else 1), bands of
// about 96 columns (at least one round of kSellWaves * CW each), and LDS segments of as
// many slots as kSellLdsBytes holds (the longest slice's count when it fits).
SellShape sell_shape(const Sell& A, int w, size_t value_bytes) {
    SellShape sh{};
    sh.cw = w >= 32 ? 4 : (w >= 16 ? 2 : 1);
    const int per_round = kSellWaves * sh.cw;
    sh.bands = std::max(1, (w + 63) / 96);
    sh.bands = std::max(1, std::min(sh.bands, (w + per_round - 1) / per_round));
    const size_t slot_bytes = (size_t)kSlice * (2 * value_bytes + sizeof(int32_t));
    sh.lseg = (int)std::max<size_t>(1, std::min<size_t>((size_t)std::max(1, A.max_slots), kSellLdsBytes / slot_bytes));
    sh.lds_bytes = (size_t)sh.lseg * slot_bytes;
    return sh;
}

void allow_dynamic_lds(const void* kernel) {
    static std::mutex mu;
    static std::set<std::pair<const void*, int>> done;
    int dev = 0;
    LABPSD_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    if (done.count({kernel, dev})) return;
    int mx = 0;
    LABPSD_HIP(hipDeviceGetAttribute(&mx, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    // static and dynamic LDS share the work-group's allotment
    hipFuncAttributes fa{};
    LABPSD_HIP(hipFuncGetAttributes(&fa, kernel));
    const int dyn = mx - (int)fa.sharedSizeBytes;
    LABPSD_REQUIRE(dyn >= (int)kSellLdsBytes, "device offers less LDS per work-group than the kernels need");
    LABPSD_HIP(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, dyn));
    done.insert({kernel, dev});
}

template <int CW>
static void spmm_hs_cw(const Sell& A, SellShape sh, const double* X, int64_t ldx, int w, double* YH,
                       double* YS, int64_t ldy, hipStream_t s, NlEpi<double, double> nl) {
    allow_dynamic_lds((const void*)k_spmm_hs<CW>);
    const int cpb = (w + sh.bands - 1) / sh.bands;
    const dim3 grid((unsigned)A.nslices, (unsigned)sh.bands);
    hipLaunchKernelGGL((k_spmm_hs<CW>), grid, dim3(64 * kSellWaves), sh.lds_bytes, s, A.slice_off.p, A.col.p,
                       A.hv.p, A.sv.p, A.n, A.nslices, X, ldx, w, cpb, sh.lseg, YH, YS, ldy, nl);
    LABPSD_HIP(hipGetLastError());
}

void launch_spmm_hs(const Sell& A, const double* X, int64_t ldx, int w, double* YH, double* YS,
                    int64_t ldy, hipStream_t s, const NonLocal* nlp) {
    if (w <= 0 || A.n == 0) return;
    const NlEpi<double, double> nl =
        nlp ? nl_prepare<double>(*nlp, X, ldx, nullptr, w, s) : NlEpi<double, double>{};
    const SellShape sh = sell_shape(A, w, sizeof(double));
    switch (sh.cw) {
        case 4: spmm_hs_cw<4>(A, sh, X, ldx, w, YH, YS, ldy, s, nl); break;
        case 2: spmm_hs_cw<2>(A, sh, X, ldx, w, YH, YS, ldy, s, nl); break;
        default: spmm_hs_cw<1>(A, sh, X, ldx, w, YH, YS, ldy, s, nl); break;
    }
}

template <typename T, int CW>
static void spmm_shift_cw(const Sell& A, SellShape sh, const T* X, int64_t ldx, int w, const double* shift,
                          T* Y, int64_t ldy, hipStream_t s, NlEpi<T, T> nl) {
    const T* hv;
    const T* sv;
    if constexpr (sizeof(T) == 8) {
        hv = A.hv.p;
        sv = A.sv.p;
    } else {
        hv = A.hv32.p;
        sv = A.sv32.p;
    }
    allow_dynamic_lds((const void*)k_spmm_shift<T, CW>);
    const int cpb = (w + sh.bands - 1) / sh.bands;
    const dim3 grid((unsigned)A.nslices, (unsigned)sh.bands);
    hipLaunchKernelGGL((k_spmm_shift<T, CW>), grid, dim3(64 * kSellWaves), sh.lds_bytes, s, A.slice_off.p,
                       A.col.p, hv, sv, A.n, A.nslices, X, ldx, w, cpb, sh.lseg, shift, Y, ldy, nl);
    LABPSD_HIP(hipGetLastError());
}

template <typename T>
void launch_spmm_shift(const Sell& A, const T* X, int64_t ldx, int w, const double* shift, T* Y,
                       int64_t ldy, hipStream_t s, const NonLocal* nlp) {
    if (w <= 0 || A.n == 0) return;
    const NlEpi<T, T> nl = nlp ? nl_prepare<T>(*nlp, X, ldx, nullptr, w, s) : NlEpi<T, T>{};
    const SellShape sh = sell_shape(A, w, sizeof(T));
    switch (sh.cw) {
        case 4: spmm_shift_cw<T, 4>(A, sh, X, ldx, w, shift, Y, ldy, s, nl); break;
        case 2: spmm_shift_cw<T, 2>(A, sh, X, ldx, w, shift, Y, ldy, s, nl); break;
        default: spmm_shift_cw<T, 1>(A, sh, X, ldx, w, shift, Y, ldy, s, nl); break;
    }
}

template void launch_spmm_shift<double>(const Sell&, const double*, int64_t, int, const double*,
                                        double*, int64_t, hipStream_t, const NonLocal*);
template void launch_spmm_shift<float>(const Sell&, const float*, int64_t, int, const double*,
                                       float*, int64_t, hipStream_t, const NonLocal*);

}  // namespace labpsd
