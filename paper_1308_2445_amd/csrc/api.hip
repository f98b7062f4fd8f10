// C ABI of liblabpsd and the LABPSD solve driver (Section 3 outline, hybrid scheme).
//
// The driver runs on the host and enqueues every step of an iteration as device
// kernels on the context's stream.  Per outer iteration it reads back one small
// vector (Res of the nev wanted pairs and the Ritz values) to take the host-side
// decisions: convergence, the unconverged set U (remark 3: step 6 only for the
// unconverged pairs) and the localisation test (remark 4).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>

#include "common.h"
#include "hermitian.h"

namespace labpsd {

void spin_event(hipEvent_t ev) {
    for (;;) {
        const hipError_t e = hipEventQuery(ev);
        if (e == hipSuccess) break;
        if (e != hipErrorNotReady) LABPSD_HIP(e);
    }
    // a query that found the event pending may leave "not ready" as the last error
    (void)hipGetLastError();
}

void spin_sync(hipStream_t s, hipEvent_t ev) {
    if (!ev) {
        LABPSD_HIP(hipStreamSynchronize(s));
        return;
    }
    LABPSD_HIP(hipEventRecord(ev, s));
    spin_event(ev);
}

namespace {
thread_local std::string g_err;

double wall() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

template <typename F>
labpsd_status guarded(F&& f) {
    try {
        g_err.clear();
        // a launch error left behind by other code on this thread is not ours
        (void)hipGetLastError();
        return f();
    } catch (const Error& e) {
        g_err = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        g_err = "host allocation failed";
        return LABPSD_ENOMEM;
    } catch (const std::exception& e) {
        g_err = e.what();
        return LABPSD_EINVAL;
    }
}

// pinned host staging buffer

// Event timing of the steps (stats.t_step_s)

struct StepTimer {
    bool on = false;
    hipStream_t s = nullptr;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> marks;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    int cur = -1;
    hipEvent_t cur_start = nullptr;
    hipEvent_t get() {
        if (used == pool.size()) {
            hipEvent_t e;
            LABPSD_HIP(hipEventCreate(&e));
            pool.push_back(e);
        }
        return pool[used++];
    }
    void begin(int step) {
        if (!on) return;
        cur = step;
        cur_start = get();
        LABPSD_HIP(hipEventRecord(cur_start, s));
    }
    void end() {
        if (!on || cur < 0) return;
        hipEvent_t e = get();
        LABPSD_HIP(hipEventRecord(e, s));
        marks.push_back({cur, {cur_start, e}});
        cur = -1;
    }
    // fold recorded intervals into the stats (stream must be synchronised)
    void collect(labpsd_stats* st) {
        if (!on) return;
        for (auto& m : marks) {
            float ms = 0.f;
            LABPSD_HIP(hipEventElapsedTime(&ms, m.second.first, m.second.second));
            if (st) st->t_step_s[m.first] += ms * 1e-3;
        }
        marks.clear();
        used = 0;
    }
    ~StepTimer() {
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

enum Step { S_PROD_PSI = 0, S_RESID, S_GLOBAL, S_LOCAL, S_PROD_P, S_GRAM, S_RR, S_UPDATE, S_CAST };

}  // namespace

void set_error(const std::string& msg) { g_err = msg; }
const char* get_error() { return g_err.c_str(); }

Problem::~Problem() { delete factor; }

// ------------------------------------------------------------------ factor upload

static void upload_factor(Problem& P, const HostFactor& H, double eps_bar, unsigned panels) {
    hipStream_t s = P.ctx->stream;
    auto F = std::make_unique<DevFactor>();
    F->n = H.n;
    F->nsn = (int)H.sn.size();
    F->nlevels = H.nlevels;
    F->eps_bar = eps_bar;
    F->rows.upload(H.rows.data(), H.rows.size(), s);
    if (panels & LABPSD_PANELS_FP64) F->panels64.upload(H.panels.data(), H.panels.size(), s);
    if (panels & LABPSD_PANELS_FP32) {
        std::vector<float> p32(H.panels.size());
        for (size_t i = 0; i < p32.size(); ++i) p32[i] = (float)H.panels[i];
        F->panels32.upload(p32.data(), p32.size(), s);
        LABPSD_HIP(hipStreamSynchronize(s));
    }
    // tasks: 64-row output tiles x 64-wide reduction chunks; per level the off-diagonal
    // products (op 1: r_B -= F r_D, op 2: x_D -= F^T x_B), then one list of the diagonal
    // products x_D = G r_D of every supernode
    constexpr int kTile = 64;
    int kChunk = 64;
    std::vector<SnTask> tk;
    F->lev_off.assign(4 * (size_t)F->nlevels, 0);
    F->lev_count.assign(4 * (size_t)F->nlevels, 0);
    auto add_tasks = [&](const Supernode& sn, int op) {
        const int ncol = sn.ncol, nb = sn.nrow - sn.ncol;
        const int nout = (op == 1) ? nb : ncol;
        const int nred = (op == 2) ? nb : ncol;
        for (int t = 0; t * kTile < nout; ++t)
            for (int kc = 0; kc < nred; kc += kChunk)
                tk.push_back(SnTask{sn.idx_off, sn.val_off, ncol, sn.nrow, t * kTile, kc});
    };
    for (int l = 0; l < F->nlevels; ++l) {
        for (int op = 1; op <= 2; ++op) {
            F->lev_off[4 * l + op] = (int64_t)tk.size();
            for (int i = 0; i < F->nsn; ++i)
                if (H.sn[i].level == l) add_tasks(H.sn[i], op);
            F->lev_count[4 * l + op] = (int64_t)tk.size() - F->lev_off[4 * l + op];
        }
    }
    F->diag_off = (int64_t)tk.size();
    for (int i = 0; i < F->nsn; ++i) add_tasks(H.sn[i], 0);
    F->diag_count = (int64_t)tk.size() - F->diag_off;
    // the single-launch sweep: forward tasks by level from the leaves, the diagonal
    // tasks by level, backward tasks by level from the roots (every dependency earlier
    // in the list); counters (children, forward tasks, diagonal + backward tasks)
    std::vector<int32_t> init, init_deep;
    std::vector<SweepTask> sw, sw_deep;
    auto build_sweep = [&](int chunk, std::vector<SweepTask>& list, std::vector<int32_t>& counts) {
        kChunk = chunk;
        counts.assign(3 * (size_t)F->nsn, 0);
        const int nsn = F->nsn;
        bool tree_ok = true;
        for (int i = 0; i < nsn; ++i) {
            const Supernode& sn = H.sn[i];
            const int nb = sn.nrow - sn.ncol;
            if (sn.parent >= 0) {
                // a child counts itself off with its last forward task, so it needs one
                if (sn.parent >= nsn || H.sn[sn.parent].level <= sn.level || nb == 0) tree_ok = false;
                else ++counts[sn.parent];
            } else if (nb > 0) {
                tree_ok = false;   // rows outside the supernode need a parent to own them
            }
        }
        auto add_sweep = [&](int i, int op_list, int op_kernel) {
            const size_t before = tk.size();
            add_tasks(H.sn[i], op_list);
            for (size_t t = before; t < tk.size(); ++t) list.push_back(SweepTask{tk[t], op_kernel, i, H.sn[i].parent, 0});
            const int32_t added = (int32_t)(tk.size() - before);
            tk.resize(before);
            if (op_list == 1) counts[nsn + i] += added;
            else counts[2 * (size_t)nsn + i] += added;
        };
        for (int l = 0; l < F->nlevels; ++l)
            for (int i = 0; i < nsn; ++i)
                if (H.sn[i].level == l) add_sweep(i, 1, 2);
        for (int l = 0; l < F->nlevels; ++l)
            for (int i = 0; i < nsn; ++i)
                if (H.sn[i].level == l) add_sweep(i, 0, 0);
        for (int l = F->nlevels - 1; l >= 0; --l)
            for (int i = 0; i < nsn; ++i)
                if (H.sn[i].level == l) add_sweep(i, 2, 3);
        return tree_ok && !list.empty();
    };
    // the single-launch sweep twice: 64-deep reductions per task, and kDeepChunk-deep ones
    // for wide right-hand-side blocks (fewer tasks per supernode, same order)
    F->use_sweep = build_sweep(kDeepChunk, sw_deep, init_deep) && build_sweep(64, sw, init);
    kChunk = 64;
    // host vectors stay alive until the copies have finished
    F->tasks.upload(tk.data(), tk.size(), s);
    if (F->use_sweep) {
        F->sweep.upload(sw.data(), sw.size(), s);
        F->sweep_init.upload(init.data(), init.size(), s);
        F->sweep_deep.upload(sw_deep.data(), sw_deep.size(), s);
        F->sweep_init_deep.upload(init_deep.data(), init_deep.size(), s);
    }
    LABPSD_HIP(hipStreamSynchronize(s));
    F->info.n_supernodes = F->nsn;
    F->info.n_levels = F->nlevels;
    F->info.nnz_factor = H.nnz_factor;
    F->info.flops_factor = H.flops;
    F->info.t_order_s = H.t_order;
    F->info.t_factor_s = H.t_factor;
    delete P.factor;
    P.factor = F.release();
}

// ------------------------------------------------------------------ workspace

namespace {

template <typename T>
struct PrecWS {
    T* Y;
    T* W1;
    T* W2;
    T* RT;
    T* mres;
};

struct SolveBuffers {
    // FP64 blocks
    double* Zb[2][3];
    double* R;
    double* HR;
    double* SR;
    double* W;
    double* gamma;
    double* res;
    double* rnorm;
    double* red;
    double* gram_ws;
    double* shifts;
    double* stopn;
    double* scal;
    void* rr_ws;
    int32_t* cols;
    int32_t* loc;
    int32_t* info;
    int32_t* its;
    int32_t* counter;
};

}  // namespace

// Reserve the solve workspace inside the problem and carve it up (sizes from
// solve_arena_elems).
template <typename T>
static void carve(Problem& P, int64_t n, int b, int m, SolveBuffers& B, PrecWS<T>& W) {
    const int kmax = b + m;
    const int nblk = residual_blocks(n);
    size_t gws = 0;
    for (int k = 1; k <= kmax; ++k) gws = std::max(gws, gram_ws_doubles(n, k, P.ctx->cu_count));
    const size_t rrb = (rr_ws_bytes(kmax) + 7) / 8;
    const ArenaElems need =
        solve_arena_elems(n, m, b - m, sizeof(T) == 8 ? LABPSD_FP64 : LABPSD_MIXED, P.ctx->cu_count);
    P.ws64.alloc(need.ws64);
    double* p = P.ws64.p;
    for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 3; ++c) { B.Zb[a][c] = p; p += (size_t)n * kmax; }
    B.R = p; p += (size_t)n * m;
    B.HR = p; p += (size_t)kmax * kmax;
    B.SR = p; p += (size_t)kmax * kmax;
    B.W = p; p += (size_t)kmax * b;
    // read back together once per iteration: Res, the residual norms, the Ritz values
    B.res = p; p += m;
    B.rnorm = p; p += m;
    B.gamma = p; p += b;
    B.red = p; p += std::max<size_t>((size_t)nblk * m * 2, (size_t)nblk * m);
    B.gram_ws = p; p += gws;
    // sent together once per iteration: shifts, stopping norms and the column lists;
    // then the MINRES counts and the Rayleigh-Ritz report, read back together
    B.shifts = p; p += m;
    B.stopn = p; p += m;
    {
        int32_t* ip = (int32_t*)p;
        B.cols = ip;
        B.loc = ip + m;
        B.its = ip + 2 * m;
        B.info = ip + 3 * m;
        B.counter = B.info + 4;
        p += 2 * (size_t)m + 4;   // 4 m + 8 int32
    }
    B.scal = p; p += minres_scal_doubles(m) + 4;
    B.rr_ws = (void*)p; p += rrb;
    // T-precision blocks
    T* t;
    if constexpr (sizeof(T) == 8) {
        // FP64 mode: the preconditioner blocks live in a second FP64 arena
        P.red.alloc(need.red);
        t = P.red.p;
    } else {
        P.ws32.alloc(need.ws32);
        t = P.ws32.p;
    }
    W.Y = t; t += (size_t)n * m;
    W.W1 = t; t += (size_t)n * m;
    W.W2 = t; t += (size_t)n * m;
    W.RT = t; t += (size_t)n * m;
    W.mres = t;
}

// ------------------------------------------------------------------ solve

template <typename T>
static labpsd_status solve_impl(Problem& P, const labpsd_solve_params& prm, const double* X0,
                                const double* E0, labpsd_mem in_where, double* lambda, double* X,
                                double* res_hist, double* ritz_hist, int* n_hist, labpsd_mem out_where,
                                labpsd_stats* stats, hipStream_t s) {
    const double t_start = wall();
    const int64_t n = P.n;
    const int m = prm.nev, b = prm.nev + prm.m0;
    const int kmax = b + m;
    const int64_t ldz = n;
    SolveBuffers B;
    PrecWS<T> Wt;
    carve<T>(P, n, b, m, B, Wt);
    const NonLocal* nlp = P.nl.k ? &P.nl : nullptr;   // H = H_loc + F G F^T
    const int nblk = residual_blocks(n);
    labpsd_stats st{};
    StepTimer tm;
    tm.on = prm.timing != 0;
    tm.s = s;

    // h_rb: [Res | norms | Ritz values]; h_ib: [unused m | Rayleigh-Ritz report]; the
    // residual and Rayleigh-Ritz kernels write them directly (device-mapped pinned memory);
    // h_sel: [shifts | stopping norms | U | localised positions] as laid out on the device
    HBuf<double>& h_rb = P.h_rb;
    HBuf<double>& h_sel = P.h_sel;
    HBuf<int32_t>& h_ib = P.h_ib;
    HBuf<int32_t>& h_int = P.h_flags;
    h_rb.alloc(2 * (size_t)m + b + 1);
    h_ib.alloc((size_t)m + 4);
    h_sel.alloc(3 * (size_t)m);
    h_int.alloc(2 * (size_t)m);   // MINRES done flags: two slots of up to m columns
    // a report word is only ever read after the kernel that writes it has completed; start
    // every solve from zeros so no value of an earlier solve can stand in for it
    std::memset(h_ib.p, 0, ((size_t)m + 4) * sizeof(int32_t));
    std::memset(h_rb.p, 0, (2 * (size_t)m + b + 1) * sizeof(double));
    P.events.ensure();
    hipEvent_t ev_sync = P.events.e[0], ev_flag0 = P.events.e[1], ev_flag1 = P.events.e[2];
    int32_t* h_cols = (int32_t*)(h_sel.p + 2 * (size_t)m);
    double* d_rb = nullptr;
    int32_t* d_ib = nullptr;
    LABPSD_HIP(hipHostGetDevicePointer((void**)&d_rb, h_rb.p, 0));
    LABPSD_HIP(hipHostGetDevicePointer((void**)&d_ib, h_ib.p, 0));
    // MINRES iterations of the whole solve, summed on the device (a spare scalar word)
    auto* its_total = (unsigned long long*)(B.scal + minres_scal_doubles(m));
    LABPSD_HIP(hipMemsetAsync(its_total, 0, sizeof(unsigned long long), s));
    int cur = 0;
    auto Z = [&](int which) { return B.Zb[cur][which]; };

    // steps 1-3: start block (given, or the seeded random block of a cold start), its
    // products and one Rayleigh-Ritz step on span(X0)
    if (X0)
        LABPSD_HIP(hipMemcpy2DAsync(Z(0), ldz * sizeof(double), X0, n * sizeof(double),
                                    n * sizeof(double), b,
                                    in_where == LABPSD_MEM_DEVICE ? hipMemcpyDeviceToDevice
                                                                  : hipMemcpyHostToDevice,
                                    s));
    else
        launch_random_block(n, b, prm.seed, Z(0), ldz, s);
    tm.begin(S_PROD_PSI);
    launch_spmm_hs(P.sell, Z(0), ldz, b, Z(1), Z(2), ldz, s, nlp);
    tm.end();
    st.n_launch[S_PROD_PSI] += 1;
    st.n_cols[S_PROD_PSI] += b;
    auto rayleigh_ritz_update = [&](int k) {
        tm.begin(S_GRAM);
        launch_gram(n, k, Z(0), Z(1), Z(2), ldz, B.HR, B.SR, kmax, B.gram_ws, P.ctx->cu_count, s);
        tm.end();
        st.n_launch[S_GRAM] += 1;
        st.n_cols[S_GRAM] += k;
        tm.begin(S_RR);
        launch_rayleigh_ritz(k, b, B.HR, B.SR, kmax, B.gamma, B.W, kmax, B.info, B.rr_ws, s, d_rb + 2 * m,
                             d_ib + m);
        tm.end();
        st.n_launch[S_RR] += 1;
        st.n_cols[S_RR] += k;
        tm.begin(S_UPDATE);
        const int nxt = 1 - cur;
        launch_block_update(n, k, b, Z(0), Z(1), Z(2), ldz, B.W, kmax, B.Zb[nxt][0], B.Zb[nxt][1],
                            B.Zb[nxt][2], ldz, s);
        tm.end();
        st.n_launch[S_UPDATE] += 1;
        st.n_cols[S_UPDATE] += k;
        cur = nxt;
        // the Ritz values and the rank report reach the host with the next residual
        // read-back (rr_check), so this step adds no synchronisation
    };
    // after a synchronisation: the last Rayleigh-Ritz step's report and Ritz values
    std::vector<double> E;
    auto rr_check = [&](const char* what) {
        st.rank_dropped += h_ib.p[m];
        if (h_ib.p[m + 1] != 0) throw Error{LABPSD_ERANK, what};
        E.assign(h_rb.p + 2 * m, h_rb.p + 2 * m + b);
    };
    rayleigh_ritz_update(b);
    std::vector<double> Eprev;
    if (E0) Eprev.assign(E0, E0 + m);
    bool fresh = false;
    int since_refresh = 0;
    bool converged = false;
    int outer = 0, nh = 0;
    std::vector<double> res(m), rn(m);
    std::vector<int32_t> U, locpos;
    std::vector<double> shifts, stopn;
    const LocalParams& lp = P.local;

    // S-orthonormality of Psi (row a8's safeguard): at every refresh, Psi^T S Psi from the
    // fresh products; max |Psi^T S Psi - I| reaches the host with the next residual read
    // (slot 2m + b of h_rb), and above reorth_tol a Rayleigh-Ritz step on span(Psi) (the
    // Cholesky of Psi^T S Psi, then the rotation to its Ritz basis) restores it
    const double reorth_tol = prm.reorth_tol > 0.0 ? prm.reorth_tol : (prm.reorth_tol < 0.0 ? -1.0 : 1e-10);
    bool orth_pending = false;
    auto refresh = [&]() {
        tm.begin(S_PROD_PSI);
        launch_spmm_hs(P.sell, Z(0), ldz, b, Z(1), Z(2), ldz, s, nlp);
        tm.end();
        st.n_launch[S_PROD_PSI] += 1;
        st.n_cols[S_PROD_PSI] += b;
        fresh = true;
        since_refresh = 0;
        st.refreshes += 1;
        tm.begin(S_GRAM);
        launch_gram(n, b, Z(0), Z(1), Z(2), ldz, B.HR, B.SR, kmax, B.gram_ws, P.ctx->cu_count, s);
        launch_orth_deviation(b, B.SR, kmax, d_rb + 2 * m + b, s);
        tm.end();
        st.n_launch[S_GRAM] += 1;
        st.n_cols[S_GRAM] += b;
        orth_pending = true;
    };
    // after a synchronisation: true if Psi had to be S-orthonormalised again (the caller
    // recomputes the residuals and reads the new Ritz values)
    auto restore_orth = [&]() -> bool {
        if (!orth_pending) return false;
        orth_pending = false;
        const double dev = h_rb.p[2 * (size_t)m + b];
        if (reorth_tol >= 0.0 && dev <= reorth_tol) return false;
        tm.begin(S_RR);
        launch_rayleigh_ritz(b, b, B.HR, B.SR, kmax, B.gamma, B.W, kmax, B.info, B.rr_ws, s, d_rb + 2 * m,
                             d_ib + m);
        tm.end();
        st.n_launch[S_RR] += 1;
        st.n_cols[S_RR] += b;
        tm.begin(S_UPDATE);
        const int nxt = 1 - cur;
        launch_block_update(n, b, b, Z(0), Z(1), Z(2), ldz, B.W, kmax, B.Zb[nxt][0], B.Zb[nxt][1],
                            B.Zb[nxt][2], ldz, s);
        tm.end();
        st.n_launch[S_UPDATE] += 1;
        st.n_cols[S_UPDATE] += b;
        cur = nxt;
        st.reorths += 1;
        return true;
    };
    auto residuals = [&]() {
        tm.begin(S_RESID);
        launch_residual(n, m, Z(1), Z(2), ldz, B.gamma, prm.sigma0, B.R, n, B.red, nblk, s);
        // the global apply's error word (a dependency wait that ran out) comes back with Res
        launch_residual_finish(m, B.red, nblk, B.res, B.rnorm, s, d_rb, P.factor->sweep_cnt.p, d_ib + m + 2);
        tm.end();
        st.n_launch[S_RESID] += 1;
        st.n_cols[S_RESID] += m;
        spin_sync(s, ev_sync);
        if (h_ib.p[m + 2] != 0) check_precond_sweep(*P.factor, s);   // raises EHIP
        for (int i = 0; i < m; ++i) { res[i] = h_rb.p[i]; rn[i] = h_rb.p[m + i]; }
    };
    auto maxres = [&]() {
        double mx = 0.0;
        for (double r : res) mx = std::max(mx, std::isnan(r) ? INFINITY : r);
        return mx;
    };
    std::vector<double> hist, rhist;   // Res and the Ritz values at the start of every iteration
    for (int it = 1; it <= prm.max_outer; ++it) {
        if (since_refresh >= prm.refresh_every) refresh();
        residuals();   // step 4 and eq. (res1)
        rr_check(it == 1 ? "start block is rank deficient"
                         : "search space [Psi P] lost rank below the block width");
        if (restore_orth()) {
            residuals();
            rr_check("Psi lost rank below the block width");
        }
        if (maxres() <= prm.tol) {   // step 5, on the true residual
            if (!fresh) {
                refresh();
                residuals();
                if (restore_orth()) {
                    residuals();
                    rr_check("Psi lost rank below the block width");
                }
            }
            if (maxres() <= prm.tol) {
                converged = true;
                hist.insert(hist.end(), res.begin(), res.end());
                rhist.insert(rhist.end(), E.begin(), E.end());
                ++nh;
                break;
            }
        }
        hist.insert(hist.end(), res.begin(), res.end());
        rhist.insert(rhist.end(), E.begin(), E.end());
        ++nh;
        outer = it;
        // step 6: directions for the unconverged pairs
        U.clear();
        for (int i = 0; i < m; ++i)
            if (!(res[i] <= prm.tol)) U.push_back(i);
        const int p = (int)U.size();
        locpos.clear();
        shifts.clear();
        stopn.clear();
        if ((lp.mode == LABPSD_HYBRID || lp.mode == LABPSD_LOCAL_ONLY) && !Eprev.empty()) {
            for (int c = 0; c < p; ++c) {
                const int i = U[c];
                if (res[i] <= lp.tau1 && std::fabs(E[i] - Eprev[i]) <= lp.tau2 * std::fabs(Eprev[i])) {
                    locpos.push_back(c);
                    shifts.push_back(E[i]);
                    stopn.push_back(rn[i]);
                }
            }
        }
        const int q = (int)locpos.size();
        // the selections in one pinned copy (shifts, stopping norms, U, localised
        // positions); the host buffer is next written after the next synchronisation
        std::copy(shifts.begin(), shifts.end(), h_sel.p);
        std::copy(stopn.begin(), stopn.end(), h_sel.p + m);
        std::copy(U.begin(), U.end(), h_cols);
        std::copy(locpos.begin(), locpos.end(), h_cols + m);
        LABPSD_HIP(hipMemcpyAsync(B.shifts, h_sel.p, 2 * (size_t)m * sizeof(double) + (m + q) * sizeof(int32_t),
                                  hipMemcpyHostToDevice, s));
        // 6(a): P = -K^{-1} R_U in the preconditioner precision
        // (the preconditioner works on row-major blocks: -R_U is cast into Y row-major)
        tm.begin(S_CAST);
        launch_cast_to_rm<double, T>(n, p, B.R, n, B.cols, -1.0, Wt.Y, s);
        if (q) launch_gather_cast<double, T>(n, p, B.R, n, B.cols, 1.0, Wt.RT, n, s);
        tm.end();
        st.n_launch[S_CAST] += q ? 2 : 1;
        st.n_cols[S_CAST] += q ? 2 * p : p;
        tm.begin(S_GLOBAL);
        launch_precond_solve<T>(*P.factor, Wt.Y, Wt.W1, Wt.W2, n, p, s, nlp);
        tm.end();
        st.n_launch[S_GLOBAL] += 1;
        st.n_cols[S_GLOBAL] += p;
        // 6(b): MINRES refinement of the localised columns (column-major copy in W1, which
        // the preconditioner no longer needs)
        if (q) {
            tm.begin(S_CAST);
            launch_cast_from_rm<T, T>(n, p, Wt.W2, 1.0, Wt.W1, n, s);
            tm.end();
            st.n_launch[S_CAST] += 1;
            st.n_cols[S_CAST] += p;
            if (lp.mode == LABPSD_LOCAL_ONLY)
                launch_scatter_cast<T, T>(n, q, Wt.W1, n, B.loc, 0.0, Wt.W1, n, s);
            tm.begin(S_LOCAL);
            int64_t nl = 0;
            run_minres<T>(P.sell, Wt.W1, n, Wt.RT, n, q, B.loc, B.shifts, B.stopn, lp.eta,
                          lp.max_inner, B.its, Wt.mres, B.scal, h_int.p, s, &nl, ev_flag0,
                          ev_flag1, its_total, lp.method, nlp);
            tm.end();
            st.n_launch[S_LOCAL] += nl;
            st.n_cols[S_LOCAL] += q;
            st.localized_cols += q;
        }
        // P into the search-space block, FP64
        tm.begin(S_CAST);
        if (q) launch_gather_cast<T, double>(n, p, Wt.W1, n, nullptr, 1.0, Z(0) + (size_t)b * ldz, ldz, s);
        else launch_cast_from_rm<T, double>(n, p, Wt.W2, 1.0, Z(0) + (size_t)b * ldz, ldz, s);
        tm.end();
        st.n_launch[S_CAST] += 1;
        st.n_cols[S_CAST] += p;
        // step 7: P_H, P_S
        tm.begin(S_PROD_P);
        launch_spmm_hs(P.sell, Z(0) + (size_t)b * ldz, ldz, p, Z(1) + (size_t)b * ldz,
                       Z(2) + (size_t)b * ldz, ldz, s, nlp);
        tm.end();
        st.n_launch[S_PROD_P] += 1;
        st.n_cols[S_PROD_P] += p;
        // steps 8-11
        Eprev.assign(E.begin(), E.begin() + m);
        rayleigh_ritz_update(b + p);
        fresh = false;
        ++since_refresh;
    }
    unsigned long long its_sum = 0;
    LABPSD_HIP(hipMemcpyAsync(&its_sum, its_total, sizeof(its_sum), hipMemcpyDeviceToHost, s));
    LABPSD_HIP(hipStreamSynchronize(s));
    st.minres_iters += (int64_t)its_sum;
    check_precond_sweep(*P.factor, s);
    // a converged exit has checked the last Rayleigh-Ritz step in its final iteration
    if (!converged)
        rr_check(outer == 0 ? "start block is rank deficient"
                            : "search space [Psi P] lost rank below the block width");
    tm.collect(&st);
    // keep the whole block (guards included) resident for a warm start
    P.resident_X.alloc((size_t)n * b);
    LABPSD_HIP(hipMemcpy2DAsync(P.resident_X.p, n * sizeof(double), Z(0), ldz * sizeof(double),
                                n * sizeof(double), b, hipMemcpyDeviceToDevice, s));
    P.resident_E = E;
    P.resident_b = b;
    // outputs
    const hipMemcpyKind kd = out_where == LABPSD_MEM_DEVICE ? hipMemcpyDeviceToDevice
                                                            : hipMemcpyDeviceToHost;
    LABPSD_HIP(hipMemcpyAsync(lambda, B.gamma, m * sizeof(double), kd, s));
    LABPSD_HIP(hipMemcpy2DAsync(X, n * sizeof(double), Z(0), ldz * sizeof(double), n * sizeof(double),
                                m, kd, s));
    if (res_hist && nh > 0) {
        if (out_where == LABPSD_MEM_DEVICE)
            LABPSD_HIP(hipMemcpyAsync(res_hist, hist.data(), hist.size() * sizeof(double),
                                      hipMemcpyHostToDevice, s));
        else
            std::memcpy(res_hist, hist.data(), hist.size() * sizeof(double));
    }
    if (ritz_hist && nh > 0) {
        if (out_where == LABPSD_MEM_DEVICE)
            LABPSD_HIP(hipMemcpyAsync(ritz_hist, rhist.data(), rhist.size() * sizeof(double),
                                      hipMemcpyHostToDevice, s));
        else
            std::memcpy(ritz_hist, rhist.data(), rhist.size() * sizeof(double));
    }
    LABPSD_HIP(hipStreamSynchronize(s));
    if (n_hist) *n_hist = nh;
    st.outer_iters = outer;
    st.hp = outer;
    st.la = outer > 0 ? (double)st.minres_iters / ((double)outer * m) : 0.0;
    st.t_solve_s = wall() - t_start;
    if (stats) *stats = st;
    return converged ? LABPSD_OK : LABPSD_NOT_CONVERGED;
}

labpsd_status run_solve(Problem& P, const labpsd_solve_params& prm, const double* X0,
                        const double* E0, labpsd_mem in_where, double* lambda, double* X,
                        double* res_hist, double* ritz_hist, int* n_hist, labpsd_mem out_where, labpsd_stats* stats,
                        hipStream_t stream) {
    if (prm.precision == LABPSD_MIXED)
        return solve_impl<float>(P, prm, X0, E0, in_where, lambda, X, res_hist, ritz_hist, n_hist, out_where,
                                 stats, stream);
    return solve_impl<double>(P, prm, X0, E0, in_where, lambda, X, res_hist, ritz_hist, n_hist, out_where,
                              stats, stream);
}

ArenaElems solve_arena_elems(int64_t n, int nev, int m0, int precision, int cu_count) {
    const int b = nev + m0, m = nev, kmax = b + m;
    const int nblk = residual_blocks(n);
    // the Gram partial layout depends on k; reserve the largest over every k <= kmax
    size_t gws = 0;
    for (int k = 1; k <= kmax; ++k) gws = std::max(gws, gram_ws_doubles(n, k, cu_count));
    const size_t rrb = (rr_ws_bytes(kmax) + 7) / 8;
    ArenaElems a;
    // carve(): the six search-space blocks, R, H_R and S_R, W, the read-back and upload
    // blocks, the residual partials, the Gram partials, the MINRES scalars, the
    // Rayleigh-Ritz workspace
    a.ws64 = 6 * (size_t)n * kmax + (size_t)n * m + 2 * (size_t)kmax * kmax + (size_t)kmax * b + (size_t)b +
             2 * (size_t)m + std::max<size_t>((size_t)nblk * m * 2, (size_t)nblk * m) + gws + 2 * (size_t)m +
             (2 * (size_t)m + 4) + minres_scal_doubles(m) + 4 + rrb + 64;
    // the preconditioner blocks Y, W1, W2, R^T and the MINRES workspace, in the solve's
    // refinement precision
    const size_t t = 4 * (size_t)n * m + minres_ws_elems(n, m);
    if (precision == LABPSD_MIXED) a.ws32 = t;
    else a.red = t;
    return a;
}

size_t solve_footprint_bytes(int64_t n, int nev, int m0, int precision, int cu_count) {
    return solve_arena_elems(n, nev, m0, precision, cu_count).bytes() +
           (size_t)n * (nev + m0) * 8 /* resident block */;
}

labpsd_status abi_guard(const std::function<labpsd_status()>& f) { return guarded(f); }

}  // namespace labpsd

using namespace labpsd;

// ------------------------------------------------------------------ C ABI


namespace labpsd {
template <typename T>
static void local_refine_impl(Problem* p, DBuf<T>& arena, const double* R, int64_t ldr,
                              double* Pm, int64_t ldp, int q, const int32_t* cols,
                              const double* shift, double eta, int max_inner, int32_t* its) {
    hipStream_t s = p->ctx->stream;
    const int64_t n = p->n;
    const size_t mw = minres_ws_elems(n, q);
    arena.alloc(2 * (size_t)n * q + mw);
    T* PT = arena.p;
    T* RT = PT + (size_t)n * q;
    T* mws = RT + (size_t)n * q;
    const int nblk = residual_blocks(n);
    p->ctx->scratch.alloc((size_t)nblk * q + minres_scal_doubles(q) + 8 + q);
    double* part = p->ctx->scratch.p;
    double* scal = part + (size_t)nblk * q;
    double* rn = scal + minres_scal_doubles(q) + 4;
    p->iws.alloc((size_t)q + 8);
    int32_t* iota = p->iws.p;
    std::vector<int32_t> h(q);
    for (int j = 0; j < q; ++j) h[j] = j;
    LABPSD_HIP(hipMemcpyAsync(iota, h.data(), q * sizeof(int32_t), hipMemcpyHostToDevice, s));
    launch_gather_cast<double, T>(n, q, Pm, ldp, cols, 1.0, PT, n, s);
    launch_gather_cast<double, T>(n, q, R, ldr, cols, 1.0, RT, n, s);
    launch_colnorms<double>(n, q, R, ldr, cols, part, rn, s);
    HBuf<int32_t> flag;
    flag.alloc(2 * (size_t)q);
    run_minres<T>(p->sell, PT, n, RT, n, q, iota, shift, rn, eta, max_inner, its, mws, scal, flag.p, s,
                  nullptr, nullptr, nullptr, nullptr, p->local.method, p->nl.k ? &p->nl : nullptr);
    launch_scatter_cast<T, double>(n, q, PT, n, cols, 1.0, Pm, ldp, s);
    LABPSD_HIP(hipStreamSynchronize(s));
}

}  // namespace labpsd

namespace labpsd {
// Host copies of caller arrays that may live on the device (read synchronously on the
// context's stream) or on the host (used in place).
template <typename T>
static const T* host_view(labpsd_ctx* ctx, const T* a, size_t count, labpsd_mem where,
                          std::vector<T>& keep) {
    if (where == LABPSD_MEM_HOST) return a;
    LABPSD_REQUIRE(where == LABPSD_MEM_DEVICE, "invalid memory kind");
    keep.resize(count);
    if (count) {
        LABPSD_HIP(hipMemcpyAsync(keep.data(), a, count * sizeof(T), hipMemcpyDeviceToHost, ctx->stream));
        LABPSD_HIP(hipStreamSynchronize(ctx->stream));
    }
    return keep.data();
}

// ESTATE unless the global factor's panels for this solve precision were uploaded
static void require_panels(const Problem& P, int precision) {
    if (precision == LABPSD_MIXED && !P.factor->panels32.p)
        throw Error{LABPSD_ESTATE, "FP32 factor panels were not uploaded (precision mask)"};
    if (precision == LABPSD_FP64 && !P.factor->panels64.p)
        throw Error{LABPSD_ESTATE, "FP64 factor panels were not uploaded (precision mask)"};
}
}  // namespace labpsd

extern "C" {

const char* labpsd_last_error(void) { return labpsd::get_error(); }
const char* labpsd_version(void) { return "liblabpsd 0.1 (gfx950)"; }

labpsd_status labpsd_ctx_create(int device, void* stream, labpsd_ctx** out) {
    return guarded([&]() -> labpsd_status {
        LABPSD_REQUIRE(out != nullptr, "out is NULL");
        *out = nullptr;
        int count = 0;
        LABPSD_HIP(hipGetDeviceCount(&count));
        LABPSD_REQUIRE(device >= 0 && device < count, "device index out of range");
        LABPSD_HIP(hipSetDevice(device));
        auto c = std::make_unique<labpsd_ctx>();
        c->device = device;
        c->stream = (hipStream_t)stream;
        hipDeviceProp_t prop;
        LABPSD_HIP(hipGetDeviceProperties(&prop, device));
        c->cu_count = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
        noalloc_setup(device);
        *out = c.release();
        return LABPSD_OK;
    });
}

void labpsd_ctx_destroy(labpsd_ctx* ctx) { delete ctx; }

labpsd_status labpsd_ctx_set_stream(labpsd_ctx* ctx, void* stream) {
    return guarded([&]() -> labpsd_status {
        LABPSD_REQUIRE(ctx != nullptr, "ctx is NULL");
        ctx->stream = (hipStream_t)stream;
        return LABPSD_OK;
    });
}

// Validate a host CSR pencil and build the problem (shared by the real and the Hermitian
// entry points).
static std::unique_ptr<labpsd_problem> make_problem(labpsd_ctx* ctx, int64_t n, int64_t nnz, const int64_t* rowptr,
                                                    const int32_t* col, const double* h_val, const double* s_val) {
    LABPSD_REQUIRE(rowptr[0] == 0 && rowptr[n] == nnz, "rowptr does not span [0, nnz]");
    for (int64_t i = 0; i < n; ++i) {
        LABPSD_REQUIRE(rowptr[i + 1] > rowptr[i], "empty row " + std::to_string(i));
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            LABPSD_REQUIRE(col[e] >= 0 && col[e] < n, "column index out of range in row " + std::to_string(i));
            if (e > rowptr[i])
                LABPSD_REQUIRE(col[e] > col[e - 1], "columns not strictly increasing in row " + std::to_string(i));
        }
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            const int32_t j = col[e];
            const int32_t* b0 = col + rowptr[j];
            const int32_t* b1 = col + rowptr[j + 1];
            LABPSD_REQUIRE(std::binary_search(b0, b1, (int32_t)i),
                           "pattern not structurally symmetric at (" + std::to_string(i) + "," +
                               std::to_string(j) + ")");
        }
    auto p = std::make_unique<labpsd_problem>();
    p->ctx = ctx;
    p->n = n;
    p->nnz = nnz;
    p->csr.n = n;
    p->csr.nnz = nnz;
    p->csr.rowptr.assign(rowptr, rowptr + n + 1);
    p->csr.col.assign(col, col + nnz);
    p->h_val.assign(h_val, h_val + nnz);
    p->s_val.assign(s_val, s_val + nnz);
    build_sell(p->sell, p->csr, h_val, s_val, ctx->stream);
    return p;
}

labpsd_status labpsd_problem_create(labpsd_ctx* ctx, int64_t n, int64_t nnz, const int64_t* rowptr_in,
                                    const int32_t* col_in, const double* h_in, const double* s_in,
                                    labpsd_mem where, labpsd_problem** out) {
    return guarded([&]() -> labpsd_status {
        LABPSD_REQUIRE(ctx && out && rowptr_in && col_in && h_in && s_in, "NULL argument");
        *out = nullptr;
        LABPSD_REQUIRE(n >= 1 && n < (int64_t)INT32_MAX, "n out of range");
        LABPSD_REQUIRE(nnz >= n, "nnz smaller than n");
        LABPSD_HIP(hipSetDevice(ctx->device));
        std::vector<int64_t> rp_keep;
        const int64_t* rowptr = host_view(ctx, rowptr_in, (size_t)n + 1, where, rp_keep);
        LABPSD_REQUIRE(rowptr[n] == nnz, "rowptr does not span [0, nnz]");
        std::vector<int32_t> col_keep;
        std::vector<double> h_keep, s_keep;
        const int32_t* col = host_view(ctx, col_in, (size_t)nnz, where, col_keep);
        const double* h_val = host_view(ctx, h_in, (size_t)nnz, where, h_keep);
        const double* s_val = host_view(ctx, s_in, (size_t)nnz, where, s_keep);
        *out = make_problem(ctx, n, nnz, rowptr, col, h_val, s_val).release();
        return LABPSD_OK;
    });
}

labpsd_status labpsd_problem_create_hermitian(labpsd_ctx* ctx, int64_t n, int64_t nnz, const int64_t* rowptr,
                                              const int32_t* col, const double* h_re, const double* h_im,
                                              const double* s_re, const double* s_im, labpsd_problem** out) {
    return guarded([&]() -> labpsd_status {
        LABPSD_REQUIRE(ctx && out && rowptr && col && h_re && h_im && s_re && s_im, "NULL argument");
        *out = nullptr;
        LABPSD_REQUIRE(n >= 1 && 2 * n < (int64_t)INT32_MAX, "n out of range");
        LABPSD_REQUIRE(nnz >= n && rowptr[0] == 0 && rowptr[n] == nnz, "rowptr does not span [0, nnz]");
        // Hermitian values: the (j, i) entry is the conjugate of (i, j)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
                const int32_t j = col[e];
                LABPSD_REQUIRE(j >= 0 && j < n, "column index out of range in row " + std::to_string(i));
                const int32_t* b0 = col + rowptr[j];
                const int32_t* b1 = col + rowptr[j + 1];
                const int32_t* f = std::lower_bound(b0, b1, (int32_t)i);
                LABPSD_REQUIRE(f != b1 && *f == (int32_t)i, "pattern not structurally symmetric");
                const int64_t t = rowptr[j] + (f - b0);
                const double tol = 1e-13 * (std::fabs(h_re[e]) + std::fabs(h_im[e]) + std::fabs(s_re[e]) +
                                            std::fabs(s_im[e])) + 1e-300;
                LABPSD_REQUIRE(std::fabs(h_re[t] - h_re[e]) <= tol && std::fabs(h_im[t] + h_im[e]) <= tol &&
                                   std::fabs(s_re[t] - s_re[e]) <= tol && std::fabs(s_im[t] + s_im[e]) <= tol,
                               "H or S is not Hermitian at (" + std::to_string(i) + "," + std::to_string(j) + ")");
            }
        LABPSD_HIP(hipSetDevice(ctx->device));
        std::vector<int64_t> rp2;
        std::vector<int32_t> col2;
        std::vector<double> h2, s2;
        embed_hermitian(n, nnz, rowptr, col, h_re, h_im, rp2, col2, h2);
        embed_hermitian(n, nnz, rowptr, col, s_re, s_im, rp2, col2, s2);
        auto p = make_problem(ctx, 2 * n, 4 * nnz, rp2.data(), col2.data(), h2.data(), s2.data());
        p->hermitian = true;
        p->nc = n;
        *out = p.release();
        return LABPSD_OK;
    });
}

labpsd_status labpsd_problem_update_h(labpsd_problem* p, const double* h_in, labpsd_mem where) {
    return guarded([&]() -> labpsd_status {
        LABPSD_REQUIRE(p && h_in, "NULL argument");
        LABPSD_REQUIRE(!p->hermitian, "Hermitian problem: use labpsd_problem_update_h_hermitian");
        LABPSD_HIP(hipSetDevice(p->ctx->device));
        std::vector<double> keep;
        const double* h_val = host_view(p->ctx, h_in, (size_t)p->nnz, where, keep);
        p->h_val.assign(h_val, h_val + p->nnz);
        refresh_sell_h(p->sell, h_val, p->ctx->stream);
        return LABPSD_OK;
    });
}

labpsd_status labpsd_problem_update_h_hermitian(labpsd_problem* p, const double* h_re, const double* h_im) {
    return guarded([&]() -> labpsd_status {
        LABPSD_REQUIRE(p && h_re && h_im, "NULL argument");
        LABPSD_REQUIRE(p->hermitian, "not a Hermitian problem");
        const int64_t nc = p->nc, nnz = p->nnz / 4;
        // the complex pattern is every other entry of the even rows of the embedding
        std::vector<int64_t> rp(nc + 1);
        std::vector<int32_t> col(nnz);
        for (int64_t i = 0; i < nc; ++i) {
            rp[i + 1] = rp[i] + (p->csr.rowptr[2 * i + 1] - p->csr.rowptr[2 * i]) / 2;
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
                col[e] = p->csr.col[p->csr.rowptr[2 * i] + 2 * (e - rp[i])] / 2;
        }
        std::vector<int64_t> rp2;
        std::vector<int32_t> col2;
        std::vector<double> h2;
        embed_hermitian(nc, nnz, rp.data(), col.data(), h_re, h_im, rp2, col2, h2);
        LABPSD_HIP(hipSetDevice(p->ctx->device));
        p->h_val = h2;
        refresh_sell_h(p->sell, h2.data(), p->ctx->stream);
        return LABPSD_OK;
    });
}

void labpsd_problem_destroy(labpsd_problem* p) { delete p; }

int64_t labpsd_problem_n(const labpsd_problem* p) { return p ? p->n : -1; }

labpsd_status labpsd_set_global_precond(labpsd_problem* p, double eps_bar, const double* coords,
                                        unsigned precisions) {
    return guarded([&]() -> labpsd_status {
        LABPSD_REQUIRE(p != nullptr, "problem is NULL");
        LABPSD_REQUIRE(std::isfinite(eps_bar), "eps_bar must be finite");
        LABPSD_REQUIRE((precisions & ~(unsigned)(LABPSD_PANELS_FP64 | LABPSD_PANELS_FP32 | LABPSD_FACTOR_FP32 |
                                                 LABPSD_APPLY_LEVELS)) == 0,
                       "precision mask has unknown bits");
        const bool single = (precisions & LABPSD_FACTOR_FP32) != 0;
        const unsigned sel = precisions & (unsigned)(LABPSD_PANELS_FP64 | LABPSD_PANELS_FP32);
        const unsigned panels = sel ? sel : (LABPSD_PANELS_FP64 | LABPSD_PANELS_FP32);
        LABPSD_HIP(hipSetDevice(p->ctx->device));
        std::vector<double> kval(p->nnz);
        for (int64_t e = 0; e < p->nnz; ++e) kval[e] = p->h_val[e] - eps_bar * p->s_val[e];
        HostFactor F;
        std::string msg;
        std::vector<double> c2;
        if (p->hermitian && coords) {   // both real dofs of a complex one sit at its point
            c2.resize(6 * (size_t)p->nc);
            for (int64_t i = 0; i < p->nc; ++i)
                for (int d = 0; d < 3; ++d) c2[6 * i + d] = c2[6 * i + 3 + d] = coords[3 * i + d];
            coords = c2.data();
        }
        const int rc = factorize(p->csr, kval.data(), coords, F, msg, single);
        if (rc == -4) throw Error{LABPSD_ENOTSPD, msg};
        if (rc != 0) throw Error{LABPSD_EINVAL, msg};
        const double t0 = wall();
        upload_factor(*p, F, eps_bar, panels);
        if (precisions & LABPSD_APPLY_LEVELS) p->factor->use_sweep = false;
        // the factor is of H_loc - eps_bar S; the nonlocal term enters through SMW
        if (p->nl.k) nonlocal_smw_setup(*p);
        p->factor->info.t_upload_s = wall() - t0;
        return LABPSD_OK;
    });
}

labpsd_status labpsd_set_local_precond(labpsd_problem* p, double tau1, double tau2, double eta,
                                       int max_inner, labpsd_precond_mode mode) {
    return guarded([&]() -> labpsd_status {
        LABPSD_REQUIRE(p != nullptr, "problem is NULL");
        LABPSD_REQUIRE(tau1 >= 0 && tau2 >= 0 && eta > 0 && max_inner >= 0, "invalid local parameters");
        LABPSD_REQUIRE(mode == LABPSD_HYBRID || mode == LABPSD_GLOBAL_ONLY || mode == LABPSD_LOCAL_ONLY,
                       "invalid mode");
        p->local.tau1 = tau1;
        p->local.tau2 = tau2;
        p->local.eta = eta;
        p->local.max_inner = max_inner;
        p->local.mode = mode;
        return LABPSD_OK;
    });
}

labpsd_status labpsd_set_refine_method(labpsd_problem* p, int method) {
    return guarded([&]() -> labpsd_status {
        LABPSD_REQUIRE(p != nullptr, "problem is NULL");
        LABPSD_REQUIRE(method == LABPSD_REFINE_MINRES || method == LABPSD_REFINE_ONESTEP,
                       "invalid refinement method");
        p->local.method = method;
        return LABPSD_OK;
    });
}

labpsd_status labpsd_get_factor_info(const labpsd_problem* p, labpsd_factor_info* info) {
    return guarded([&]() -> labpsd_status {
        LABPSD_REQUIRE(p && info, "NULL argument");
        if (!p->factor) throw Error{LABPSD_ESTATE, "no global preconditioner set"};
        *info = p->factor->info;
        return LABPSD_OK;
    });
}

labpsd_status labpsd_solve(labpsd_problem* p, const labpsd_solve_params* prm, const double* X0,
                           const double* E0, labpsd_mem in_where, double* lambda, double* X,
                           double* res_hist, double* ritz_hist, int* n_hist, labpsd_mem out_where, labpsd_stats* stats) {
    return guarded([&]() -> labpsd_status {
        LABPSD_REQUIRE(p && prm && lambda && X, "NULL argument");
        LABPSD_REQUIRE(!p->hermitian, "Hermitian problem: use labpsd_solve_hermitian");
        if (!p->factor) throw Error{LABPSD_ESTATE, "labpsd_set_global_precond must come first"};
        require_panels(*p, prm->precision);
        LABPSD_REQUIRE(prm->nev >= 1 && prm->m0 >= 0, "nev must be >= 1 and m0 >= 0");
        LABPSD_REQUIRE((int64_t)(2 * prm->nev + prm->m0) <= p->n, "n < 2 nev + m0");
        LABPSD_REQUIRE(prm->nev + prm->m0 + prm->nev <= kRRMax, "block too wide");
        LABPSD_REQUIRE(prm->tol > 0 && prm->max_outer >= 1 && prm->refresh_every >= 1,
                       "tol, max_outer and refresh_every must be positive");
        LABPSD_REQUIRE(prm->precision == LABPSD_FP64 || prm->precision == LABPSD_MIXED,
                       "invalid precision");
        LABPSD_HIP(hipSetDevice(p->ctx->device));
        return run_solve(*p, *prm, X0, E0, in_where, lambda, X, res_hist, ritz_hist, n_hist, out_where, stats,
                         p->ctx->stream);
    });
}

// The complex Hermitian pencil through its real embedding: LABPSD on (R(H), R(S)) with
// 2 nev pairs and 2 m0 guards (every complex pair appears twice), then the complex pairs:
// Z = the 2 nev real eigenvectors read as complex vectors spans the nev-dimensional
// complex invariant subspace twice over; a Rayleigh-Ritz step on span(Z) with the
// rank-revealing cut keeps it once.  The O(n) parts run on the device: the products HZ,
// SZ, the Gram matrices Re(Z^H Y) = U^T R(Y) and Im(Z^H Y) = U^T J^T R(Y) (U = R(Z), J the
// real form of i; the imaginary parts are antisymmetric, so their upper triangles
// suffice), and X = Z C = [U, J U] [Re C; Im C] on the block-update kernel.  The
// 2 nev x 2 nev Hermitian eigenproblems run on the host (cyclic Jacobi), as the paper
// solves its reduced problem with ZHEGVX.
labpsd_status labpsd_solve_hermitian(labpsd_problem* p, const labpsd_solve_params* prm, const double* X0,
                                     const double* E0, labpsd_mem in_where, double* lambda, double* X,
                                     double* res_hist, double* ritz_hist, int* n_hist, labpsd_mem out_where,
                                     labpsd_stats* stats) {
    return guarded([&]() -> labpsd_status {
        LABPSD_REQUIRE(p && prm && lambda && X, "NULL argument");
        LABPSD_REQUIRE(p->hermitian, "not a Hermitian problem (labpsd_problem_create_hermitian)");
        if (!p->factor) throw Error{LABPSD_ESTATE, "labpsd_set_global_precond must come first"};
        require_panels(*p, prm->precision);
        const int nev = prm->nev, m0 = prm->m0, b = nev + m0;
        LABPSD_REQUIRE(nev >= 1 && m0 >= 0, "nev must be >= 1 and m0 >= 0");
        LABPSD_REQUIRE((int64_t)(2 * nev + m0) <= p->nc, "n < 2 nev + m0");
        LABPSD_REQUIRE(4 * nev + 2 * m0 <= kRRMax, "block too wide");
        LABPSD_REQUIRE(prm->tol > 0 && prm->max_outer >= 1 && prm->refresh_every >= 1,
                       "tol, max_outer and refresh_every must be positive");
        LABPSD_HIP(hipSetDevice(p->ctx->device));
        hipStream_t s = p->ctx->stream;
        const int64_t nc = p->nc, n2 = 2 * nc;
        const int kk = 2 * nev, br = 2 * b;
        labpsd_solve_params pr = *prm;
        pr.nev = kk;
        pr.m0 = 2 * m0;
        // start block: R(x_j) and R(i x_j) for the b complex columns of X0
        DBuf<double> start, lam_r, U, HU, SU, JH, JS, GH, GS, GHi, GSi, Zc, Wd, o1, o2;
        const double* X0r = nullptr;
        if (X0) {
            start.alloc((size_t)n2 * br);
            LABPSD_HIP(hipMemcpyAsync(start.p, X0, (size_t)n2 * b * sizeof(double),
                                      in_where == LABPSD_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
            launch_apply_j(nc, b, start.p, n2, start.p + (size_t)n2 * b, n2, false, s);
            X0r = start.p;
        }
        std::vector<double> E0r;
        if (E0) {
            E0r.resize(br);
            for (int j = 0; j < b; ++j) E0r[2 * j] = E0r[2 * j + 1] = E0[j];
        }
        lam_r.alloc(kk);
        U.alloc((size_t)n2 * kk);
        const labpsd_status rc = run_solve(*p, pr, X0r, E0 ? E0r.data() : nullptr, LABPSD_MEM_DEVICE, lam_r.p, U.p,
                                           res_hist, ritz_hist, n_hist, LABPSD_MEM_HOST, stats, s);
        // products and the complex Gram matrices of span(Z)
        HU.alloc((size_t)n2 * kk);
        SU.alloc((size_t)n2 * kk);
        JH.alloc((size_t)n2 * kk);
        JS.alloc((size_t)n2 * kk);
        launch_spmm_hs(p->sell, U.p, n2, kk, HU.p, SU.p, n2, s);
        launch_apply_j(nc, kk, HU.p, n2, JH.p, n2, true, s);
        launch_apply_j(nc, kk, SU.p, n2, JS.p, n2, true, s);
        GH.alloc((size_t)kk * kk);
        GS.alloc((size_t)kk * kk);
        GHi.alloc((size_t)kk * kk);
        GSi.alloc((size_t)kk * kk);
        p->ctx->scratch.alloc(gram_ws_doubles(n2, kk, p->ctx->cu_count) + 1);
        launch_gram(n2, kk, U.p, HU.p, SU.p, n2, GH.p, GS.p, kk, p->ctx->scratch.p, p->ctx->cu_count, s);
        LABPSD_HIP(hipStreamSynchronize(s));
        launch_gram(n2, kk, U.p, JH.p, JS.p, n2, GHi.p, GSi.p, kk, p->ctx->scratch.p, p->ctx->cu_count, s);
        std::vector<double> hr((size_t)kk * kk), sr(hr.size()), hi(hr.size()), si(hr.size());
        LABPSD_HIP(hipMemcpyAsync(hr.data(), GH.p, hr.size() * 8, hipMemcpyDeviceToHost, s));
        LABPSD_HIP(hipMemcpyAsync(sr.data(), GS.p, sr.size() * 8, hipMemcpyDeviceToHost, s));
        LABPSD_HIP(hipMemcpyAsync(hi.data(), GHi.p, hi.size() * 8, hipMemcpyDeviceToHost, s));
        LABPSD_HIP(hipMemcpyAsync(si.data(), GSi.p, si.size() * 8, hipMemcpyDeviceToHost, s));
        LABPSD_HIP(hipStreamSynchronize(s));
        // the Gram kernel mirrors its upper triangle; the imaginary parts are antisymmetric
        for (int j = 0; j < kk; ++j)
            for (int i = 0; i <= j; ++i) {
                const size_t u = (size_t)i + (size_t)j * kk, l = (size_t)j + (size_t)i * kk;
                hi[l] = -hi[u];
                si[l] = -si[u];
                if (i == j) hi[u] = si[u] = 0.0;
            }
        // S-orthonormal basis of the complex span: the nev dominant eigenvectors of Z^H S Z
        std::vector<double> Vr, Vi;
        hermitian_jacobi(kk, sr, si, Vr, Vi);
        std::vector<int> ord(kk);
        for (int i = 0; i < kk; ++i) ord[i] = i;
        std::sort(ord.begin(), ord.end(), [&](int a, int c) { return sr[(size_t)a * kk + a] > sr[(size_t)c * kk + c]; });
        const double mu_min = sr[(size_t)ord[nev - 1] * kk + ord[nev - 1]];
        if (!(mu_min > 1e-8 * sr[(size_t)ord[0] * kk + ord[0]]))
            throw Error{LABPSD_ERANK, "the real eigenvectors span fewer than nev complex directions"};
        std::vector<double> Tr((size_t)kk * nev), Ti(Tr.size());
        for (int c = 0; c < nev; ++c) {
            const int q = ord[c];
            const double sc = 1.0 / std::sqrt(sr[(size_t)q * kk + q]);
            for (int i = 0; i < kk; ++i) {
                Tr[i + (size_t)c * kk] = Vr[i + (size_t)q * kk] * sc;
                Ti[i + (size_t)c * kk] = Vi[i + (size_t)q * kk] * sc;
            }
        }
        // reduced Hermitian matrix T^H (Z^H H Z) T and its eigenpairs
        std::vector<double> Mr((size_t)kk * nev), Mi(Mr.size()), Ar((size_t)nev * nev), Ai(Ar.size());
        for (int c = 0; c < nev; ++c)
            for (int i = 0; i < kk; ++i) {
                double a = 0.0, bb = 0.0;
                for (int k2 = 0; k2 < kk; ++k2) {
                    const double gr = hr[i + (size_t)k2 * kk], gi = hi[i + (size_t)k2 * kk];
                    const double tr = Tr[k2 + (size_t)c * kk], ti = Ti[k2 + (size_t)c * kk];
                    a += gr * tr - gi * ti;
                    bb += gr * ti + gi * tr;
                }
                Mr[i + (size_t)c * kk] = a;
                Mi[i + (size_t)c * kk] = bb;
            }
        for (int c = 0; c < nev; ++c)
            for (int r = 0; r < nev; ++r) {
                double a = 0.0, bb = 0.0;
                for (int i = 0; i < kk; ++i) {   // conj(T[i, r]) * M[i, c]
                    const double tr = Tr[i + (size_t)r * kk], ti = Ti[i + (size_t)r * kk];
                    const double mr = Mr[i + (size_t)c * kk], mi = Mi[i + (size_t)c * kk];
                    a += tr * mr + ti * mi;
                    bb += tr * mi - ti * mr;
                }
                Ar[r + (size_t)c * nev] = a;
                Ai[r + (size_t)c * nev] = bb;
            }
        for (int c = 0; c < nev; ++c)
            for (int r = 0; r < c; ++r) {   // exact Hermitian symmetry
                const size_t u = r + (size_t)c * nev, l = c + (size_t)r * nev;
                const double ar = 0.5 * (Ar[u] + Ar[l]), ai = 0.5 * (Ai[u] - Ai[l]);
                Ar[u] = Ar[l] = ar;
                Ai[u] = ai;
                Ai[l] = -ai;
            }
        std::vector<double> Wr, Wi;
        hermitian_jacobi(nev, Ar, Ai, Wr, Wi);
        std::vector<int> o2i(nev);
        for (int i = 0; i < nev; ++i) o2i[i] = i;
        std::sort(o2i.begin(), o2i.end(), [&](int a, int c) { return Ar[(size_t)a * nev + a] < Ar[(size_t)c * nev + c]; });
        std::vector<double> lam_h(nev), W2((size_t)2 * kk * nev);
        for (int c = 0; c < nev; ++c) {
            const int q = o2i[c];
            lam_h[c] = Ar[(size_t)q * nev + q];
            // C[:, c] = T W[:, q]; W2 = [Re C ; Im C] (2 kk x nev)
            for (int i = 0; i < kk; ++i) {
                double a = 0.0, bb = 0.0;
                for (int r = 0; r < nev; ++r) {
                    const double tr = Tr[i + (size_t)r * kk], ti = Ti[i + (size_t)r * kk];
                    const double wr = Wr[r + (size_t)q * nev], wi = Wi[r + (size_t)q * nev];
                    a += tr * wr - ti * wi;
                    bb += tr * wi + ti * wr;
                }
                W2[i + (size_t)c * 2 * kk] = a;
                W2[kk + i + (size_t)c * 2 * kk] = bb;
            }
        }
        // X = [U, J U] [Re C ; Im C]
        Zc.alloc((size_t)n2 * 2 * kk);
        Wd.alloc(W2.size());
        o1.alloc((size_t)n2 * nev);
        o2.alloc((size_t)n2 * nev);
        LABPSD_HIP(hipMemcpyAsync(Zc.p, U.p, (size_t)n2 * kk * 8, hipMemcpyDeviceToDevice, s));
        launch_apply_j(nc, kk, U.p, n2, Zc.p + (size_t)n2 * kk, n2, false, s);
        LABPSD_HIP(hipMemcpyAsync(Wd.p, W2.data(), W2.size() * 8, hipMemcpyHostToDevice, s));
        double* Xd = out_where == LABPSD_MEM_DEVICE ? X : o1.p;
        launch_block_update(n2, 2 * kk, nev, Zc.p, Zc.p, Zc.p, n2, Wd.p, 2 * kk, Xd, o2.p, o2.p, n2, s);
        if (out_where == LABPSD_MEM_DEVICE) {
            LABPSD_HIP(hipMemcpyAsync(lambda, lam_h.data(), nev * 8, hipMemcpyHostToDevice, s));
        } else {
            LABPSD_HIP(hipMemcpyAsync(X, o1.p, (size_t)n2 * nev * 8, hipMemcpyDeviceToHost, s));
            std::memcpy(lambda, lam_h.data(), nev * 8);
        }
        LABPSD_HIP(hipStreamSynchronize(s));
        return rc;
    });
}

// ------------------------------------------------------------------ steps

labpsd_status labpsd_spmm(labpsd_problem* p, const double* X, int64_t ldx, int w, double* YH,
                          double* YS, int64_t ldy) {
    return guarded([&]() -> labpsd_status {
        LABPSD_REQUIRE(p && X && YH && YS, "NULL argument");
        LABPSD_REQUIRE(w >= 0 && ldx >= p->n && ldy >= p->n, "bad width or leading dimension");
        launch_spmm_hs(p->sell, X, ldx, w, YH, YS, ldy, p->ctx->stream, p->nl.k ? &p->nl : nullptr);
        return LABPSD_OK;
    });
}

labpsd_status labpsd_spmm_shifted(labpsd_problem* p, int precision, const void* X, int64_t ldx,
                                  int w, const double* shift, void* Y, int64_t ldy) {
    return guarded([&]() -> labpsd_status {
        LABPSD_REQUIRE(p && X && Y && shift, "NULL argument");
        LABPSD_REQUIRE(w >= 0 && ldx >= p->n && ldy >= p->n, "bad width or leading dimension");
        if (precision == LABPSD_MIXED)
            launch_spmm_shift<float>(p->sell, (const float*)X, ldx, w, shift, (float*)Y, ldy, p->ctx->stream,
                                     p->nl.k ? &p->nl : nullptr);
        else if (precision == LABPSD_FP64)
            launch_spmm_shift<double>(p->sell, (const double*)X, ldx, w, shift, (double*)Y, ldy,
                                      p->ctx->stream, p->nl.k ? &p->nl : nullptr);
        else
            throw Error{LABPSD_EINVAL, "invalid precision"};
        return LABPSD_OK;
    });
}

labpsd_status labpsd_residual(labpsd_ctx* ctx, int64_t n, int m, const double* PsiH,
                              const double* PsiS, int64_t ld, const double* E, double sigma0,
                              double* R, int64_t ldr, double* res, double* rnorm) {
    return guarded([&]() -> labpsd_status {
        LABPSD_REQUIRE(ctx && PsiH && PsiS && E && R && res && rnorm, "NULL argument");
        LABPSD_REQUIRE(n >= 1 && m >= 0 && ld >= n && ldr >= n, "bad sizes");
        const int nblk = residual_blocks(n);
        ctx->scratch.alloc((size_t)nblk * m * 2 + 1);
        launch_residual(n, m, PsiH, PsiS, ld, E, sigma0, R, ldr, ctx->scratch.p, nblk, ctx->stream);
        launch_residual_finish(m, ctx->scratch.p, nblk, res, rnorm, ctx->stream);
        return LABPSD_OK;
    });
}

labpsd_status labpsd_precond_apply(labpsd_problem* p, int precision, const double* R, int64_t ldr,
                                   int ncols, double* Pout, int64_t ldp) {
    return guarded([&]() -> labpsd_status {
        LABPSD_REQUIRE(p && R && Pout, "NULL argument");
        if (!p->factor) throw Error{LABPSD_ESTATE, "no global preconditioner set"};
        LABPSD_REQUIRE(ncols >= 0 && ldr >= p->n && ldp >= p->n, "bad sizes");
        require_panels(*p, precision);
        if (ncols == 0) return LABPSD_OK;
        hipStream_t s = p->ctx->stream;
        const int64_t n = p->n;
        if (precision == LABPSD_MIXED) {
            p->ws32.alloc(3 * (size_t)n * ncols);
            float* Y = p->ws32.p;
            launch_cast_to_rm<double, float>(n, ncols, R, ldr, nullptr, -1.0, Y, s);
            launch_precond_solve<float>(*p->factor, Y, Y + n * ncols, Y + 2 * n * ncols, n, ncols, s,
                                        p->nl.k ? &p->nl : nullptr);
            launch_cast_from_rm<float, double>(n, ncols, Y + 2 * n * ncols, 1.0, Pout, ldp, s);
        } else if (precision == LABPSD_FP64) {
            p->red.alloc(3 * (size_t)n * ncols);
            double* Y = p->red.p;
            launch_cast_to_rm<double, double>(n, ncols, R, ldr, nullptr, -1.0, Y, s);
            launch_precond_solve<double>(*p->factor, Y, Y + n * ncols, Y + 2 * n * ncols, n, ncols, s,
                                         p->nl.k ? &p->nl : nullptr);
            launch_cast_from_rm<double, double>(n, ncols, Y + 2 * n * ncols, 1.0, Pout, ldp, s);
        } else {
            throw Error{LABPSD_EINVAL, "invalid precision"};
        }
        // the workspace is reused by the next call: finish before returning it
        LABPSD_HIP(hipStreamSynchronize(s));
        check_precond_sweep(*p->factor, s);
        return LABPSD_OK;
    });
}

labpsd_status labpsd_local_refine(labpsd_problem* p, int precision, const double* R, int64_t ldr,
                                  double* Pm, int64_t ldp, int q, const int32_t* cols,
                                  const double* shift, double eta, int max_inner, int32_t* its) {
    return guarded([&]() -> labpsd_status {
        LABPSD_REQUIRE(p && R && Pm && cols && shift && its, "NULL argument");
        LABPSD_REQUIRE(q >= 0 && ldr >= p->n && ldp >= p->n && eta > 0 && max_inner >= 0, "bad arguments");
        if (q == 0) return LABPSD_OK;
        if (precision == LABPSD_MIXED)
            local_refine_impl<float>(p, p->ws32, R, ldr, Pm, ldp, q, cols, shift, eta, max_inner, its);
        else if (precision == LABPSD_FP64)
            local_refine_impl<double>(p, p->red, R, ldr, Pm, ldp, q, cols, shift, eta, max_inner, its);
        else
            throw Error{LABPSD_EINVAL, "invalid precision"};
        return LABPSD_OK;
    });
}

labpsd_status labpsd_gram(labpsd_ctx* ctx, int64_t n, int k, const double* Z, const double* ZH,
                          const double* ZS, int64_t ldz, double* HR, double* SR, int64_t ldr) {
    return guarded([&]() -> labpsd_status {
        LABPSD_REQUIRE(ctx && Z && ZH && ZS && HR && SR, "NULL argument");
        LABPSD_REQUIRE(n >= 1 && k >= 0 && ldz >= n && ldr >= k, "bad sizes");
        ctx->scratch.alloc(gram_ws_doubles(n, k, ctx->cu_count) + 1);
        launch_gram(n, k, Z, ZH, ZS, ldz, HR, SR, ldr, ctx->scratch.p, ctx->cu_count, ctx->stream);
        LABPSD_HIP(hipStreamSynchronize(ctx->stream));
        return LABPSD_OK;
    });
}

labpsd_status labpsd_rayleigh_ritz(labpsd_ctx* ctx, int k, int nwant, const double* HR,
                                   const double* SR, int64_t ldr, double* gamma, double* W,
                                   int64_t ldw, int32_t* info) {
    return guarded([&]() -> labpsd_status {
        LABPSD_REQUIRE(ctx && HR && SR && gamma && W && info, "NULL argument");
        LABPSD_REQUIRE(k >= 1 && nwant >= 1 && nwant <= k && ldr >= k && ldw >= k, "bad sizes");
        ctx->rr_ws.alloc(rr_ws_bytes(k));
        launch_rayleigh_ritz(k, nwant, HR, SR, ldr, gamma, W, ldw, info, ctx->rr_ws.p, ctx->stream);
        LABPSD_HIP(hipStreamSynchronize(ctx->stream));
        return LABPSD_OK;
    });
}

labpsd_status labpsd_block_update(labpsd_ctx* ctx, int64_t n, int k, int b, const double* Z,
                                  const double* ZH, const double* ZS, int64_t ldz, const double* W,
                                  int64_t ldw, double* Psi, double* PsiH, double* PsiS, int64_t ldo) {
    return guarded([&]() -> labpsd_status {
        LABPSD_REQUIRE(ctx && Z && ZH && ZS && W && Psi && PsiH && PsiS, "NULL argument");
        LABPSD_REQUIRE(n >= 1 && k >= 1 && b >= 1 && ldz >= n && ldw >= k && ldo >= n, "bad sizes");
        launch_block_update(n, k, b, Z, ZH, ZS, ldz, W, ldw, Psi, PsiH, PsiS, ldo, ctx->stream);
        return LABPSD_OK;
    });
}

}  // extern "C"
