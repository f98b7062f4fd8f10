// Host nested-dissection ordering and multifrontal supernodal Cholesky of
// K = H - eps_bar S (the global preconditioner's factorisation, eq. (ldl)).
#include "factor.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <numeric>
#include <thread>

namespace labpsd {
namespace {

double wall() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

int host_threads() {
    static int nt = [] {
        int h = (int)std::thread::hardware_concurrency();
        if (const char* e = std::getenv("LABPSD_HOST_THREADS")) h = std::atoi(e);
        return std::max(1, std::min(h, 16));
    }();
    return nt;
}

// Dynamic parallel loop over [0, n): each index runs exactly once.
void parallel_for(int64_t n, int nthreads, const std::function<void(int64_t)>& f) {
    if (n <= 0) return;
    nthreads = (int)std::min<int64_t>(nthreads, n);
    if (nthreads <= 1) {
        for (int64_t i = 0; i < n; ++i) f(i);
        return;
    }
    std::atomic<int64_t> next(0);
    auto work = [&]() {
        for (;;) {
            int64_t i = next.fetch_add(1);
            if (i >= n) break;
            f(i);
        }
    };
    std::vector<std::thread> th;
    th.reserve(nthreads - 1);
    for (int t = 1; t < nthreads; ++t) th.emplace_back(work);
    work();
    for (auto& t : th) t.join();
}

// ------------------------------------------------------------------ dissection

struct TreeNode {
    std::vector<int32_t> verts;
    std::vector<int> children;
};

class Dissector {
  public:
    Dissector(const HostCSR& A, const double* coords, std::vector<TreeNode>& nodes)
        : A_(A), xyz_(coords), nodes_(nodes), mark_(A.n, 0), side_(A.n, 0), level_(A.n, -1) {}

    std::vector<int> build(std::vector<int32_t>& V) {
        if ((int64_t)V.size() <= kLeaf) return {leaf(V)};
        const int label = ++label_;
        for (int32_t v : V) mark_[v] = label;
        bool ok = xyz_ ? split_coords(V) : false;
        if (!ok) split_bfs(V, label);
        // vertex separator: the layer of the smaller side adjacent to the other side
        std::vector<int32_t> SA, SB;
        for (int32_t v : V) {
            bool cross = false;
            for (int64_t e = A_.rowptr[v]; e < A_.rowptr[v + 1]; ++e) {
                int32_t u = A_.col[e];
                if (mark_[u] == label && side_[u] != side_[v]) { cross = true; break; }
            }
            if (cross) (side_[v] == 0 ? SA : SB).push_back(v);
        }
        const int8_t sep_side = SA.size() <= SB.size() ? 0 : 1;
        std::vector<int32_t>& S = sep_side == 0 ? SA : SB;
        std::vector<int32_t> Ap, Bp;
        for (int32_t v : S) side_[v] = 2;
        for (int32_t v : V) {
            if (side_[v] == 0) Ap.push_back(v);
            else if (side_[v] == 1) Bp.push_back(v);
        }
        if (Ap.empty() || Bp.empty()) {
            // no useful cut (tiny or degenerate set): keep it whole
            return {leaf(V)};
        }
        std::vector<int32_t> Ssave = S;
        std::vector<int> roots = build(Ap);
        std::vector<int> rb = build(Bp);
        roots.insert(roots.end(), rb.begin(), rb.end());
        if (Ssave.empty()) return roots;   // disconnected: a forest
        std::sort(Ssave.begin(), Ssave.end());
        TreeNode t;
        t.verts = std::move(Ssave);
        t.children = std::move(roots);
        nodes_.push_back(std::move(t));
        return {(int)nodes_.size() - 1};
    }

  private:
    static constexpr int64_t kLeaf = 128;

    int leaf(std::vector<int32_t>& V) {
        TreeNode t;
        t.verts = V;
        std::sort(t.verts.begin(), t.verts.end());
        nodes_.push_back(std::move(t));
        return (int)nodes_.size() - 1;
    }

    // median bisection along the widest coordinate
    bool split_coords(const std::vector<int32_t>& V) {
        double lo[3], hi[3];
        for (int d = 0; d < 3; ++d) { lo[d] = 1e300; hi[d] = -1e300; }
        for (int32_t v : V)
            for (int d = 0; d < 3; ++d) {
                double c = xyz_[3 * (int64_t)v + d];
                lo[d] = std::min(lo[d], c);
                hi[d] = std::max(hi[d], c);
            }
        int dim = 0;
        for (int d = 1; d < 3; ++d)
            if (hi[d] - lo[d] > hi[dim] - lo[dim]) dim = d;
        if (!(hi[dim] > lo[dim])) return false;
        std::vector<double> c(V.size());
        for (size_t i = 0; i < V.size(); ++i) c[i] = xyz_[3 * (int64_t)V[i] + dim];
        std::nth_element(c.begin(), c.begin() + c.size() / 2, c.end());
        double thr = c[c.size() / 2];
        if (!(thr > lo[dim])) {
            // everything at or below the median shares the minimum: cut just above it
            double nxt = 1e300;
            for (int32_t v : V) {
                double x = xyz_[3 * (int64_t)v + dim];
                if (x > lo[dim]) nxt = std::min(nxt, x);
            }
            thr = nxt;
        }
        for (int32_t v : V) side_[v] = xyz_[3 * (int64_t)v + dim] < thr ? 0 : 1;
        return true;
    }

    // breadth-first level structure from a pseudo-peripheral vertex, cut at the
    // level holding the median; an unreached remainder (disconnected set) is side 1
    void split_bfs(const std::vector<int32_t>& V, int label) {
        int32_t start = V[0];
        std::vector<int32_t> order;
        int depth = 0, prev_depth = -1;
        for (int pass = 0; pass < 4 && depth > prev_depth; ++pass) {
            prev_depth = depth;
            depth = bfs(start, label, order);
            start = order.back();
        }
        depth = bfs(start, label, order);
        if ((int64_t)order.size() < (int64_t)V.size()) {
            for (int32_t v : V) side_[v] = 1;
            for (int32_t v : order) side_[v] = 0;
            return;
        }
        int64_t half = (int64_t)V.size() / 2, cum = 0;
        int cut = 0;
        for (size_t i = 0; i < order.size(); ++i) {
            ++cum;
            if (cum >= half) { cut = level_[order[i]]; break; }
        }
        for (int32_t v : V) side_[v] = level_[v] <= cut ? 0 : 1;
        (void)depth;
    }

    int bfs(int32_t s, int label, std::vector<int32_t>& order) {
        const int tag = ++visit_tag_;
        order.clear();
        order.push_back(s);
        visit_[s] = tag;
        level_[s] = 0;
        int depth = 0;
        for (size_t head = 0; head < order.size(); ++head) {
            const int32_t v = order[head];
            for (int64_t e = A_.rowptr[v]; e < A_.rowptr[v + 1]; ++e) {
                const int32_t u = A_.col[e];
                if (mark_[u] != label || visit_[u] == tag) continue;
                visit_[u] = tag;
                level_[u] = level_[v] + 1;
                depth = std::max(depth, level_[u]);
                order.push_back(u);
            }
        }
        return depth;
    }

    const HostCSR& A_;
    const double* xyz_;
    std::vector<TreeNode>& nodes_;
    std::vector<int> mark_;
    std::vector<int8_t> side_;
    std::vector<int> level_;
    std::vector<int> visit_ = std::vector<int>(A_.n, 0);
    int visit_tag_ = 0;
    int label_ = 0;
};

// ------------------------------------------------------------------ dense kernels

// C[i, j] -= sum_p A[i, p] * A[j, p] for rows i in [r0, nf), i >= j, columns j in
// [j0, j1).  A is the packed panel: rows [a0, nf) in blocks of 8, each block
// kw x 8 contiguous (block-major), so A[i, p] = Ap[((i - a0) / 8) * kw * 8 + p * 8 + (i - a0) % 8].
template <typename T>
void syrk_cols(T* F, int64_t ld, int64_t nf, const T* Ap, int64_t a0, int kw, int64_t j0,
               int64_t j1) {
    constexpr int MR = 8, NR = 4;
    T bj[64 * NR];
    for (int64_t j = j0; j < j1; j += NR) {
        const int nr = (int)std::min<int64_t>(NR, j1 - j);
        for (int jj = 0; jj < NR; ++jj) {
            int64_t col = j + (jj < nr ? jj : 0);
            int64_t blk = (col - a0) / MR, off = (col - a0) % MR;
            for (int p = 0; p < kw; ++p) bj[p * NR + jj] = jj < nr ? Ap[blk * kw * MR + p * MR + off] : T(0);
        }
        // first 8-row block containing row j
        int64_t ib0 = ((j - a0) / MR) * MR + a0;
        for (int64_t i = ib0; i < nf; i += MR) {
            const T* a = Ap + ((i - a0) / MR) * kw * MR;
            T acc[NR][MR];
            for (int jj = 0; jj < NR; ++jj)
                for (int r = 0; r < MR; ++r) acc[jj][r] = T(0);
            for (int p = 0; p < kw; ++p) {
                const T* ap = a + p * MR;
                for (int jj = 0; jj < NR; ++jj) {
                    const T b = bj[p * NR + jj];
                    for (int r = 0; r < MR; ++r) acc[jj][r] += ap[r] * b;
                }
            }
            for (int jj = 0; jj < nr; ++jj) {
                T* c = F + (j + jj) * ld;
                for (int r = 0; r < MR; ++r) {
                    int64_t row = i + r;
                    if (row >= j + jj && row < nf) c[row] -= acc[jj][r];
                }
            }
        }
    }
}

// Partial Cholesky of the front F (nf x nf, ld nf, lower triangle): eliminate the
// first ncol columns.  Returns -1 on success or the failing column.
template <typename T>
int64_t partial_cholesky(T* F, int64_t nf, int64_t ncol, int nthreads) {
    const int64_t ld = nf;
    constexpr int NB = 64;
    std::vector<T> Ap;
    for (int64_t k0 = 0; k0 < ncol; k0 += NB) {
        const int kw = (int)std::min<int64_t>(NB, ncol - k0);
        const int64_t k1 = k0 + kw;
        // 1. diagonal block, unblocked right-looking
        for (int64_t j = k0; j < k1; ++j) {
            T d = F[j + j * ld];
            if (!(d > T(0)) || !std::isfinite(d)) return j;
            d = std::sqrt(d);
            F[j + j * ld] = d;
            const T inv = T(1) / d;
            for (int64_t i = j + 1; i < k1; ++i) F[i + j * ld] *= inv;
            for (int64_t jj = j + 1; jj < k1; ++jj) {
                const T f = F[jj + j * ld];
                for (int64_t i = jj; i < k1; ++i) F[i + jj * ld] -= F[i + j * ld] * f;
            }
        }
        if (k1 >= nf) break;
        // 2. rows below: F[k1:nf, k0:k1] <- F[k1:nf, k0:k1] L_kk^{-T}
        const int64_t nbelow = nf - k1;
        const int64_t rchunk = 512;
        parallel_for((nbelow + rchunk - 1) / rchunk, nthreads, [&](int64_t c) {
            const int64_t r0 = k1 + c * rchunk, r1 = std::min(nf, r0 + rchunk);
            for (int64_t j = k0; j < k1; ++j) {
                T* cj = F + j * ld;
                for (int64_t p = k0; p < j; ++p) {
                    const T l = F[j + p * ld];
                    const T* cp = F + p * ld;
                    for (int64_t i = r0; i < r1; ++i) cj[i] -= cp[i] * l;
                }
                const T inv = T(1) / F[j + j * ld];
                for (int64_t i = r0; i < r1; ++i) cj[i] *= inv;
            }
        });
        // 3. trailing update of the lower triangle F[k1:nf, k1:nf] by the panel
        const int64_t a0 = k1;
        const int64_t nblk = (nbelow + 7) / 8;
        Ap.assign((size_t)nblk * kw * 8, T(0));
        parallel_for(nblk, nthreads, [&](int64_t b) {
            for (int p = 0; p < kw; ++p)
                for (int r = 0; r < 8; ++r) {
                    int64_t row = a0 + b * 8 + r;
                    Ap[b * kw * 8 + p * 8 + r] = row < nf ? F[row + (k0 + p) * ld] : T(0);
                }
        });
        const int64_t cblk = 32;
        const int64_t ncb = (nbelow + cblk - 1) / cblk;
        parallel_for(ncb, nthreads, [&](int64_t c) {
            const int64_t j0 = k1 + c * cblk, j1 = std::min(nf, j0 + cblk);
            syrk_cols<T>(F, ld, nf, Ap.data(), a0, kw, j0, j1);
        });
    }
    return -1;
}

// X = L^{-1} for the lower-triangular L (n x n, ld ldl); X column-major ld n.
template <typename T>
void invert_lower(const T* L, int64_t ldl, int64_t n, T* X, int nthreads) {
    parallel_for(n, nthreads, [&](int64_t j) {
        T* x = X + j * n;
        for (int64_t i = 0; i < j; ++i) x[i] = T(0);
        for (int64_t i = j; i < n; ++i) x[i] = T(0);
        x[j] = T(1);
        for (int64_t k = j; k < n; ++k) {
            const T xk = x[k] / L[k + k * ldl];
            x[k] = xk;
            if (xk == T(0)) continue;
            const T* lk = L + k * ldl;
            for (int64_t i = k + 1; i < n; ++i) x[i] -= lk[i] * xk;
        }
    });
}

}  // namespace

// ------------------------------------------------------------------ factorize

int factorize(const HostCSR& A, const double* kval, const double* coords, HostFactor& F,
              std::string& msg, bool single) {
    const int64_t n = A.n;
    const int nthreads = host_threads();
    double t0 = wall();
    std::vector<TreeNode> nodes;
    std::vector<int> roots;
    {
        Dissector D(A, coords, nodes);
        std::vector<int32_t> all(n);
        std::iota(all.begin(), all.end(), 0);
        roots = D.build(all);
    }
    // postorder
    std::vector<int> post;
    post.reserve(nodes.size());
    {
        std::vector<std::pair<int, size_t>> st;
        for (int r : roots) {
            st.push_back({r, 0});
            while (!st.empty()) {
                auto& top = st.back();
                if (top.second < nodes[top.first].children.size()) {
                    int c = nodes[top.first].children[top.second++];
                    st.push_back({c, 0});
                } else {
                    post.push_back(top.first);
                    st.pop_back();
                }
            }
        }
    }
    const int nsn = (int)post.size();
    std::vector<int> sn_of_node(nodes.size(), -1);
    for (int i = 0; i < nsn; ++i) sn_of_node[post[i]] = i;
    F = HostFactor();
    F.n = n;
    F.sn.resize(nsn);
    F.perm.resize(n);
    std::vector<int32_t> invperm(n, -1);
    {
        int64_t pos = 0;
        for (int i = 0; i < nsn; ++i) {
            const TreeNode& t = nodes[post[i]];
            F.sn[i].pos0 = pos;
            F.sn[i].ncol = (int32_t)t.verts.size();
            for (int32_t v : t.verts) {
                F.perm[pos] = v;
                invperm[v] = (int32_t)pos;
                ++pos;
            }
            for (int c : t.children) F.sn[sn_of_node[c]].parent = i;
        }
        if (pos != n) {
            msg = "nested dissection lost vertices";
            return -1;
        }
    }
    std::vector<std::vector<int>> kids(nsn);
    for (int i = 0; i < nsn; ++i)
        if (F.sn[i].parent >= 0) kids[F.sn[i].parent].push_back(i);
    // levels (height)
    int32_t maxlev = 0;
    for (int i = 0; i < nsn; ++i) {
        int32_t lv = 0;
        for (int c : kids[i]) lv = std::max(lv, F.sn[c].level + 1);
        F.sn[i].level = lv;
        maxlev = std::max(maxlev, lv);
    }
    F.nlevels = maxlev + 1;
    // symbolic: B_t = positions after D_t reached from D_t's adjacency or children's B
    std::vector<std::vector<int32_t>> B(nsn);
    {
        std::vector<int32_t> flag(n, -1);
        for (int i = 0; i < nsn; ++i) {
            const int64_t end = F.sn[i].pos0 + F.sn[i].ncol;
            std::vector<int32_t>& b = B[i];
            for (int64_t p = F.sn[i].pos0; p < end; ++p) {
                int32_t v = F.perm[p];
                for (int64_t e = A.rowptr[v]; e < A.rowptr[v + 1]; ++e) {
                    int32_t q = invperm[A.col[e]];
                    if (q >= end && flag[q] != i) { flag[q] = i; b.push_back(q); }
                }
            }
            for (int c : kids[i])
                for (int32_t q : B[c])
                    if (q >= end && flag[q] != i) { flag[q] = i; b.push_back(q); }
            std::sort(b.begin(), b.end());
        }
    }
    // layout of rows and panels
    int64_t idx = 0, val = 0;
    for (int i = 0; i < nsn; ++i) {
        F.sn[i].nrow = F.sn[i].ncol + (int32_t)B[i].size();
        F.sn[i].idx_off = idx;
        F.sn[i].val_off = val;
        idx += F.sn[i].nrow;
        val += (int64_t)F.sn[i].nrow * F.sn[i].ncol;
        const double nc = F.sn[i].ncol, nb = (double)B[i].size();
        F.flops += nc * nc * nc / 3.0 + nb * nc * nc + nb * nb * nc;
        F.nnz_factor += (int64_t)(nc * (nc + 1) / 2) + (int64_t)(nb * nc);
    }
    F.rows.resize(idx);
    F.panels.assign(val, 0.0);
    for (int i = 0; i < nsn; ++i) {
        int32_t* r = F.rows.data() + F.sn[i].idx_off;
        for (int32_t k = 0; k < F.sn[i].ncol; ++k) r[k] = F.perm[F.sn[i].pos0 + k];
        for (size_t k = 0; k < B[i].size(); ++k) r[F.sn[i].ncol + k] = F.perm[B[i][k]];
    }
    double t1 = wall();
    F.t_order = t1 - t0;

    // numeric: subtrees below the top levels run in parallel, one thread each;
    // the top supernodes then run one at a time with threaded dense kernels
    std::atomic<int> fail(-1);
    // the arithmetic of the fronts in FP64, or in FP32 (single: the conclusions'
    // single-precision factorisation); the panels are kept in FP64 either way
    auto numeric = [&](auto zero) {
    using T = decltype(zero);
    std::vector<std::unique_ptr<std::vector<T>>> upd(nsn);
    auto do_node = [&](int i, std::vector<int32_t>& loc, int nt) {
        const Supernode& s = F.sn[i];
        const int64_t nc = s.ncol, nf = s.nrow, nb = nf - nc;
        std::vector<T> Fr((size_t)nf * nf, T(0));
        for (int64_t k = 0; k < nc; ++k) loc[s.pos0 + k] = (int32_t)k;
        for (int64_t k = 0; k < nb; ++k) loc[B[i][k]] = (int32_t)(nc + k);
        for (int64_t jj = 0; jj < nc; ++jj) {
            const int64_t pj = s.pos0 + jj;
            const int32_t v = F.perm[pj];
            for (int64_t e = A.rowptr[v]; e < A.rowptr[v + 1]; ++e) {
                const int32_t q = invperm[A.col[e]];
                if (q >= pj) Fr[loc[q] + jj * nf] += (T)kval[e];
            }
        }
        for (int c : kids[i]) {
            const std::vector<int32_t>& bc = B[c];
            const int64_t m = (int64_t)bc.size();
            const T* U = upd[c]->data();
            std::vector<int32_t> li(m);
            for (int64_t a = 0; a < m; ++a) li[a] = loc[bc[a]];
            for (int64_t bcol = 0; bcol < m; ++bcol) {
                T* fc = Fr.data() + (int64_t)li[bcol] * nf;
                const T* uc = U + bcol * m;
                for (int64_t a = bcol; a < m; ++a) fc[li[a]] += uc[a];
            }
            upd[c].reset();
        }
        for (int64_t k = 0; k < nc; ++k) loc[s.pos0 + k] = -1;
        for (int64_t k = 0; k < nb; ++k) loc[B[i][k]] = -1;
        int64_t bad = partial_cholesky<T>(Fr.data(), nf, nc, nt);
        if (bad >= 0) {
            int expected = -1;
            fail.compare_exchange_strong(expected, i);
            return;
        }
        double* panel = F.panels.data() + s.val_off;
        // X = inv(L11) (lower, ld nc); the panel receives G = X^T X = (L11 L11^T)^{-1} on
        // top (full, symmetric) and F = L21 X below
        std::vector<T> X((size_t)nc * nc);
        invert_lower<T>(Fr.data(), nf, nc, X.data(), nt);
        parallel_for(nc, nt, [&](int64_t b) {
            // column b of G: G[a, b] = sum_{k >= max(a, b)} X[k, a] X[k, b]
            const T* xb = X.data() + b * nc;
            for (int64_t a = 0; a < nc; ++a) {
                const T* xa = X.data() + a * nc;
                T acc = T(0);
                for (int64_t k = std::max(a, b); k < nc; ++k) acc += xa[k] * xb[k];
                panel[a + b * nf] = (double)acc;
            }
            // column b of F: F[i, b] = sum_{k >= b} L21[i, k] X[k, b]
            std::vector<T> fb(nb, T(0));
            for (int64_t k = b; k < nc; ++k) {
                const T xkb = xb[k];
                if (xkb == T(0)) continue;
                const T* l21k = Fr.data() + k * nf + nc;
                for (int64_t i = 0; i < nb; ++i) fb[i] += l21k[i] * xkb;
            }
            double* fp = panel + b * nf + nc;
            for (int64_t i = 0; i < nb; ++i) fp[i] = (double)fb[i];
        });
        if (nb > 0) {
            auto U = std::make_unique<std::vector<T>>((size_t)nb * nb);
            for (int64_t j = 0; j < nb; ++j)
                std::memcpy(U->data() + j * nb + j, Fr.data() + (nc + j) * nf + nc + j,
                            sizeof(T) * (nb - j));
            upd[i] = std::move(U);
        }
    };
    // split: supernodes whose level is below `cutlev` belong to parallel subtrees
    std::vector<int> top_nodes, sub_roots;
    const int cutlev = std::max(0, F.nlevels - 5);
    for (int i = 0; i < nsn; ++i) {
        if (F.sn[i].level >= cutlev) top_nodes.push_back(i);
        else if (F.sn[i].parent < 0 || F.sn[F.sn[i].parent].level >= cutlev) sub_roots.push_back(i);
    }
    // each subtree is a contiguous postorder range ending at its root
    std::vector<int> first_of(nsn);
    for (int i = 0; i < nsn; ++i) {
        int f = i;
        for (int c : kids[i]) f = std::min(f, first_of[c]);
        first_of[i] = f;
    }
    const double t_sub0 = wall();
    parallel_for((int64_t)sub_roots.size(), nthreads, [&](int64_t k) {
        std::vector<int32_t> loc(n, -1);
        const int r = sub_roots[k];
        for (int i = first_of[r]; i <= r && fail.load() < 0; ++i) do_node(i, loc, 1);
    });
    F.t_subtrees = wall() - t_sub0;
    {
        std::vector<int32_t> loc(n, -1);
        for (int i : top_nodes) {
            if (fail.load() >= 0) break;
            do_node(i, loc, nthreads);
        }
    }
    };
    if (single) numeric(0.0f);
    else numeric(0.0);
    F.t_factor = wall() - t1;
    if (fail.load() >= 0) {
        msg = "H - eps_bar S is not positive definite (non-positive pivot in supernode " +
              std::to_string(fail.load()) + ")";
        return -4;
    }
    return 0;
}

void host_solve(const HostFactor& F, double* b) {
    // forward: r_B -= F r_D, supernodes in postorder; then x_D = G r_D; backward:
    // x_D -= F^T x_B, supernodes in reverse postorder
    for (const Supernode& s : F.sn) {
        const int32_t* r = F.rows.data() + s.idx_off;
        const double* P = F.panels.data() + s.val_off;
        const int64_t nc = s.ncol, nf = s.nrow;
        for (int64_t j = 0; j < nc; ++j)
            for (int64_t i = nc; i < nf; ++i) b[r[i]] -= P[i + j * nf] * b[r[j]];
    }
    std::vector<double> z;
    for (const Supernode& s : F.sn) {
        const int32_t* r = F.rows.data() + s.idx_off;
        const double* P = F.panels.data() + s.val_off;
        const int64_t nc = s.ncol, nf = s.nrow;
        z.assign(nc, 0.0);
        for (int64_t j = 0; j < nc; ++j)
            for (int64_t i = 0; i < nc; ++i) z[i] += P[i + j * nf] * b[r[j]];
        for (int64_t i = 0; i < nc; ++i) b[r[i]] = z[i];
    }
    for (auto it = F.sn.rbegin(); it != F.sn.rend(); ++it) {
        const Supernode& s = *it;
        const int32_t* r = F.rows.data() + s.idx_off;
        const double* P = F.panels.data() + s.val_off;
        const int64_t nc = s.ncol, nf = s.nrow;
        for (int64_t j = 0; j < nc; ++j) {
            double acc = 0.0;
            for (int64_t i = nc; i < nf; ++i) acc += P[i + j * nf] * b[r[i]];
            b[r[j]] -= acc;
        }
    }
}

}  // namespace labpsd
