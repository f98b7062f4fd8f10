// CPU test driver of the host factorisation (paper_1308_2445_amd/csrc/factor.cpp):
// reads a sparse SPD matrix K (CSR, values on the pattern), optional coordinates and a
// right-hand side from a binary file, factorises, checks the ordering and the symbolic
// structure in C++, solves K x = b with the factor and writes the results.
//
//   factor_harness <in.bin> <out.bin>
// in:  int64 n, nnz, has_coords, single; rowptr[n+1] int64; col[nnz] int32; val[nnz] f64;
//      coords[3n] f64 (if has_coords); b[n] f64
// out: int64 status, n_supernodes, perm_ok, symbolic_ok, levels_ok; x[n] f64
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "factor.h"

using namespace labpsd;

template <typename T>
static bool rd(FILE* f, T* p, size_t n) { return fread(p, sizeof(T), n, f) == n; }

int main(int argc, char** argv) {
    if (argc != 3) return 2;
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t hdr[4];
    if (!rd(f, hdr, 4)) return 2;
    const int64_t n = hdr[0], nnz = hdr[1];
    HostCSR A;
    A.n = n;
    A.nnz = nnz;
    A.rowptr.resize(n + 1);
    A.col.resize(nnz);
    std::vector<double> val(nnz), coords, b(n);
    if (!rd(f, A.rowptr.data(), n + 1) || !rd(f, A.col.data(), nnz) || !rd(f, val.data(), nnz)) return 2;
    if (hdr[2]) {
        coords.resize(3 * n);
        if (!rd(f, coords.data(), 3 * n)) return 2;
    }
    if (!rd(f, b.data(), n)) return 2;
    fclose(f);

    HostFactor F;
    std::string msg;
    const int rc = factorize(A, val.data(), hdr[2] ? coords.data() : nullptr, F, msg, hdr[3] != 0);
    int64_t perm_ok = 0, sym_ok = 0, lev_ok = 0;
    if (rc == 0) {
        // the ordering is a permutation, and every supernode's own rows are its block of it
        std::vector<int> seen(n, 0);
        perm_ok = (int64_t)F.perm.size() == n;
        for (int32_t v : F.perm) {
            if (v < 0 || v >= n || seen[v]++) perm_ok = 0;
        }
        std::vector<int64_t> pos(n, -1), owner(n, -1);
        for (int64_t p = 0; p < n && perm_ok; ++p) pos[F.perm[p]] = p;
        for (size_t i = 0; i < F.sn.size() && perm_ok; ++i) {
            const Supernode& s = F.sn[i];
            for (int32_t k = 0; k < s.ncol; ++k) {
                if (F.rows[s.idx_off + k] != F.perm[s.pos0 + k]) perm_ok = 0;
                owner[F.rows[s.idx_off + k]] = (int64_t)i;
            }
        }
        // symbolic structure: for every entry K[i, j] with pos(i) > pos(j), row i is in the
        // row list of j's supernode (the factor's pattern contains K's), and every B row of
        // a supernode lies after its own rows
        sym_ok = perm_ok;
        std::vector<std::vector<int32_t>> rows(F.sn.size());
        for (size_t i = 0; i < F.sn.size(); ++i) {
            const Supernode& s = F.sn[i];
            rows[i].assign(F.rows.begin() + s.idx_off, F.rows.begin() + s.idx_off + s.nrow);
            std::vector<int32_t> sorted(rows[i]);
            std::sort(sorted.begin(), sorted.end());
            rows[i] = sorted;
            for (int32_t k = s.ncol; k < s.nrow; ++k)
                if (pos[F.rows[s.idx_off + k]] < s.pos0 + s.ncol) sym_ok = 0;
        }
        for (int64_t i = 0; i < n && sym_ok; ++i)
            for (int64_t e = A.rowptr[i]; e < A.rowptr[i + 1]; ++e) {
                const int32_t j = A.col[e];
                if (pos[i] <= pos[j]) continue;
                const std::vector<int32_t>& r = rows[owner[j]];
                if (!std::binary_search(r.begin(), r.end(), (int32_t)i)) { sym_ok = 0; break; }
            }
        // the tree: a parent sits higher than its children and comes after them
        lev_ok = 1;
        for (size_t i = 0; i < F.sn.size(); ++i) {
            const int32_t p = F.sn[i].parent;
            if (p >= 0 && (p <= (int32_t)i || F.sn[p].level <= F.sn[i].level)) lev_ok = 0;
        }
        host_solve(F, b.data());
    }
    FILE* o = fopen(argv[2], "wb");
    if (!o) return 2;
    const int64_t out[5] = {rc, (int64_t)F.sn.size(), perm_ok, sym_ok, lev_ok};
    fwrite(out, sizeof(int64_t), 5, o);
    fwrite(b.data(), sizeof(double), n, o);
    fclose(o);
    return 0;
}
