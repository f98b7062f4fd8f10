// Host-side sparse Cholesky of K = H - eps_bar S for the global preconditioner.
//
// The paper factors H^(loc,1) - eps_bar S once, with a fill-reducing permutation
// (eq. (ldl)), and reuses the factor for every application (Section 4).  With
// eps_bar below the lowest eigenvalue the matrix is positive definite, so the
// factorisation is a Cholesky factorisation P^T K P = L L^T (1x1 pivots only).
//
// Ordering: nested dissection.  With dof coordinates the vertex set is bisected at
// the median of its widest coordinate and the separator is the layer of one side
// adjacent to the other (periodic wrap-around edges put both cut planes into the
// separator without any special case); without coordinates a breadth-first level
// structure from a pseudo-peripheral vertex supplies the cut.
//
// Numeric factorisation: multifrontal, one frontal matrix per separator or leaf of
// the dissection tree (each is one supernode: its diagonal block is dense after the
// elimination of its subtrees), blocked dense Cholesky / triangular solve / rank-k
// update on the front, children's update matrices extended-added into the parent.
//
// Output for the device apply: per supernode a column-major panel of nrow x ncol,
// rows = [D (its own columns) ; B (rows in ancestors)], whose top ncol x ncol block
// holds G = (L11 L11^T)^{-1} (full, symmetric) and whose bottom nB x ncol block holds
// F = L21 L11^{-1}.  With them K^{-1} r is: r_B -= F r_D up the tree, x_D = G r_D for
// every supernode, x_D -= F^T x_B down the tree; each supernode needs only the
// right-hand side's own rows, so a tree level is one product.  Row lists hold original
// dof indices, so the symmetric permutation is folded into the gathers and scatters.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace labpsd {

struct HostCSR {
    int64_t n = 0;
    int64_t nnz = 0;
    std::vector<int64_t> rowptr;
    std::vector<int32_t> col;
};

struct Supernode {
    int64_t pos0 = 0;     // first elimination position of its columns
    int32_t ncol = 0;     // |D|
    int32_t nrow = 0;     // |D| + |B|
    int64_t idx_off = 0;  // offset of its row list in HostFactor::rows
    int64_t val_off = 0;  // offset of its panel in HostFactor::panels
    int32_t parent = -1;  // -1 for a root
    int32_t level = 0;    // height above the leaves (leaves are level 0)
};

struct HostFactor {
    int64_t n = 0;
    std::vector<Supernode> sn;      // in postorder (children before parents)
    std::vector<int32_t> rows;      // concatenated row lists (original dof indices)
    std::vector<double> panels;     // concatenated panels [G ; F], ld nrow
    std::vector<int32_t> perm;      // perm[position] = dof
    int32_t nlevels = 0;
    int64_t nnz_factor = 0;
    double flops = 0.0;
    double t_order = 0.0;
    double t_factor = 0.0;
    double t_subtrees = 0.0;   // part of t_factor spent in the parallel subtrees
};

// Factor K (values `kval` on the pattern of A).  single: the numeric factorisation
// (fronts, Cholesky, inverses, panels) in FP32 arithmetic, the panels then stored
// widened to FP64.  Returns 0, or -4 when a pivot is not positive (msg names the
// supernode), or -1 on an internal inconsistency.
int factorize(const HostCSR& A, const double* kval, const double* coords, HostFactor& F,
              std::string& msg, bool single = false);

// Solve K x = b on the host with the factor (for self-checks): x overwrites b.
void host_solve(const HostFactor& F, double* b);

}  // namespace labpsd
