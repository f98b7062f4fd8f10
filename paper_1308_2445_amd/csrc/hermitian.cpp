// Host pieces of the complex Hermitian (k-point) variant: the real symmetric embedding of a
// Hermitian pencil, and the small dense Hermitian eigenproblems of the extraction step.
//
// Embedding: a complex n-vector x = a + i b is stored interleaved as the real 2n-vector
// R(x) = (a_0, b_0, a_1, b_1, ...), so the complex block and its embedding are the same
// memory.  H x corresponds to R(H) R(x) with the 2 x 2 blocks [Re h, -Im h; Im h, Re h]
// per entry h of H; R(H) is real symmetric when H is Hermitian, R(S) is positive definite
// when S is, and every eigenvalue of (H, S) is an eigenvalue of (R(H), R(S)) twice, with
// eigenvectors R(x) and R(i x).
#include "hermitian.h"

#include <algorithm>
#include <cmath>

namespace labpsd {

void embed_hermitian(int64_t n, int64_t nnz, const int64_t* rowptr, const int32_t* col, const double* re,
                     const double* im, std::vector<int64_t>& rp2, std::vector<int32_t>& col2,
                     std::vector<double>& val2) {
    rp2.assign(2 * n + 1, 0);
    col2.resize(4 * (size_t)nnz);
    val2.resize(4 * (size_t)nnz);
    int64_t e2 = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int half = 0; half < 2; ++half) {
            for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
                const int32_t j = col[e];
                const double a = re[e], b = im[e];
                // row 2i: [a, -b] at (2j, 2j+1); row 2i+1: [b, a]
                col2[e2] = 2 * j;
                val2[e2] = half == 0 ? a : b;
                ++e2;
                col2[e2] = 2 * j + 1;
                val2[e2] = half == 0 ? -b : a;
                ++e2;
            }
            rp2[2 * i + half + 1] = e2;
        }
    }
}

// Cyclic Jacobi for a complex Hermitian matrix (column-major, n x n, re/im parts): on
// return the diagonal holds the eigenvalues and V (n x n, same layout) the eigenvectors.
// Each rotation first takes the phase out of A[p, q] and then zeroes it with the real
// rotation of the resulting real symmetric 2 x 2 block.
void hermitian_jacobi(int n, std::vector<double>& Ar, std::vector<double>& Ai, std::vector<double>& Vr,
                      std::vector<double>& Vi) {
    auto at = [n](int i, int j) { return (size_t)i + (size_t)j * n; };
    Vr.assign((size_t)n * n, 0.0);
    Vi.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Vr[at(i, i)] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                const double m2 = Ar[at(i, j)] * Ar[at(i, j)] + Ai[at(i, j)] * Ai[at(i, j)];
                tot += m2;
                if (i != j) off += m2;
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double xr = Ar[at(p, q)], xi = Ai[at(p, q)];
                const double r = std::hypot(xr, xi);
                if (r == 0.0) continue;
                // phase e^{i phi} of A[p, q]
                const double er = xr / r, ei = xi / r;
                const double app = Ar[at(p, p)], aqq = Ar[at(q, q)];
                // real rotation of [app, r; r, aqq]
                const double tau = (aqq - app) / (2.0 * r);
                const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                // unitary G on columns p, q: col_p' = c col_p - s conj(e) col_q ... applied as
                // A <- G^H A G with G = [c, s e; -s conj(e), c] (columns p, q)
                for (int k = 0; k < n; ++k) {   // A G (columns)
                    const double apr = Ar[at(k, p)], api = Ai[at(k, p)];
                    const double aqr = Ar[at(k, q)], aqi = Ai[at(k, q)];
                    // new col p = c a_p - s conj(e) a_q
                    Ar[at(k, p)] = c * apr - s * (er * aqr + ei * aqi);
                    Ai[at(k, p)] = c * api - s * (er * aqi - ei * aqr);
                    // new col q = s e a_p + c a_q
                    Ar[at(k, q)] = s * (er * apr - ei * api) + c * aqr;
                    Ai[at(k, q)] = s * (er * api + ei * apr) + c * aqi;
                }
                for (int k = 0; k < n; ++k) {   // G^H A (rows)
                    const double apr = Ar[at(p, k)], api = Ai[at(p, k)];
                    const double aqr = Ar[at(q, k)], aqi = Ai[at(q, k)];
                    // new row p = c a_p - s e a_q
                    Ar[at(p, k)] = c * apr - s * (er * aqr - ei * aqi);
                    Ai[at(p, k)] = c * api - s * (er * aqi + ei * aqr);
                    // new row q = s conj(e) a_p + c a_q
                    Ar[at(q, k)] = s * (er * apr + ei * api) + c * aqr;
                    Ai[at(q, k)] = s * (er * api - ei * apr) + c * aqi;
                }
                Ar[at(p, q)] = Ai[at(p, q)] = Ar[at(q, p)] = Ai[at(q, p)] = 0.0;
                Ai[at(p, p)] = Ai[at(q, q)] = 0.0;
                for (int k = 0; k < n; ++k) {   // V G
                    const double vpr = Vr[at(k, p)], vpi = Vi[at(k, p)];
                    const double vqr = Vr[at(k, q)], vqi = Vi[at(k, q)];
                    Vr[at(k, p)] = c * vpr - s * (er * vqr + ei * vqi);
                    Vi[at(k, p)] = c * vpi - s * (er * vqi - ei * vqr);
                    Vr[at(k, q)] = s * (er * vpr - ei * vpi) + c * vqr;
                    Vi[at(k, q)] = s * (er * vpi + ei * vpr) + c * vqi;
                }
            }
    }
}

}  // namespace labpsd
