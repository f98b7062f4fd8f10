// Host pieces of the complex Hermitian (k-point) variant; see hermitian.cpp.
#pragma once

#include <cstdint>
#include <vector>

namespace labpsd {

// The real symmetric embedding R(A) (2n x 2n, interleaved) of the complex matrix A given
// on the CSR pattern (rowptr, col) by its real and imaginary parts.
void embed_hermitian(int64_t n, int64_t nnz, const int64_t* rowptr, const int32_t* col, const double* re,
                     const double* im, std::vector<int64_t>& rp2, std::vector<int32_t>& col2,
                     std::vector<double>& val2);

// Eigen-decomposition of a complex Hermitian n x n matrix (column-major re/im parts) by
// cyclic Jacobi: the diagonal of (Ar, Ai) ends as the eigenvalues (unsorted), (Vr, Vi) the
// unitary eigenvector matrix.
void hermitian_jacobi(int n, std::vector<double>& Ar, std::vector<double>& Ai, std::vector<double>& Vr,
                      std::vector<double>& Vi);

}  // namespace labpsd
