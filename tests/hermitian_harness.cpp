// CPU test driver of the host pieces of the k-point variant (hermitian.cpp): the complex
// Hermitian Jacobi eigensolver on seeded random matrices, and the real embedding's
// structure.  Prints "jacobi n resid orth" and "embed symmetric ok" lines.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <random>

#include "hermitian.h"

using namespace labpsd;
using cd = std::complex<double>;

int main() {
    std::mt19937_64 g(7);
    std::normal_distribution<double> d;
    for (int n : {1, 2, 7, 33, 64}) {
        std::vector<double> Ar((size_t)n * n), Ai(Ar.size());
        for (int j = 0; j < n; ++j)
            for (int i = 0; i <= j; ++i) {
                const double a = d(g), b = i == j ? 0.0 : d(g);
                Ar[i + (size_t)j * n] = Ar[j + (size_t)i * n] = a;
                Ai[i + (size_t)j * n] = b;
                Ai[j + (size_t)i * n] = -b;
            }
        if (n == 64)   // a degenerate block: eigenvalue 3 five times
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    Ar[i + (size_t)j * n] = (i == j) ? (i < 5 ? 3.0 : 3.0 + i) : 0.0;
                    Ai[i + (size_t)j * n] = 0.0;
                }
        auto Br = Ar, Bi = Ai;
        std::vector<double> Vr, Vi;
        hermitian_jacobi(n, Ar, Ai, Vr, Vi);
        double res = 0.0, orth = 0.0, scale = 0.0;
        for (double v : Br) scale = std::max(scale, std::fabs(v));
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                cd s = 0.0;
                for (int k = 0; k < n; ++k)
                    s += cd(Br[i + (size_t)k * n], Bi[i + (size_t)k * n]) * cd(Vr[k + (size_t)j * n], Vi[k + (size_t)j * n]);
                s -= Ar[j + (size_t)j * n] * cd(Vr[i + (size_t)j * n], Vi[i + (size_t)j * n]);
                res = std::max(res, std::abs(s));
                cd o = 0.0;
                for (int k = 0; k < n; ++k)
                    o += std::conj(cd(Vr[k + (size_t)i * n], Vi[k + (size_t)i * n])) * cd(Vr[k + (size_t)j * n], Vi[k + (size_t)j * n]);
                orth = std::max(orth, std::abs(o - (i == j ? 1.0 : 0.0)));
            }
        printf("jacobi %d %.3e %.3e\n", n, res / std::max(scale, 1e-300), orth);
    }
    // embedding of a random Hermitian 3 x 3 with a full pattern: symmetric, and R(A) R(x) = R(A x)
    const int n = 3;
    std::vector<int64_t> rp = {0, 3, 6, 9};
    std::vector<int32_t> col = {0, 1, 2, 0, 1, 2, 0, 1, 2};
    std::vector<cd> A(9);
    for (int i = 0; i < n; ++i)
        for (int j = i; j < n; ++j) {
            const cd a(d(g), i == j ? 0.0 : d(g));
            A[i * 3 + j] = a;
            A[j * 3 + i] = std::conj(a);
        }
    std::vector<double> re(9), im(9);
    for (int e = 0; e < 9; ++e) { re[e] = A[e].real(); im[e] = A[e].imag(); }
    std::vector<int64_t> rp2;
    std::vector<int32_t> col2;
    std::vector<double> v2;
    embed_hermitian(n, 9, rp.data(), col.data(), re.data(), im.data(), rp2, col2, v2);
    std::vector<double> M(36, 0.0);
    for (int r = 0; r < 6; ++r)
        for (int64_t e = rp2[r]; e < rp2[r + 1]; ++e) M[r * 6 + col2[e]] = v2[e];
    bool sym = true;
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) sym = sym && M[r * 6 + c] == M[c * 6 + r];
    std::vector<cd> x = {cd(d(g), d(g)), cd(d(g), d(g)), cd(d(g), d(g))};
    double err = 0.0;
    for (int i = 0; i < n; ++i) {
        cd y = 0.0;
        for (int j = 0; j < n; ++j) y += A[i * 3 + j] * x[j];
        double yr = 0.0, yi = 0.0;
        for (int j = 0; j < n; ++j) {
            yr += M[(2 * i) * 6 + 2 * j] * x[j].real() + M[(2 * i) * 6 + 2 * j + 1] * x[j].imag();
            yi += M[(2 * i + 1) * 6 + 2 * j] * x[j].real() + M[(2 * i + 1) * 6 + 2 * j + 1] * x[j].imag();
        }
        err = std::max(err, std::abs(cd(yr, yi) - y));
    }
    printf("embed %d %.3e\n", sym ? 1 : 0, err);
    return 0;
}
