// Small dense Hermitian eigenproblems on the host (the 2 x 2 line search and the
// n x n Rayleigh-Ritz step of the low-eigenmode solver).
#pragma once

#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

namespace cola {

using cd = std::complex<double>;

// Lower eigenvector (u0, u1) of the Hermitian [[m, b], [conj b, c]], from whichever row
// of (H - lambda) gives the longer null vector.
inline void lower_eigvec(double m, cd b, double c, cd *u0, cd *u1) {
    const double h = 0.5 * (m - c);
    const double lam = 0.5 * (m + c) - std::sqrt(h * h + std::norm(b));
    cd a0, a1;
    if (m >= c) {
        a0 = b;
        a1 = cd(lam - m, 0);
    } else {
        a0 = cd(lam - c, 0);
        a1 = std::conj(b);
    }
    const double nn = std::sqrt(std::norm(a0) + std::norm(a1));
    if (!(nn > 0)) {
        *u0 = cd(1, 0);
        *u1 = cd(0, 0);
        return;
    }
    *u0 = a0 / nn;
    *u1 = a1 / nn;
}

// Eigenvalues (ascending) and orthonormal eigenvectors (columns of V, row-major n x n) of
// a Hermitian n x n matrix A (row-major), by cyclic Jacobi rotations: each rotation
// R = diag(1, conj(phase)) G zeroes one off-diagonal pair, with G the real Jacobi
// rotation of the modulus.
inline void herm_eig(int n, std::vector<cd> A, std::vector<double> &w, std::vector<cd> &V) {
    V.assign((size_t)n * n, cd(0, 0));
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    auto a = [&](int i, int j) -> cd & { return A[(size_t)i * n + j]; };
    double fro = 0;
    for (auto &z : A) fro += std::norm(z);
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += std::norm(a(p, q));
        if (off <= 1e-32 * fro) break;
        for (int p = 0; p < n - 1; ++p) {
            for (int q = p + 1; q < n; ++q) {
                const cd apq = a(p, q);
                const double r = std::abs(apq);
                if (r <= 1e-300) continue;
                const cd ph = apq / r;
                const double tau = (a(q, q).real() - a(p, p).real()) / (2 * r);
                const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1 + tau * tau));
                const double c = 1 / std::sqrt(1 + t * t), s = t * c;
                // R = [[c, s], [-s conj(ph), c conj(ph)]] on (p, q)
                const cd rpp = c, rpq = s, rqp = -s * std::conj(ph), rqq = c * std::conj(ph);
                for (int k = 0; k < n; ++k) {  // A <- A R
                    const cd x = a(k, p), y = a(k, q);
                    a(k, p) = x * rpp + y * rqp;
                    a(k, q) = x * rpq + y * rqq;
                }
                for (int k = 0; k < n; ++k) {  // A <- R^H A
                    const cd x = a(p, k), y = a(q, k);
                    a(p, k) = std::conj(rpp) * x + std::conj(rqp) * y;
                    a(q, k) = std::conj(rpq) * x + std::conj(rqq) * y;
                }
                a(p, q) = a(q, p) = 0;
                for (int k = 0; k < n; ++k) {  // V <- V R
                    const cd x = V[(size_t)k * n + p], y = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = x * rpp + y * rqp;
                    V[(size_t)k * n + q] = x * rpq + y * rqq;
                }
            }
        }
    }
    std::vector<int> ord(n);
    for (int i = 0; i < n; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(),
                     [&](int x, int y) { return a(x, x).real() < a(y, y).real(); });
    w.resize(n);
    std::vector<cd> Vs((size_t)n * n);
    for (int j = 0; j < n; ++j) {
        w[j] = a(ord[j], ord[j]).real();
        for (int k = 0; k < n; ++k) Vs[(size_t)k * n + j] = V[(size_t)k * n + ord[j]];
    }
    V.swap(Vs);
}

}  // namespace cola
