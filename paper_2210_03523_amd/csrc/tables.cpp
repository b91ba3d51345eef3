// Host computation of the 1D nodal tables of the DGSEM (Section 2.1: tensor-product
// Lagrange basis on Legendre-Gauss-Lobatto nodes with collocated quadrature).
//
//   nodes   : +-1 and the eigenvalues of the Jacobi matrix of the (1,1) Jacobi
//             weight (Golub-Welsch), found by Sturm-sequence bisection;
//   weights : 2 / (N (N+1) L_N(x_j)^2);
//   D       : closed form of the Gauss-Lobatto differentiation matrix,
//             D_ij = L_N(x_i) / (L_N(x_j) (x_i - x_j)), D_00 = -N(N+1)/4, D_NN = N(N+1)/4;
//   I^{A<-B}: Lagrange basis of order B (product form) at the order-A nodes;
//   P^{A<-B}: L2 projection from order B onto order A, through the Legendre
//             coefficients, integrated with a Gauss-Legendre rule of B+1 points
//             (exact for the degrees involved).
#include <cmath>
#include <vector>

#include "common.h"

namespace dgt {
namespace {

using ld = long double;

// Legendre L_n(x) by the three-term recurrence.
ld legendre(int n, ld x) {
    if (n == 0) return 1.0L;
    ld a = 1.0L, b = x;
    for (int k = 1; k < n; ++k) {
        ld c = ((2 * k + 1) * x * b - k * a) / (k + 1);
        a = b;
        b = c;
    }
    return b;
}

ld legendre_deriv(int n, ld x) {
    // n (x L_n - L_{n-1}) / (x^2 - 1) is singular at +-1; use the series sum
    // L_n' = sum_{k = n-1, n-3, ...} (2k+1) L_k
    ld s = 0.0L;
    for (int k = n - 1; k >= 0; k -= 2) s += (2 * k + 1) * legendre(k, x);
    return s;
}

// Eigenvalues of the symmetric tridiagonal matrix with zero diagonal and
// off-diagonal sqrt(beta[k]) (k = 1..m-1), sorted ascending, by bisection.
std::vector<ld> tridiag_eigs(const std::vector<ld> &beta, int m) {
    std::vector<ld> ev(m);
    auto count_below = [&](ld x) {
        // number of eigenvalues < x (Sturm sequence of the LDL^T pivots)
        int c = 0;
        ld q = -x;
        if (q < 0) ++c;
        for (int k = 1; k < m; ++k) {
            if (q == 0.0L) q = 1e-300L;
            q = -x - beta[k] / q;
            if (q < 0) ++c;
        }
        return c;
    };
    for (int i = 0; i < m; ++i) {
        ld lo = -1.0L, hi = 1.0L;
        for (int it = 0; it < 200; ++it) {
            ld mid = 0.5L * (lo + hi);
            if (count_below(mid) > i) hi = mid; else lo = mid;
            if (hi - lo < 1e-30L) break;
        }
        ev[i] = 0.5L * (lo + hi);
    }
    return ev;
}

std::vector<ld> lgl_nodes(int N) {
    std::vector<ld> x(N + 1);
    x[0] = -1.0L;
    x[N] = 1.0L;
    if (N > 1) {
        int m = N - 1;  // roots of the Jacobi (1,1) polynomial of degree N-1
        std::vector<ld> beta(m);
        for (int k = 1; k < m; ++k) beta[k] = (ld)k * (k + 2) / ((ld)(2 * k + 1) * (2 * k + 3));
        auto ev = tridiag_eigs(beta, m);
        for (int j = 0; j < m; ++j) x[j + 1] = ev[j];
    }
    // antisymmetric and exactly zero in the middle
    for (int j = 0; j < (N + 1) / 2; ++j) {
        ld s = 0.5L * (x[N - j] - x[j]);
        x[j] = -s;
        x[N - j] = s;
    }
    if (N % 2 == 0) x[N / 2] = 0.0L;
    return x;
}

void gauss_legendre(int n, std::vector<ld> &y, std::vector<ld> &om) {
    std::vector<ld> beta(n);
    for (int k = 1; k < n; ++k) beta[k] = (ld)k * k / (4.0L * k * k - 1.0L);
    y = tridiag_eigs(beta, n);
    om.resize(n);
    for (int g = 0; g < n; ++g) {
        ld d = legendre_deriv(n, y[g]);
        om[g] = 2.0L / ((1.0L - y[g] * y[g]) * d * d);
    }
}

ld lagrange(const std::vector<ld> &x, int k, ld t) {
    ld p = 1.0L;
    for (size_t j = 0; j < x.size(); ++j)
        if ((int)j != k) p *= (t - x[j]) / (x[k] - x[j]);
    return p;
}

}  // namespace

void build_tables(double *t64, float *t32) {
    std::vector<ld> tab(T_TOT, 0.0L);
    std::vector<std::vector<ld>> X(NMAX + 1);
    for (int N = 1; N <= NMAX; ++N) X[N] = lgl_nodes(N);
    for (int N = 1; N <= NMAX; ++N) {
        const auto &x = X[N];
        for (int j = 0; j <= N; ++j) {
            ld L = legendre(N, x[j]);
            tab[T_X + xoff(N) + j] = x[j];
            tab[T_W + xoff(N) + j] = 2.0L / ((ld)N * (N + 1) * L * L);
        }
        int n = N + 1;
        for (int i = 0; i <= N; ++i)
            for (int j = 0; j <= N; ++j) {
                ld v;
                if (i != j) v = legendre(N, x[i]) / (legendre(N, x[j]) * (x[i] - x[j]));
                else if (i == 0) v = -(ld)N * (N + 1) / 4.0L;
                else if (i == N) v = (ld)N * (N + 1) / 4.0L;
                else v = 0.0L;
                tab[T_D + doff(N) + i * n + j] = v;
            }
    }
    for (int A = 1; A <= NMAX; ++A)
        for (int B = 1; B <= NMAX; ++B) {
            int na = A + 1, nb = B + 1;
            // interpolation: order-B basis at the order-A nodes
            for (int a = 0; a < na; ++a)
                for (int k = 0; k < nb; ++k) tab[T_I + moff(A, B) + a * nb + k] = lagrange(X[B], k, X[A][a]);
            // projection from order B onto order A (defined for A <= B)
            if (A > B) continue;
            if (A == B) {
                for (int a = 0; a < na; ++a)
                    for (int q = 0; q < nb; ++q) tab[T_P + moff(A, B) + a * nb + q] = (a == q) ? 1.0L : 0.0L;
                continue;
            }
            std::vector<ld> y, om;
            gauss_legendre(B + 1, y, om);
            for (int q = 0; q < nb; ++q) {
                // Legendre coefficients c_m (m <= A) of the order-B basis function l_q
                std::vector<ld> c(A + 1, 0.0L);
                for (int m = 0; m <= A; ++m) {
                    ld s = 0.0L;
                    for (size_t g = 0; g < y.size(); ++g) s += om[g] * legendre(m, y[g]) * lagrange(X[B], q, y[g]);
                    c[m] = s * (2 * m + 1) / 2.0L;
                }
                for (int a = 0; a < na; ++a) {
                    ld v = 0.0L;
                    for (int m = 0; m <= A; ++m) v += c[m] * legendre(m, X[A][a]);
                    tab[T_P + moff(A, B) + a * nb + q] = v;
                }
            }
        }
    for (int i = 0; i < T_TOT; ++i) {
        t64[i] = (double)tab[i];
        t32[i] = (float)tab[i];
    }
}

}  // namespace dgt
