// 1D spectral-element basis on Gauss-Legendre-Lobatto (GLL) points, host side.
//
// The NekBone section of the paper uses tensor products of Lagrange
// polynomials interpolating the GLL quadrature points and the 1D derivative
// matrix D.  This file computes them for one degree N at mesh setup:
//  - nodes: the N+1 zeros of (1 - x^2) P_N'(x), by the fixed-point form of
//    Newton's method x <- x - (x P_N - P_{N-1}) / ((N+1) P_N) started from the
//    Chebyshev-Gauss-Lobatto points (the update is Newton's step for
//    x P_N - P_{N-1}, which shares its zeros with (1-x^2) P_N');
//  - weights: w_i = 2 / (N (N+1) P_N(x_i)^2);
//  - D[i][j] = l_j'(x_i) from barycentric weights (Berrut & Trefethen 2004):
//    D_ij = (b_j / b_i) / (x_i - x_j) for i != j and D_ii = -sum_{j != i} D_ij,
//    which makes D annihilate constants to rounding.
#include <cmath>

#include "common.h"

namespace hb {

namespace {

// P_{n-1}(x) and P_n(x) by the three-term recurrence.
void legendre_pair(int n, double x, double &pnm1, double &pn)
{
    double a = 1.0, b = x;  // P_0, P_1
    if (n == 0) {
        pnm1 = 0.0;
        pn = 1.0;
        return;
    }
    for (int k = 2; k <= n; ++k) {
        double c = ((2 * k - 1) * x * b - (k - 1) * a) / k;
        a = b;
        b = c;
    }
    pnm1 = a;
    pn = b;
}

}  // namespace

void gll_basis(int N, double *xi, double *w, double *D)
{
    const int n1 = N + 1;
    for (int i = 0; i <= N; ++i) {
        // descending Chebyshev-Gauss-Lobatto guess, stored ascending
        double x = std::cos(M_PI * (N - i) / N);
        if (i == 0) x = -1.0;
        if (i == N) x = 1.0;
        if (i != 0 && i != N) {
            for (int it = 0; it < 200; ++it) {
                double pm, p;
                legendre_pair(N, x, pm, p);
                double dx = (x * p - pm) / (n1 * p);
                x -= dx;
                if (std::fabs(dx) <= 2e-16 * std::fabs(x) + 1e-300) break;
            }
        }
        xi[i] = x;
    }
    for (int i = 0; i <= N; ++i) {
        double pm, p;
        legendre_pair(N, xi[i], pm, p);
        w[i] = 2.0 / (N * (N + 1.0) * p * p);
    }
    double bw[kMaxN + 1];
    for (int j = 0; j <= N; ++j) {
        double prod = 1.0;
        for (int k = 0; k <= N; ++k)
            if (k != j) prod *= (xi[j] - xi[k]);
        bw[j] = 1.0 / prod;
    }
    for (int i = 0; i <= N; ++i) {
        double diag = 0.0;
        for (int j = 0; j <= N; ++j) {
            if (j == i) continue;
            double v = (bw[j] / bw[i]) / (xi[i] - xi[j]);
            D[i * n1 + j] = v;
            diag -= v;
        }
        D[i * n1 + i] = diag;
    }
}

}  // namespace hb
