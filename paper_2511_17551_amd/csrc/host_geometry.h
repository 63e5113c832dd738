// Host-side reference-element operators and element geometry of libdgx.
//
// LGL points (Sec. Methodology, Eqs. lag, divergenc_quadrature): the roots
// of P_{N+1} - P_{N-1} (proportional to (1 - x^2) P_N'), found by Newton's
// method; weights 2 / (N (N+1) P_N(x)^2).  Derivative matrix by barycentric
// weights.  Modal transform: V^-1 = diag(1/gamma) V^T W with the discrete
// norms gamma_j of the orthonormal Legendre polynomials (exact inverse on LGL
// points).  Metric terms (Eqs. mapped_equation, jacobian): 2D cross form,
// 3D conservative curl form, evaluated on element-local coordinates (x minus
// the element's first node; the discrete curl form is translation invariant).
#pragma once

#include <cmath>
#include <vector>

namespace dgx {

struct HostBasis {
    int N = 0, N1 = 0;
    std::vector<double> x, w, D, Vinv;  // D row-major [a][b]
};

inline void legendre_pd(int n, double x, double &p, double &dp) {
    if (n == 0) {
        p = 1.0;
        dp = 0.0;
        return;
    }
    double pm = 1.0, pc = x, dm = 0.0, dc = 1.0;
    for (int k = 2; k <= n; ++k) {
        const double pn = ((2.0 * k - 1.0) * x * pc - (k - 1.0) * pm) / k;
        const double dn = dm + (2.0 * k - 1.0) * pc;
        pm = pc;
        pc = pn;
        dm = dc;
        dc = dn;
    }
    p = pc;
    dp = dc;
}

inline HostBasis make_basis(int N) {
    HostBasis B;
    B.N = N;
    B.N1 = N + 1;
    const int n1 = N + 1;
    B.x.assign(n1, 0.0);
    B.w.assign(n1, 0.0);
    B.x[0] = -1.0;
    B.x[N] = 1.0;
    for (int j = 1; j < N; ++j) {
        double x = -std::cos(M_PI * j / N);
        for (int it = 0; it < 100; ++it) {
            double pa, da, pb, db;
            legendre_pd(N + 1, x, pa, da);
            legendre_pd(N - 1, x, pb, db);
            const double q = pa - pb, dq = da - db;
            const double dx = q / dq;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        B.x[j] = x;
    }
    for (int j = 0; j < n1; ++j) {
        double p, dp;
        legendre_pd(N, B.x[j], p, dp);
        B.w[j] = 2.0 / (N * (N + 1.0) * p * p);
    }
    std::vector<double> lam(n1, 1.0);
    for (int j = 0; j < n1; ++j)
        for (int k = 0; k < n1; ++k)
            if (k != j) lam[j] /= (B.x[j] - B.x[k]);
    B.D.assign(n1 * n1, 0.0);
    for (int a = 0; a < n1; ++a) {
        double s = 0.0;
        for (int b = 0; b < n1; ++b) {
            if (a == b) continue;
            const double v = lam[b] / lam[a] / (B.x[a] - B.x[b]);
            B.D[a * n1 + b] = v;
            s += v;
        }
        B.D[a * n1 + a] = -s;
    }
    // modal transform
    std::vector<double> V(n1 * n1);
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n1; ++j) {
            double p, dp;
            legendre_pd(j, B.x[i], p, dp);
            V[i * n1 + j] = std::sqrt((2.0 * j + 1.0) / 2.0) * p;
        }
    B.Vinv.assign(n1 * n1, 0.0);
    for (int j = 0; j < n1; ++j) {
        double g = 0.0;
        for (int i = 0; i < n1; ++i) g += B.w[i] * V[i * n1 + j] * V[i * n1 + j];
        for (int i = 0; i < n1; ++i) B.Vinv[j * n1 + i] = B.w[i] * V[i * n1 + j] / g;
    }
    return B;
}

// Nodal derivative of f (one element, nn values) along reference direction d.
inline void ref_derivative(const HostBasis &B, int dim, int d, const double *f, double *out) {
    const int n1 = B.N1;
    const int nn = dim == 2 ? n1 * n1 : n1 * n1 * n1;
    const int st = d == 0 ? 1 : (d == 1 ? n1 : n1 * n1);
    for (int n = 0; n < nn; ++n) {
        const int a = (n / st) % n1;
        const int base = n - a * st;
        double s = 0.0;
        for (int j = 0; j < n1; ++j) s += B.D[a * n1 + j] * f[base + j * st];
        out[n] = s;
    }
}

// Working storage of element_metrics (one per host thread).
struct MetricScratch {
    std::vector<double> xl, dx, V, t1, t2;
};

// Metric terms Ja[i][c] (i: reference direction, c: Cartesian component) and
// J at the nodes of one element.  x: [dim][nn] of that element.
inline void element_metrics(const HostBasis &B, int dim, const double *const *xe, double *Ja /*[dim*dim][nn]*/,
                            double *J /*[nn]*/, MetricScratch &ws) {
    const int n1 = B.N1;
    const int nn = dim == 2 ? n1 * n1 : n1 * n1 * n1;
    std::vector<double> &xl = ws.xl, &dx = ws.dx;
    xl.resize(dim * nn);
    for (int c = 0; c < dim; ++c)
        for (int n = 0; n < nn; ++n) xl[c * nn + n] = xe[c][n] - xe[c][0];
    dx.resize(dim * dim * nn);  // dx[(c*dim+d)*nn+n] = d x_c / d X_d
    for (int c = 0; c < dim; ++c)
        for (int d = 0; d < dim; ++d) ref_derivative(B, dim, d, &xl[c * nn], &dx[(c * dim + d) * nn]);
    auto DX = [&](int c, int d, int n) { return dx[(c * dim + d) * nn + n]; };
    if (dim == 2) {
        for (int n = 0; n < nn; ++n) {
            Ja[0 * nn + n] = DX(1, 1, n);
            Ja[1 * nn + n] = -DX(0, 1, n);
            Ja[2 * nn + n] = -DX(1, 0, n);
            Ja[3 * nn + n] = DX(0, 0, n);
            J[n] = DX(0, 0, n) * DX(1, 1, n) - DX(0, 1, n) * DX(1, 0, n);
        }
        return;
    }
    std::vector<double> &V = ws.V, &t1 = ws.t1, &t2 = ws.t2;
    V.resize(3 * nn);
    t1.resize(nn);
    t2.resize(nn);
    for (int comp = 0; comp < 3; ++comp) {
        const int m = (comp + 1) % 3, l = (comp + 2) % 3;
        // V_d = x_l * d x_m / d X_d
        for (int d = 0; d < 3; ++d)
            for (int n = 0; n < nn; ++n) V[d * nn + n] = xl[l * nn + n] * DX(m, d, n);
        // Ja^i_comp = -(curl V)_i
        const int cyc[3][2] = {{1, 2}, {2, 0}, {0, 1}};
        for (int i = 0; i < 3; ++i) {
            const int p = cyc[i][0], q = cyc[i][1];
            ref_derivative(B, 3, p, &V[q * nn], t1.data());  // d_p V_q
            ref_derivative(B, 3, q, &V[p * nn], t2.data());  // d_q V_p
            for (int n = 0; n < nn; ++n) Ja[(i * 3 + comp) * nn + n] = -(t1[n] - t2[n]);
        }
    }
    for (int n = 0; n < nn; ++n) {
        J[n] = DX(0, 0, n) * (DX(1, 1, n) * DX(2, 2, n) - DX(1, 2, n) * DX(2, 1, n)) -
               DX(0, 1, n) * (DX(1, 0, n) * DX(2, 2, n) - DX(1, 2, n) * DX(2, 0, n)) +
               DX(0, 2, n) * (DX(1, 0, n) * DX(2, 1, n) - DX(1, 1, n) * DX(2, 0, n));
    }
}

// Value of the Lagrange basis polynomial j on the LGL nodes at point y.
inline double lagrange(const HostBasis &B, int j, double y) {
    double v = 1.0;
    for (int k = 0; k < B.N1; ++k)
        if (k != j) v *= (y - B.x[k]) / (B.x[j] - B.x[k]);
    return v;
}

// Mortar operators: interpolation of a face edge to its lower/upper half,
// I_s[i][j] = l_j((x_i -+ 1)/2), and the exact L2 projection back,
// P_s = 1/2 M^-1 I_s^T M with the exact mass matrix M_ij = int l_i l_j
// (Gauss-Legendre quadrature with N+1 points).
inline void mortar_operators(const HostBasis &B, double Im[2][25], double Pm[2][25]) {
    const int n1 = B.N1;
    // Gauss-Legendre points: roots of P_{n1} by Newton
    std::vector<double> xg(n1), wg(n1);
    for (int i = 0; i < n1; ++i) {
        double x = -std::cos(M_PI * (i + 0.75) / (n1 + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p, dp;
            legendre_pd(n1, x, p, dp);
            const double dx = p / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        double p, dp;
        legendre_pd(n1, x, p, dp);
        xg[i] = x;
        wg[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    std::vector<double> M(n1 * n1, 0.0);
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n1; ++j)
            for (int q = 0; q < n1; ++q) M[i * n1 + j] += wg[q] * lagrange(B, i, xg[q]) * lagrange(B, j, xg[q]);
    // inverse by Gauss-Jordan elimination with partial pivoting
    std::vector<double> A(M), Inv(n1 * n1, 0.0);
    for (int i = 0; i < n1; ++i) Inv[i * n1 + i] = 1.0;
    for (int c = 0; c < n1; ++c) {
        int piv = c;
        for (int r = c + 1; r < n1; ++r)
            if (std::fabs(A[r * n1 + c]) > std::fabs(A[piv * n1 + c])) piv = r;
        for (int k = 0; k < n1; ++k) {
            std::swap(A[c * n1 + k], A[piv * n1 + k]);
            std::swap(Inv[c * n1 + k], Inv[piv * n1 + k]);
        }
        const double d = A[c * n1 + c];
        for (int k = 0; k < n1; ++k) {
            A[c * n1 + k] /= d;
            Inv[c * n1 + k] /= d;
        }
        for (int r = 0; r < n1; ++r) {
            if (r == c) continue;
            const double f = A[r * n1 + c];
            for (int k = 0; k < n1; ++k) {
                A[r * n1 + k] -= f * A[c * n1 + k];
                Inv[r * n1 + k] -= f * Inv[c * n1 + k];
            }
        }
    }
    for (int s = 0; s < 2; ++s) {
        const double sh = s == 0 ? -1.0 : 1.0;
        std::vector<double> I(n1 * n1), T(n1 * n1, 0.0);
        for (int i = 0; i < n1; ++i)
            for (int j = 0; j < n1; ++j) I[i * n1 + j] = lagrange(B, j, 0.5 * (B.x[i] + sh));
        // T = I^T M
        for (int i = 0; i < n1; ++i)
            for (int j = 0; j < n1; ++j)
                for (int k = 0; k < n1; ++k) T[i * n1 + j] += I[k * n1 + i] * M[k * n1 + j];
        for (int i = 0; i < n1; ++i)
            for (int j = 0; j < n1; ++j) {
                double v = 0.0;
                for (int k = 0; k < n1; ++k) v += Inv[i * n1 + k] * T[k * n1 + j];
                Pm[s][i * n1 + j] = 0.5 * v;
                Im[s][i * n1 + j] = I[i * n1 + j];
            }
    }
}

}  // namespace dgx
