// Dynamic AMR kernels: the refinement indicator per element and the
// solution transfer to an adapted octree mesh (3D, perfect gas).
//
// Sec. Results (AMR Taylor-Green case: Loehner's weighted second-derivative
// estimate or the Hennemann-Gassner modal-energy coefficient of a derived
// variable) and Sec. New Developments (interpolation from large to small
// elements, exact L2 projection back).
#pragma once

#include "dgx_internal.h"
#include "physics.h"

namespace dgx {

// Applies the 1D matrix M (N1 x N1, row-major [out][in]) along direction d
// of the element values in LDS src, writing dst (one thread per node).
template <int N1>
__device__ __forceinline__ void amr_apply_dir(const double *M, const double *src, double *dst, int node, int d) {
    const int stride = d == 0 ? 1 : d == 1 ? N1 : N1 * N1;
    const int a = (node / stride) % N1;
    const int base = node - a * stride;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < N1; ++j) s = fma(M[a * N1 + j], src[base + j * stride], s);
    dst[node] = s;
}

// Indicator per element, one workgroup of (N+1)^3 threads per element.
// var: 0 rho, 1 p, 2 rho p, 3 |v|.  kind 0 (Loehner): the variable is
// sampled at N+1 equidistant points per direction (eq: [sample][node]) and
// the element takes the largest
//   |f+ - 2 f0 + f-| / (|f+ - f0| + |f0 - f-| + 0.2 (|f+| + 2|f0| + |f-|))
// over interior samples of all lines (0 where the denominator is 0).  kind
// 1 (Hennemann-Gassner): orthonormal Legendre modes of the variable, E =
// max((E_all - E_{<=N-1})/E_all, (E_{<=N-1} - E_{<=N-2})/E_{<=N-1}) and the
// coefficient 1/(1 + exp(-(s/T)(E - T))), T = 0.5 * 10^(-1.8 (N+1)^(1/4)),
// s = ln((1 - 1e-4)/1e-4), set to 0 below 1e-4.
template <int N>
__global__ void __launch_bounds__(128) k_amr_indicator(const double *__restrict__ u, int nelem, double gamma,
                                                        int kind, int var, const double *__restrict__ eq,
                                                        BasisC B, double *__restrict__ ind) {
    constexpr int N1 = N + 1, NN = N1 * N1 * N1;
    __shared__ double s0[NN], s1[NN], sm[N1 * N1];
    __shared__ double red[NN];
    const int e = blockIdx.x;
    const int node = threadIdx.x;
    if (node < N1 * N1) sm[node] = kind == 0 ? eq[node] : B.Vinv[node];
    if (node < NN) {
        const size_t stride = (size_t)nelem * NN, gi = (size_t)e * NN + node;
        const double rho = u[gi];
        double v[3], v2 = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            v[c] = u[(1 + c) * stride + gi] / rho;
            v2 = fma(v[c], v[c], v2);
        }
        const double p = (gamma - 1.0) * (u[4 * stride + gi] - 0.5 * rho * v2);
        s0[node] = var == 0 ? rho : var == 1 ? p : var == 2 ? rho * p : sqrt(v2);
    }
    __syncthreads();
    // the three 1D transforms: s0 -> s1 -> s0 -> s1
    if (node < NN) amr_apply_dir<N1>(sm, s0, s1, node, 0);
    __syncthreads();
    if (node < NN) amr_apply_dir<N1>(sm, s1, s0, node, 1);
    __syncthreads();
    if (node < NN) amr_apply_dir<N1>(sm, s0, s1, node, 2);
    __syncthreads();
    if (node < NN) {
        double r = 0.0;
        if (kind == 0) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int stride = d == 0 ? 1 : d == 1 ? N1 : N1 * N1;
                const int a = (node / stride) % N1;
                if (a == 0 || a == N) continue;
                const double fm = s1[node - stride], f0 = s1[node], fp = s1[node + stride];
                const double num = fabs(fp - 2.0 * f0 + fm);
                const double den = fabs(fp - f0) + fabs(f0 - fm) + 0.2 * (fabs(fp) + 2.0 * fabs(f0) + fabs(fm));
                if (den > 0.0) r = fmax(r, num / den);
            }
        }
        red[node] = r;
    }
    __syncthreads();
    if (node == 0) {
        if (kind == 0) {
            double r = 0.0;
            for (int n = 0; n < NN; ++n) r = fmax(r, red[n]);
            ind[e] = r;
        } else {
            // mode energies by the largest mode index of each coefficient
            double ea = 0.0, e1 = 0.0, e2 = 0.0;
            for (int n = 0; n < NN; ++n) {
                const int a = n % N1, b = (n / N1) % N1, c = n / (N1 * N1);
                const int mx = max(a, max(b, c));
                const double m2 = s1[n] * s1[n];
                ea += m2;
                if (mx <= N - 1) e1 += m2;
                if (mx <= N - 2) e2 += m2;
            }
            const double E = fmax((ea - e1) / ea, (e1 - e2) / e1);
            const double T = 0.5 * pow(10.0, -1.8 * pow((double)(N + 1), 0.25));
            const double s = log((1.0 - 1e-4) / 1e-4);
            const double a = 1.0 / (1.0 + exp(-(s / T) * (E - T)));
            ind[e] = a < 1e-4 ? 0.0 : a;
        }
    }
}

// Transfer to the adapted mesh: one thread per (new element, node).  Row
// tab[e] (kOctTab ints): kind 0 copies the old element, kind 1 interpolates
// the old element along the split path (per direction the composite of the
// half-interval interpolations I_0 / I_1), kind 2 sums the L2 projections
// (P_0 / P_1 per direction) of the 8 old children.  ops: [I_0, I_1, P_0, P_1]
// as 25-wide [out][in] blocks.
template <int N>
__global__ void __launch_bounds__(256) k_amr_transfer(const double *__restrict__ uold, int nold,
                                                       double *__restrict__ unew, int nnew, int nvar,
                                                       const int *__restrict__ tab, const double *__restrict__ ops) {
    constexpr int N1 = N + 1, NN = N1 * N1 * N1, TB = 12;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nnew * NN) return;
    const int e = t / NN, node = t - e * NN;
    const int a = node % N1, b = (node / N1) % N1, c = node / (N1 * N1);
    const int *row = tab + (size_t)e * TB;
    const size_t so = (size_t)nold * NN, sn = (size_t)nnew * NN;
    if (row[0] == 0) {
        const size_t g = (size_t)row[3] * NN + node;
        for (int v = 0; v < nvar; ++v) unew[v * sn + t] = uold[v * so + g];
        return;
    }
    if (row[0] == 1) {
        // composite 1D rows of this node: M_d[out = node index][in]
        double Mx[N1], My[N1], Mz[N1];
        const int depth = row[1], code = row[2];
        const int pos[3] = {a, b, c};
        double *M[3] = {Mx, My, Mz};
        for (int d = 0; d < 3; ++d) {
            // row pos[d] of I_{path[depth-1]} ... I_{path[0]} (first split applied first)
            double r[N1];
            for (int j = 0; j < N1; ++j) r[j] = j == pos[d] ? 1.0 : 0.0;
            for (int q = depth - 1; q >= 0; --q) {
                const int ch = (code >> (3 * q)) & 7;
                const double *I = ops + ((ch >> d) & 1) * 25;
                double nr[N1];
                for (int j = 0; j < N1; ++j) {
                    double s = 0.0;
                    for (int m = 0; m < N1; ++m) s = fma(r[m], I[m * N1 + j], s);
                    nr[j] = s;
                }
                for (int j = 0; j < N1; ++j) r[j] = nr[j];
            }
            for (int j = 0; j < N1; ++j) M[d][j] = r[j];
        }
        const size_t g0 = (size_t)row[3] * NN;
        for (int v = 0; v < nvar; ++v) {
            double s = 0.0;
            for (int k = 0; k < N1; ++k)
                for (int j = 0; j < N1; ++j) {
                    const double w = Mz[k] * My[j];
                    for (int i = 0; i < N1; ++i) s = fma(w * Mx[i], uold[v * so + g0 + i + N1 * (j + N1 * k)], s);
                }
            unew[v * sn + t] = s;
        }
        return;
    }
    for (int v = 0; v < nvar; ++v) {
        double s = 0.0;
        for (int ch = 0; ch < 8; ++ch) {
            const double *Px = ops + 50 + (ch & 1) * 25 + a * N1;
            const double *Py = ops + 50 + ((ch >> 1) & 1) * 25 + b * N1;
            const double *Pz = ops + 50 + ((ch >> 2) & 1) * 25 + c * N1;
            const size_t g0 = (size_t)row[3 + ch] * NN;
            for (int k = 0; k < N1; ++k)
                for (int j = 0; j < N1; ++j) {
                    const double w = Pz[k] * Py[j];
                    for (int i = 0; i < N1; ++i) s = fma(w * Px[i], uold[v * so + g0 + i + N1 * (j + N1 * k)], s);
                }
        }
        unew[v * sn + t] = s;
    }
}

}  // namespace dgx
