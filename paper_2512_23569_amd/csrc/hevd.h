// Host half of learning the t-SVD basis pair from an image (Sec. III-B, Eq. 10-11): the
// per-slice covariances from the channel Gram sums, their Hermitian eigendecomposition and the
// inverse channel DFT back to real basis tensors.  Plain C++ (no HIP), so that it also builds
// with a host compiler.
#pragma once

#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstdint>
#include <vector>

namespace htsvd {

typedef std::complex<double> cplx;

// Eigendecomposition of the n x n Hermitian matrix A (row-major, n <= 8) by cyclic Jacobi
// rotations (Jacobi's method, as in Golub and Van Loan, Sec. 8.5, with a complex rotation: a
// diagonal phase first makes the pivot real, then a real plane rotation removes it).
// Outputs the eigenvalues in descending order and the matching unit eigenvectors as the columns
// of Q (row-major); each column's phase is fixed so that its entry of largest modulus (the first
// among equals) is real and positive.
inline void hermitian_evd(int n, const cplx *A_in, double *ev, cplx *Q) {
    cplx A[64], V[64];
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) {
            A[i * n + k] = 0.5 * (A_in[i * n + k] + std::conj(A_in[k * n + i]));
            V[i * n + k] = i == k ? 1.0 : 0.0;
        }
    for (int i = 0; i < n; ++i) A[i * n + i] = A[i * n + i].real();
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += std::abs(A[p * n + q]);
        if (off == 0.0) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double r = std::abs(A[p * n + q]);
                if (r == 0.0) continue;
                const double app = A[p * n + p].real(), aqq = A[q * n + q].real();
                // Past the first sweeps a pivot below the last bit of both diagonal entries is
                // dropped instead of rotated (the usual termination of the cyclic method).
                if (sweep > 3 && std::fabs(app) + 100.0 * r == std::fabs(app) &&
                    std::fabs(aqq) + 100.0 * r == std::fabs(aqq)) {
                    A[p * n + q] = A[q * n + p] = 0.0;
                    continue;
                }
                const cplx e = A[p * n + q] / r;  // unit phase of the pivot
                const double theta = (aqq - app) / (2.0 * r);
                double t = 1.0 / (std::fabs(theta) + std::sqrt(1.0 + theta * theta));
                if (theta < 0.0) t = -t;
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                const cplx ec = std::conj(e);
                // A <- A J with J = [[c, s], [-s conj(e), c conj(e)]] on the (p, q) plane ...
                for (int i = 0; i < n; ++i) {
                    const cplx xp = A[i * n + p], xq = A[i * n + q];
                    A[i * n + p] = c * xp - s * ec * xq;
                    A[i * n + q] = s * xp + c * ec * xq;
                    const cplx vp = V[i * n + p], vq = V[i * n + q];
                    V[i * n + p] = c * vp - s * ec * vq;
                    V[i * n + q] = s * vp + c * ec * vq;
                }
                // ... then A <- J^H A.
                for (int k = 0; k < n; ++k) {
                    const cplx xp = A[p * n + k], xq = A[q * n + k];
                    A[p * n + k] = c * xp - s * e * xq;
                    A[q * n + k] = s * xp + c * e * xq;
                }
                A[p * n + q] = A[q * n + p] = 0.0;
                A[p * n + p] = A[p * n + p].real();
                A[q * n + q] = A[q * n + q].real();
            }
    }
    int order[8];
    for (int j = 0; j < n; ++j) order[j] = j;
    std::stable_sort(order, order + n, [&](int x, int y) { return A[x * n + x].real() > A[y * n + y].real(); });
    for (int j = 0; j < n; ++j) {
        const int src = order[j];
        ev[j] = A[src * n + src].real();
        int kmax = 0;
        double amax = -1.0;
        for (int i = 0; i < n; ++i) {
            const double m = std::abs(V[i * n + src]);
            if (m > amax) {
                amax = m;
                kmax = i;
            }
        }
        const cplx ph = amax > 0.0 ? V[kmax * n + src] / amax : cplx(1.0, 0.0);
        for (int i = 0; i < n; ++i) Q[i * n + j] = V[i * n + src] * std::conj(ph);
        Q[kmax * n + j] = amax;
    }
}

// Basis pair (U, V) of one image from its channel Gram sums over all reference patches P:
//   gram[0][a][b][i][k] = sum_P sum_j P(i, j, a) P(k, j, b)   (rows of the patches)
//   gram[1][a][b][i][k] = sum_P sum_j P(j, i, a) P(j, k, b)   (columns of the patches)
// for channels a, b < c (any count: colour channels or hyperspectral bands), ps = 8.  Slice f of
// the channel DFT (Eq. 5, w = exp(-2 pi i / c)) has
// C_row^(f) = sum_P P_hat P_hat^H = sum_ab w^(f(a-b)) gram[0][a][b] and
// C_col^(f) = sum_P P_hat^H P_hat = sum_ab w^(f(b-a)) gram[1][a][b]; U_hat^(f) and V_hat^(f)
// hold their eigenvectors by descending eigenvalue.  Slice c-f is the conjugate of slice f, so
// the inverse DFT gives real tensors, written slice-major: U[(k*8 + i)*8 + j] = U(i, j, k).
inline void basis_from_gram(int c, const int64_t *gram, double *U, double *V, double *ev_row, double *ev_col) {
    const int n = 8;
    const double two_pi = 2.0 * M_PI;
    std::vector<std::array<cplx, 64>> Uh(c), Vh(c);
    for (int f = 0; f <= c / 2; ++f) {
        for (int g = 0; g < 2; ++g) {
            cplx C[64];
            for (int e = 0; e < 64; ++e) C[e] = 0.0;
            for (int a = 0; a < c; ++a)
                for (int b = 0; b < c; ++b) {
                    const int d = g == 0 ? a - b : b - a;
                    const int m = ((f * d) % c + c) % c;
                    const cplx tw = std::polar(1.0, -two_pi * m / c);
                    const int64_t *G = gram + ((size_t)(g * c + a) * c + b) * 64;
                    for (int e = 0; e < 64; ++e) C[e] += (double)G[e] * tw;
                }
            cplx Q[64];
            double ev[8];
            hermitian_evd(n, C, ev, Q);
            cplx *dst = g == 0 ? Uh[f].data() : Vh[f].data();
            for (int e = 0; e < 64; ++e) dst[e] = Q[e];
            double *evo = g == 0 ? ev_row : ev_col;
            if (evo)
                for (int j = 0; j < n; ++j) evo[f * n + j] = ev[j];
        }
    }
    for (int f = c / 2 + 1; f < c; ++f)
        for (int e = 0; e < 64; ++e) {
            Uh[f][e] = std::conj(Uh[c - f][e]);
            Vh[f][e] = std::conj(Vh[c - f][e]);
        }
    // Inverse DFT along the channel mode: T(k) = (1/c) sum_f T_hat^(f) exp(+2 pi i f k / c).
    for (int k = 0; k < c; ++k)
        for (int e = 0; e < 64; ++e) {
            cplx u = 0.0, v = 0.0;
            for (int f = 0; f < c; ++f) {
                const cplx tw = std::polar(1.0, two_pi * ((f * k) % c) / c);
                u += Uh[f][e] * tw;
                v += Vh[f][e] * tw;
            }
            U[k * 64 + e] = u.real() / c;
            V[k * 64 + e] = v.real() / c;
        }
}

}  // namespace htsvd
