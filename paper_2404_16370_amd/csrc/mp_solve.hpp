// mp_solve.hpp -- the damped 6x6 Gauss-Newton solve shared by the
// likelihood's per-particle step and the scan-to-scan odometry (Eq. 4).
#pragma once
#include <hip/hip_runtime.h>

// Damped Gauss-Newton step psi = -(H + diag(lam_rel H_ii + lam_abs))^-1 b,
// solved as a Cholesky factorisation of the diagonally scaled system.
template <class T>
__device__ inline bool chol_solve6(const T Hs[21], const T b[6], T lam_rel, T lam_abs, T psi[6], T& kappa) {
    T A[6][6];
    int q = 0;
    for (int r = 0; r < 6; ++r)
        for (int c = r; c < 6; ++c) {
            A[r][c] = Hs[q];
            A[c][r] = Hs[q];
            ++q;
        }
    T d[6];
    for (int r = 0; r < 6; ++r) {
        A[r][r] = A[r][r] + (lam_rel * A[r][r] + lam_abs);
        if (!(A[r][r] > T(0))) return false;
        d[r] = T(1) / sqrt(A[r][r]);
    }
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) A[r][c] = A[r][c] * d[r] * d[c];
    T L[6][6];
    T lmin = T(1e30), lmax = T(0);
    for (int j = 0; j < 6; ++j) {
        T s = A[j][j];
        for (int k = 0; k < j; ++k) s -= L[j][k] * L[j][k];
        if (!(s > T(0))) return false;
        const T ljj = sqrt(s);
        L[j][j] = ljj;
        lmin = ljj < lmin ? ljj : lmin;
        lmax = ljj > lmax ? ljj : lmax;
        for (int i = j + 1; i < 6; ++i) {
            T t = A[i][j];
            for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
            L[i][j] = t / ljj;
        }
    }
    kappa = (lmax / lmin) * (lmax / lmin);
    T y[6];
    for (int i = 0; i < 6; ++i) {
        T t = -b[i] * d[i];
        for (int k = 0; k < i; ++k) t -= L[i][k] * y[k];
        y[i] = t / L[i][i];
    }
    T x[6];
    for (int i = 5; i >= 0; --i) {
        T t = y[i];
        for (int k = i + 1; k < 6; ++k) t -= L[k][i] * x[k];
        x[i] = t / L[i][i];
    }
    for (int i = 0; i < 6; ++i) psi[i] = x[i] * d[i];
    return true;
}

