// linalg6.hpp -- register-resident 6x6 symmetric linear algebra in FP64.
//
// Symmetric matrices are stored packed, lower triangle row by row: entry
// (i, j), j <= i, at i (i + 1) / 2 + j (21 doubles). Everything is fully
// unrolled so that the packed arrays live in VGPRs.
#pragma once

#include "ad.hpp"

#pragma clang fp reassociate(on)

namespace automat {
namespace la {

AD_FN constexpr int pk(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

// In-place Cholesky factorization M = L L^T of a packed SPD matrix. On
// return the packed array holds the strictly lower part of L and, on the
// diagonal, the inverse pivots 1 / L_jj (the solves below multiply by them;
// L_jj itself is never needed). Returns false if a pivot is not positive
// (matrix not positive definite or not finite).
AD_FN bool cholesky6(double *L) {
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double d = L[pk(j, j)];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= L[pk(j, k)] * L[pk(j, k)];
        ok = ok && (d > 0.0);
        const double inv = fm::rsqrt(d);
        L[pk(j, j)] = inv;
#pragma unroll
        for (int i = j + 1; i < 6; ++i) {
            double s = L[pk(i, j)];
#pragma unroll
            for (int k = 0; k < j; ++k) s -= L[pk(i, k)] * L[pk(j, k)];
            L[pk(i, j)] = s * inv;
        }
    }
    return ok;
}

// Solve L z = b in place (L as returned by cholesky6).
AD_FN void forward6(const double *L, double *b) {
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double s = b[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= L[pk(i, k)] * b[k];
        b[i] = s * L[pk(i, i)];
    }
}

// Solve L^T y = z in place (L as returned by cholesky6).
AD_FN void backward6(const double *L, double *b) {
#pragma unroll
    for (int i = 5; i >= 0; --i) {
        double s = b[i];
#pragma unroll
        for (int k = i + 1; k < 6; ++k) s -= L[pk(k, i)] * b[k];
        b[i] = s * L[pk(i, i)];
    }
}

// Solve (L L^T) x = b in place (L as returned by cholesky6).
AD_FN void chol_solve6(const double *L, double *b) {
    forward6(L, b);
    backward6(L, b);
}

// y = S x for packed symmetric S.
AD_FN void symv6(const double *S, const double *x, double *y) {
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < 6; ++j) s += S[pk(i, j)] * x[j];
        y[i] = s;
    }
}

AD_FN double dot6(const double *x, const double *y) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) s += x[i] * y[i];
    return s;
}

AD_FN double norm_inf6(const double *x) {
    double m = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) m = ::fmax(m, ::fabs(x[i]));
    return m;
}

}  // namespace la
}  // namespace automat

#pragma clang fp reassociate(off)
